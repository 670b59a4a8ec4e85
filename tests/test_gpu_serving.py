"""Serving on the GPU: a Poisson stream of 2D boosted-frame runs is served
with continuous batching; every run's result equals the same run served
alone (FP64: to rounding; split FP32: within the stated 1e-3 field-energy
and wake tolerance)."""
import pytest

from paper_0909_5603_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_0909_5603_amd import pic, serve  # noqa: E402


def _stream(n):
    # small grids and step counts so the test stays short
    return workloads.serving_stream(n, seed=7, rate_per_s=200.0, z_range=(32, 128),
                                    x_range=(16, 64), steps_range=(20, 80))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-9), ("fp32", 1e-3)])
def test_results_equal_alone_and_in_the_mix(precision, tol):
    stream = _stream(12)
    stats = serve.serve_stream(stream, budget_bytes=1 << 30, chunk_steps=10, precision=precision,
                               keep_results=True)
    assert stats["n_requests"] == 12
    assert stats["max_concurrency"] > 1
    for rid, (t, cfg) in enumerate(stream):
        run = pic.Run(cfg, precision)
        run.step(cfg["steps"])
        alone = run.diag(pic.PIC_DIAG_FIELDS | pic.PIC_DIAG_PARTICLES)
        run.close()
        mixed = stats["results"][rid]
        assert mixed["step"] == cfg["steps"]
        assert mixed["n_particles"] == alone["n_particles"]
        for k in ("U_E", "U_B", "Ez_max", "KE"):
            a, b = alone[k], mixed[k]
            assert abs(a - b) <= tol * max(abs(a), 1e-12), (rid, k, a, b)


def test_latency_stats_reported():
    stats = serve.serve_stream(_stream(16), budget_bytes=1 << 30, chunk_steps=10)
    assert stats["n_requests"] == 16
    assert 0 < stats["p50_ms"] <= stats["p99_ms"]
    assert stats["throughput"] > 0
