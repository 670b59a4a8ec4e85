"""Serving on the GPU: a Poisson stream of 2D boosted-frame runs is served
with continuous batching; every run's result equals the same run served
alone: every electron's momentum (matched by id) within the stated FP32
bound of 1e-5 relative (FP64: 1e-12), and the field energies and wake
amplitude (FP64 1e-9, FP32 1e-3)."""
import numpy as np
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


@pytest.mark.parametrize("precision,tol,utol", [("fp64", 1e-9, 1e-12), ("fp32", 1e-3, 1e-5)])
def test_results_equal_alone_and_in_the_mix(precision, tol, utol):
    stream = _stream(12)
    stats = serve.serve_stream(stream, budget_bytes=1 << 30, chunk_steps=10, precision=precision,
                               keep_results=True)
    assert stats["n_requests"] == 12 and not stats["status"]
    assert stats["max_concurrency"] > 1
    worst = 0.0
    for rid, (t, cfg) in enumerate(stream):
        run = pic.Run(cfg, precision)
        run.step(cfg["steps"])
        alone = run.diag(pic.PIC_DIAG_FIELDS | pic.PIC_DIAG_PARTICLES)
        pa = run.particles()
        run.close()
        mixed = stats["results"][rid]
        assert mixed["step"] == cfg["steps"]
        assert mixed["n_particles"] == alone["n_particles"]
        for k in ("U_E", "U_B", "Ez_max", "KE"):
            a, b = alone[k], mixed[k]
            assert abs(a - b) <= tol * max(abs(a), 1e-12), (rid, k, a, b)
        pm = mixed["particles"]
        oa, om = np.argsort(pa["id"]), np.argsort(pm["id"])
        assert np.array_equal(pa["id"][oa], pm["id"][om])
        ua = np.stack([pa[k][oa] for k in ("ux", "uy", "uz")], 1)
        um = np.stack([pm[k][om] for k in ("ux", "uy", "uz")], 1)
        err = np.linalg.norm(ua - um, axis=1) / np.maximum(np.linalg.norm(ua, axis=1), 1e-3)
        worst = max(worst, float(err.max()) if err.size else 0.0)
        assert err.size == 0 or err.max() <= utol, (rid, float(err.max()))
    print(f"\n{precision}: max per-electron momentum difference alone vs in the mix {worst:.2e}")


def test_latency_stats_reported():
    stats = serve.serve_stream(_stream(16), budget_bytes=1 << 30, chunk_steps=10)
    assert stats["n_requests"] == 16 and stats["n_failed"] == 0 and stats["n_rejected"] == 0
    assert 0 < stats["p50_ms"] <= stats["p99_ms"]
    assert stats["throughput"] > 0


def test_request_over_the_budget_is_rejected_alone():
    """One request larger than the whole memory budget is rejected; the
    others are served."""
    stream = _stream(8)
    big = dict(stream[3][1], nz=1024, nx=512, ppc=16)
    stream[3] = (stream[3][0], big)
    stats = serve.serve_stream(stream, budget_bytes=256 << 20, chunk_steps=10)
    assert stats["status"] == {3: "rejected"}
    assert stats["n_requests"] == 7 and stats["n_rejected"] == 1
