"""GPU parity of the laboratory-frame stations against the oracle's stations.

Stations are placed so that, during the run, one leaves the box at z' = 0,
one stays inside throughout, one starts near the top and one enters from
above: sample counts and lab times must equal the oracle's exactly (same
FP64 expressions, unfused) and the recorded lab fields match to rounding on
the FP64 path, to FP32 field rounding on the split-precision path.  Graph
replay, the timed eager path and batched runs record the same samples."""
import numpy as np
import pytest

import oracle
from paper_0909_5603_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_0909_5603_amd import pic  # noqa: E402


def _with_stations(cfg, z_first, z_step, n=4, stride=1, cap=64):
    """Stations whose boosted positions at t' = 0 are z_first + q z_step (in
    units of the box length)."""
    st = oracle.State(dict(cfg, ppc=0))
    g = st.derived["gamma_b"]
    st.close()
    Lz = cfg["nz"] * cfg["dz"]
    return dict(cfg, n_stations=n, station_z0=g * z_first * Lz, station_dz=g * z_step * Lz,
                station_stride=stride, station_cap=cap)


CASES = {
    # 2D open z, laser and drifting plasma: 40 steps move a station ~0.2 Lz
    "c1_open": lambda: _with_stations(workloads.config("c1"), 0.08, 0.33, stride=2),
    # 3D periodic z, stations on every other transverse node
    "3d_periodic": lambda: _with_stations(
        workloads.config("c5", nz=32, nx=16, ny=16, ppc=2, gamma_boost=13.0, waist=0.3,
                         bc_z="periodic"), 0.15, 0.3, stride=2),
    # 3D open z with the current filter on
    "3d_open_filter": lambda: _with_stations(
        workloads.config("c5", nz=48, nx=16, ny=16, ppc=2, gamma_boost=13.0, waist=0.3,
                         filter_passes=1, filter_compensate=1), 0.1, 0.31, stride=4),
}
STEPS = {"c1_open": 40, "3d_periodic": 24, "3d_open_filter": 24}


def _compare(run, st, n_stations, tol):
    worst = 0.0
    seen = 0
    for q in range(n_stations):
        tg, dg, ng = run.station(q)
        to, do, no = st.station(q)
        assert ng == no, f"station {q}: {ng} samples, oracle {no}"
        assert tg.shape == to.shape and dg.shape == do.shape
        np.testing.assert_allclose(tg, to, rtol=1e-15, atol=0)
        if no:
            scale = max(np.abs(do).max(), 1e-300)
            worst = max(worst, np.abs(dg - do).max() / scale)
            seen += no
    assert seen > 0
    assert worst < tol, worst
    return worst


@pytest.mark.parametrize("case", list(CASES))
def test_stations_fp64_match_oracle(case):
    cfg = CASES[case]()
    run = pic.Run(cfg, "fp64")
    st = oracle.State(cfg)
    run.step(STEPS[case])
    st.step(STEPS[case])
    counts = [st.station(q)[2] for q in range(cfg["n_stations"])]
    print(f"\n{case}: samples per station {counts}")
    # the placement exercises leaving, staying, and entering
    assert 0 < min(counts) < STEPS[case] and max(counts) == STEPS[case]
    w = _compare(run, st, cfg["n_stations"], 1e-10)
    print(f"{case}: max |lab field - oracle| / max |oracle| = {w:.3e}")
    run.close()
    st.close()


def test_stations_fp32_within_rounding_of_oracle():
    """FP32 fields carry a relative rounding of 2^-24 per value, compounded
    over 40 leapfrog steps and the lab transform (factor <= 2 gamma_b in the
    boosted-frame values, already part of the lab scale): 1e-5 of the largest
    lab field bounds it with margin."""
    cfg = CASES["c1_open"]()
    run = pic.Run(cfg, "fp32")
    st = oracle.State(cfg, round_f32=True)
    run.step(40)
    st.step(40)
    w = _compare(run, st, cfg["n_stations"], 1e-5)
    print(f"\nfp32 c1: max |lab field - oracle| / max |oracle| = {w:.3e}")
    run.close()
    st.close()


def test_capacity_keeps_the_first_samples_and_counts_the_rest():
    cfg = dict(CASES["c1_open"](), station_cap=5)
    run = pic.Run(cfg, "fp64")
    st = oracle.State(cfg)
    run.step(30)
    st.step(30)
    for q in range(cfg["n_stations"]):
        tg, dg, ng = run.station(q)
        to, do, no = st.station(q)
        assert ng == no and tg.size == min(no, 5)
        np.testing.assert_allclose(dg, do, rtol=0, atol=1e-10 * max(np.abs(do).max(), 1.0))
    # fewer samples requested than stored
    t2, d2, n2 = run.station(1, max_samples=2)
    assert t2.size == min(2, n2) and n2 == st.station(1)[2]
    run.close()
    st.close()


def test_graph_eager_and_timed_paths_record_the_same():
    cfg = CASES["c1_open"]()
    a = pic.Run(cfg, "fp64")
    b = pic.Run(cfg, "fp64", graph=False)
    c = pic.Run(cfg, "fp64")
    a.step(25)
    b.step(25)
    pic.pic_step_timed(c.handle, 25)
    for q in range(cfg["n_stations"]):
        ra, rb, rc = a.station(q), b.station(q), c.station(q)
        for r in (rb, rc):
            assert r[2] == ra[2]
            np.testing.assert_array_equal(r[0], ra[0])
            np.testing.assert_array_equal(r[1], ra[1])
    for r in (a, b, c):
        r.close()


def test_batch_with_and_without_stations_equals_alone():
    base = workloads.config("c1")
    cfgs = [_with_stations(dict(base, seed=1), 0.08, 0.33, stride=2),
            dict(base, seed=2),
            _with_stations(dict(base, seed=3), 0.5, 0.2, n=3, stride=4, cap=10)]
    steps = [(18, 7, 18), (5, 0, 0)]
    alone = []
    for i, cfg in enumerate(cfgs):
        r = pic.Run(cfg, "fp64")
        r.step(sum(s[i] for s in steps))
        alone.append([r.station(q) for q in range(cfg.get("n_stations", 0))])
        r.close()
    shared = torch.cuda.Stream()  # batched runs share one stream
    runs = [pic.Run(cfg, "fp64", stream=shared) for cfg in cfgs]
    for s in steps:
        idx = [i for i in range(3) if s[i] > 0]
        pic.pic_step_batch([runs[i].handle for i in idx], [s[i] for i in idx])
    shared.synchronize()
    for r, recs in zip(runs, alone):
        for q, (t, d, n) in enumerate(recs):
            tg, dg, ng = r.station(q)
            assert ng == n
            np.testing.assert_array_equal(tg, t)
            np.testing.assert_array_equal(dg, d)
        r.close()


def test_read_station_rejects_bad_indices():
    cfg = CASES["c1_open"]()
    run = pic.Run(cfg, "fp32")
    with pytest.raises(pic.PicError):
        run.station(cfg["n_stations"])
    with pytest.raises(pic.PicError):
        run.station(-1)
    run.close()
    plain = pic.Run(workloads.config("c1"), "fp32")
    with pytest.raises(pic.PicError):
        pic.pic_read_station(plain.handle, plain.params, 0)
    plain.close()
