"""GPU parity of the laser antenna against the oracle's antenna, and the
lab -> boosted -> lab round trip.

* FP64 runs with the antenna (2D with plasma; 3D open z) match the oracle to
  rounding in fields, momenta and positions; the split-precision path keeps
  the FP32 bounds.
* In vacuum the emitted boosted field is the boosted lab pulse to the Yee
  scheme's error, with no backward emission.
* A lab-frame station downstream of the antenna records the laboratory
  pulse: the laser given in the lab, emitted by the drifting plane, evolved
  in the boosted frame and transformed back at a lab-fixed plane.
* Graph replay, eager and timed paths, and batches with and without an
  antenna give the same state."""
import numpy as np
import pytest

import oracle
from paper_0909_5603_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_0909_5603_amd import pic  # noqa: E402


def _antenna(cfg, z_frac, delay, box_frac=12.0):
    """Antenna at z_frac of the box at t' = 0, pulse of boosted length
    box/box_frac, envelope peak reaching the plane `delay` lab e-folds
    after t' = 0."""
    st = oracle.State(dict(cfg, ppc=0))
    d = st.derived
    st.close()
    Lz = cfg["nz"] * cfg["dz"]
    Ll = Lz / box_frac / d["dplus"]
    Za = d["gamma_b"] * z_frac * Lz
    return dict(cfg, laser_antenna=1, antenna_z_lab=Za, antenna_t_peak=d["beta_b"] * Za + delay * Ll,
                tau_lab=Ll)


def _match(a, b):
    oa, ob = np.argsort(a["id"]), np.argsort(b["id"])
    ids, ia, ib = np.intersect1d(a["id"][oa], b["id"][ob], assume_unique=True, return_indices=True)
    return ({k: v[oa][ia] for k, v in a.items()}, {k: v[ob][ib] for k, v in b.items()}, ids.size)


def _urel(g, o):
    ug = np.stack([g["ux"], g["uy"], g["uz"]], 1)
    uo = np.stack([o["ux"], o["uy"], o["uz"]], 1)
    return np.linalg.norm(ug - uo, axis=1) / np.linalg.norm(uo, axis=1)


def _frel(run, st):
    diff, scale = 0.0, 1e-300
    for c in range(6):
        g, o = run.field(c), st.field(c)
        scale = max(scale, np.abs(o).max())
        diff = max(diff, np.abs(g - o).max())
    return diff / scale


CASES = {
    # 2D, plasma streaming through the plane while it emits
    "c1_plasma": lambda: _antenna(workloads.config("c1", ppc=2), 0.6, 1.0),
    # 3D open z, x polarisation, pulse already crossing the plane at t' = 0
    "3d_open": lambda: _antenna(workloads.config(
        "c5", nz=64, nx=16, ny=16, ppc=1, gamma_boost=13.0, waist=0.4), 0.5, 0.0),
}


@pytest.mark.parametrize("case", list(CASES))
def test_antenna_fp64_matches_oracle(case):
    cfg = CASES[case]()
    run = pic.Run(cfg, "fp64")
    st = oracle.State(cfg)
    nsteps = 30
    run.step(nsteps)
    st.step(nsteps)
    fr = _frel(run, st)
    g, o, m = _match(run.particles(), st.particles())
    print(f"\n{case}: field rel {fr:.3e}, {m} particles")
    assert fr < 1e-10
    assert m > 0.99 * st.particles()["id"].size
    if m:
        assert _urel(g, o).max() < 1e-10
        for k in ("z", "x", "y"):
            assert np.abs(g[k] - o[k]).max() < 1e-10
    d, do = run.diag(), st.diag()
    for k in ("U_E", "U_B", "Ez_max"):
        assert d[k] == pytest.approx(do[k], rel=1e-9), k
    assert d["U_E"] > 0
    run.close()
    st.close()


def test_antenna_fp32_within_bounds():
    cfg = CASES["c1_plasma"]()
    run = pic.Run(cfg, "fp32", continuity=True)
    st = oracle.State(cfg, round_f32=True)
    worst = 0.0
    for _ in range(20):
        run.step(1)
        st.step(1)
        g, o, m = _match(run.particles(), st.particles())
        worst = max(worst, _urel(g, o).max())
        assert run.diag(pic.PIC_DIAG_FIELDS)["cont_resid"] <= 1e-6
    fr = _frel(run, st)
    print(f"\nfp32 antenna: momentum {worst:.3e}, fields {fr:.3e}")
    assert worst <= 1e-5
    assert fr < 1e-5
    run.close()
    st.close()


def _vacuum(nz=512, lam=2.0):
    dz = 12.8 / nz
    base = workloads.config("c1", nz=nz, nx=16, dz=dz, dx=dz, ppc=0, lambda0_um=lam)
    return _antenna(base, 0.55, 3.0)


def test_emitted_wave_is_the_boosted_pulse():
    cfg = _vacuum()
    run = pic.Run(cfg, "fp64")
    d = run.derived
    g, b, dt = d["gamma_b"], d["beta_b"], d["dt"]
    nsteps = int(6 * d["L_lab"] * g / dt) + 5
    run.step(nsteps)
    tp = nsteps * dt
    za = cfg["antenna_z_lab"] / g - b * tp
    ey = run.field(pic.PIC_F_EY)[0, 8]
    zs = np.arange(ey.size) * cfg["dz"]
    st = oracle.State(dict(cfg, ppc=0))
    ana = np.array([oracle.boost_fields(b, *st.laser_lab(g * (z + b * tp), g * (tp + b * z), 8 * cfg["dx"]))[0][1]
                    for z in zs])
    st.close()
    ana[zs <= za] = 0.0
    pk = np.abs(ana).max()
    err = np.abs(ey - ana)[zs > za + 0.2].max() / pk
    leak = np.abs(ey[zs < za - 0.2]).max() / pk
    print(f"\nvacuum antenna on the GPU: error {err:.3e}, backward {leak:.2e}")
    assert err < 1e-2 and leak < 1e-4
    run.close()


def test_station_downstream_records_the_lab_pulse():
    """Antenna at lab z = Z_a, station at Z_s > Z_a: the station's lab-frame
    record E_y(t_lab) is the lab pulse at z = Z_s (peak at t_peak + Z_s - Z_a),
    up to the Yee error of the boosted run and the z interpolation."""
    cfg = _vacuum()
    d0 = oracle.State(dict(cfg, ppc=0))
    g, b, Lz = d0.derived["gamma_b"], d0.derived["beta_b"], cfg["nz"] * cfg["dz"]
    Zs = cfg["antenna_z_lab"] + 0.1 * g * Lz
    cfg.update(n_stations=1, station_z0=Zs, station_dz=0.0, station_stride=16, station_cap=2000)
    run = pic.Run(cfg, "fp64")
    dt = run.derived["dt"]
    nsteps = int(0.5 * Lz / (b * dt))
    run.step(nsteps)
    t, data, n = run.station(0)
    run.close()
    assert n == t.size > 50
    ey = data[:, 1, 0, 0]
    ana = np.array([d0.laser_lab(Zs, tl, 0.0)[0][1] for tl in t])  # x = 0 node of the record
    d0.close()
    pk = np.abs(ana).max()
    err = np.abs(ey - ana).max() / pk
    print(f"\nlab pulse at the station: peak {pk:.3f}, max error {err:.3e} over {n} samples")
    assert pk > 0.9 * run.derived["E0_lab"]  # the whole pulse went past
    assert err < 2e-2


def test_graph_eager_timed_and_batch_agree():
    cfg = CASES["c1_plasma"]()
    plain = workloads.config("c1", seed=9)
    a = pic.Run(cfg, "fp64")
    b = pic.Run(cfg, "fp64", graph=False)
    c = pic.Run(cfg, "fp64")
    a.step(25)
    b.step(25)
    pic.pic_step_timed(c.handle, 25)
    ref = {comp: a.field(comp) for comp in range(6)}
    for r in (b, c):
        for comp in range(6):
            np.testing.assert_array_equal(r.field(comp), ref[comp])
    alone = pic.Run(plain, "fp64")
    alone.step(25)
    plain_ref = alone.field(pic.PIC_F_EY)
    alone.close()
    shared = torch.cuda.Stream()
    runs = [pic.Run(cfg, "fp64", stream=shared), pic.Run(plain, "fp64", stream=shared)]
    pic.pic_step_batch([r.handle for r in runs], [25, 25])
    shared.synchronize()
    for comp in range(6):
        np.testing.assert_array_equal(runs[0].field(comp), ref[comp])
    np.testing.assert_array_equal(runs[1].field(pic.PIC_F_EY), plain_ref)
    for r in runs + [a, b, c]:
        r.close()
