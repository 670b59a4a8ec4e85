"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Tolerances: the FP64 path matches the oracle to rounding (1e-10 relative
after ten steps); the split-precision FP32 path meets the stated bounds:
per-particle momentum relative error <= 1e-5 over 10 steps, field energy and
wake amplitude (max |E_z|) relative error <= 1e-3 over the full run, and a
continuity residual <= 1e-6 relative on every step.  FP32 runs are compared
with an oracle whose created offsets and momenta are rounded to FP32 the way
split storage keeps them, so the comparison measures the step, not the
initial rounding."""
import numpy as np
import pytest

import oracle
from paper_0909_5603_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_0909_5603_amd import pic  # noqa: E402


def _by_id(p):
    o = np.argsort(p["id"], kind="stable")
    return {k: v[o] for k, v in p.items()}


def _match(a, b):
    """Particles present in both sets, aligned by lattice id."""
    a, b = _by_id(a), _by_id(b)
    common, ia, ib = np.intersect1d(a["id"], b["id"], assume_unique=True, return_indices=True)
    return {k: v[ia] for k, v in a.items()}, {k: v[ib] for k, v in b.items()}, common.size


def _u_relerr(g, o, floor=0.0):
    """|u_gpu - u_oracle| / max(|u_oracle|, floor) per particle; the floor
    (the thermal momentum) keeps the error of an electron at rest, as in an
    unboosted run, from being divided by a momentum near zero."""
    ug = np.stack([g["ux"], g["uy"], g["uz"]], 1)
    uo = np.stack([o["ux"], o["uy"], o["uz"]], 1)
    return np.linalg.norm(ug - uo, axis=1) / np.maximum(np.linalg.norm(uo, axis=1), floor)


def _field_relerr(run, st):
    """max |F_gpu - F_oracle| over all E and B components, relative to the
    largest field magnitude (components that vanish exactly in the oracle,
    such as B_z of a plane wave, carry only rounding on the GPU)."""
    diff, scale = 0.0, 1e-300
    for c in range(6):
        g = run.field(c)
        o = st.field(c)
        scale = max(scale, np.abs(o).max())
        diff = max(diff, np.abs(g - o).max())
    return diff / scale


def _small3d(**over):
    cfg = workloads.config("c5", nz=48, nx=16, ny=16, ppc=2, gamma_boost=13.0, waist=0.3)
    cfg.update(over)
    return cfg


CASES = {
    "c1": lambda: workloads.config("c1"),
    "c1_periodic": lambda: workloads.config("c1", nz=64, bc_z="periodic"),
    "3d_open": lambda: _small3d(),
    "3d_periodic": lambda: _small3d(nz=32, bc_z="periodic"),
    # smallest boxes: one 8x8x8 tile (two 8x8x4 tiles in FP64), smaller than
    # a tile's LDS window, which then wraps onto itself in every direction
    "3d_min_periodic": lambda: _small3d(nz=8, nx=8, ny=8, bc_z="periodic"),
    "3d_min_open": lambda: _small3d(nz=8, nx=8, ny=8),
    "2d_min_periodic": lambda: workloads.config("c1", nz=16, nx=16, bc_z="periodic"),
    # z not a multiple of the tile depth: a ragged last tile, whose window
    # also wraps across the periodic z boundary
    "3d_ragged_z_periodic": lambda: _small3d(nz=27, bc_z="periodic"),
    "3d_ragged_z_open": lambda: _small3d(nz=29),
    "2d_ragged_z_periodic": lambda: workloads.config("c1", nz=40, nx=32, bc_z="periodic"),
    # no boost (gamma_b = 1): the laboratory frame itself, plasma at rest; the
    # wavelength is long enough to be resolved without the boost
    "2d_lab_frame": lambda: workloads.config("c1", gamma_boost=1.0, lambda0_um=20.0),
    "3d_lab_frame": lambda: _small3d(nz=24, gamma_boost=1.0, lambda0_um=20.0),
    # the other polarisation in each dimension: in the simulation plane in
    # 2D (E along x), along y in 3D
    "2d_pol_x": lambda: workloads.config("c1", nz=64, pol_axis=1),
    "3d_pol_y": lambda: _small3d(nz=24, pol_axis=2),
}


@pytest.mark.parametrize("case", list(CASES))
def test_init_transform_fp64(case):
    """Boosted laser fields and plasma (positions, boosted momenta, ids)."""
    cfg = CASES[case]()
    run = pic.Run(cfg, "fp64")
    st = oracle.State(cfg)
    assert _field_relerr(run, st) < 1e-12
    g, o, n = _match(run.particles(), st.particles())
    assert n == st.particles()["id"].size == run.particles()["id"].size
    for k in ("z", "x", "y"):
        np.testing.assert_allclose(g[k], o[k], rtol=0, atol=1e-12)
    assert _u_relerr(g, o).max() < 1e-12
    d = run.diag()
    do = st.diag()
    assert d["n_particles"] == do["n_particles"]
    assert d["U_E"] == pytest.approx(do["U_E"], rel=1e-12)
    assert d["U_B"] == pytest.approx(do["U_B"], rel=1e-10)
    run.close()
    st.close()


@pytest.mark.parametrize("case", list(CASES))
def test_steps_fp64_match_oracle(case):
    cfg = CASES[case]()
    run = pic.Run(cfg, "fp64")
    st = oracle.State(cfg)
    for n in (1, 4, 10):
        run.step(n - run.diag(0)["step"])
        st.step(n - st.step_index)
        g, o, m = _match(run.particles(), st.particles())
        assert m > 0.99 * st.particles()["id"].size
        assert _u_relerr(g, o, cfg["u_th"]).max() < 1e-10, f"step {n}"
        for k in ("z", "x", "y"):
            assert np.abs(g[k] - o[k]).max() < 1e-10
        assert _field_relerr(run, st) < 1e-10, f"step {n}"
    d, do = run.diag(), st.diag()
    for k in ("U_E", "U_B", "KE", "Ez_max"):
        assert d[k] == pytest.approx(do[k], rel=1e-9), k
    assert d["n_particles"] == do["n_particles"]
    assert d["gauss_drift"] < 1e-10
    run.close()
    st.close()


@pytest.mark.parametrize("case", ["c1", "3d_open", "3d_min_periodic", "3d_ragged_z_periodic"])
def test_fp32_momentum_and_continuity_10_steps(case):
    cfg = CASES[case]()
    run = pic.Run(cfg, "fp32", continuity=True)
    st = oracle.State(cfg, round_f32=True)
    worst = 0.0
    for n in range(1, 11):
        run.step(1)
        st.step(1)
        g, o, m = _match(run.particles(), st.particles())
        assert m > 0.99 * st.particles()["id"].size
        worst = max(worst, _u_relerr(g, o).max())
        d = run.diag(pic.PIC_DIAG_FIELDS)
        assert d["cont_resid"] <= 1e-6, f"step {n}: continuity {d['cont_resid']}"
    assert worst <= 1e-5
    run.close()
    st.close()


def test_fp32_energy_and_wake_full_parity_run():
    """Parity configuration (2D, 200 steps): field energy and wake amplitude
    within 1e-3 of the FP64 oracle every 10 steps."""
    cfg = workloads.config("c1")
    run = pic.Run(cfg, "fp32")
    st = oracle.State(cfg, round_f32=True)
    worst = {"U": 0.0, "Ez": 0.0}
    for n in range(10, cfg["steps"] + 1, 10):
        run.step(10)
        st.step(10)
        d, do = run.diag(), st.diag()
        U, Uo = d["U_E"] + d["U_B"], do["U_E"] + do["U_B"]
        worst["U"] = max(worst["U"], abs(U - Uo) / Uo)
        worst["Ez"] = max(worst["Ez"], abs(d["Ez_max"] - do["Ez_max"]) / do["Ez_max"])
        assert d["err_bits"] == 0
    assert worst["U"] <= 1e-3, worst
    assert worst["Ez"] <= 1e-3, worst
    run.close()
    st.close()


def test_graph_replay_matches_eager():
    cfg = workloads.config("c1", nz=64, nx=32)
    a = pic.Run(cfg, "fp64", graph=True)
    b = pic.Run(cfg, "fp64", graph=False)
    for _ in range(4):
        a.step(7)
        b.step(7)
        ga, gb, m = _match(a.particles(), b.particles())
        assert m == ga["id"].size
        assert _u_relerr(ga, gb).max() < 1e-12
        np.testing.assert_allclose(a.field(pic.PIC_F_EZ), b.field(pic.PIC_F_EZ), rtol=0, atol=1e-11)
    a.close()
    b.close()


def test_batched_runs_equal_alone():
    """Runs advanced together in one set of launches give the same state as
    each run advanced alone."""
    cfgs = [workloads.config("c1", nz=64, nx=32, seed=11),
            workloads.config("c1", nz=128, nx=16, gamma_boost=3.0, seed=12),
            workloads.config("c1", nz=32, nx=64, ppc=2, a0=2.0, seed=13)]
    steps = [12, 25, 7]
    alone = []
    for c, s in zip(cfgs, steps):
        r = pic.Run(c, "fp64")
        r.step(s)
        alone.append(r)
    shared = torch.cuda.Stream()
    mixed = [pic.Run(c, "fp64", stream=shared) for c in cfgs]
    pic.pic_step_batch([r.handle for r in mixed], steps)
    shared.synchronize()
    for r1, r2, s in zip(alone, mixed, steps):
        assert r2.diag(0)["step"] == s
        g1, g2, m = _match(r1.particles(), r2.particles())
        assert m == g1["id"].size
        assert _u_relerr(g1, g2).max() < 1e-12
        np.testing.assert_allclose(r1.field(pic.PIC_F_EY), r2.field(pic.PIC_F_EY), rtol=0, atol=1e-10)
    for r in alone + mixed:
        r.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_batched_3d_runs_equal_alone_bitwise(prec):
    """3D runs advanced in one batch equal each run advanced alone bit for
    bit (currents are integer sums, so the order in which tiles and
    particles are visited cannot show), through a cadence sort with
    injection.  The batch holds more than 2048 tiles, not a multiple of 64,
    so the particle kernel deals its tiles to the XCDs in full 64-tile
    blocks and a short last one; the runs drift at different speeds, so the
    sort's work items differ from run to run."""
    cfgs = [workloads.config("c5", nz=128, nx=64, ny=64, ppc=2, seed=21),
            workloads.config("c5", nz=136, nx=64, ny=72, ppc=2, gamma_boost=13.0, a0=1.0, seed=22),
            workloads.config("c5", nz=20, nx=24, ny=16, ppc=3, gamma_boost=5.0, a0=0.0, seed=23)]
    steps = [23, 21, 22]  # each crosses the cadence sort at step 20
    alone = []
    for c, s in zip(cfgs, steps):
        r = pic.Run(c, prec)
        r.step(s)
        alone.append(r)
    shared = torch.cuda.Stream()
    mixed = [pic.Run(c, prec, stream=shared) for c in cfgs]
    tiles = sum(pic.pic_get_derived(r.handle)["ntiles"] for r in mixed)
    assert tiles > 2048 and tiles % 64 != 0, tiles
    pic.pic_step_batch([r.handle for r in mixed], steps)
    shared.synchronize()
    for r1, r2, s in zip(alone, mixed, steps):
        assert r2.diag(0)["step"] == s
        g1, g2, m = _match(r1.particles(), r2.particles())
        assert m == g1["id"].size == g2["id"].size
        for k in ("z", "x", "y", "ux", "uy", "uz"):
            assert np.array_equal(g1[k], g2[k]), k
        for f in (pic.PIC_F_EX, pic.PIC_F_EY, pic.PIC_F_EZ, pic.PIC_F_BX, pic.PIC_F_BY, pic.PIC_F_BZ):
            assert np.array_equal(r1.field(f), r2.field(f)), f
    for r in alone + mixed:
        r.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_vacuum_laser_against_the_oracle(prec, tol):
    """No plasma (ppc = 0): the boosted laser alone propagates through the
    Yee grid and out through the Mur ends; fields and the diagnostics match
    the oracle's."""
    cfg = workloads.config("c1", nz=32, nx=16, ppc=0)
    r = pic.Run(cfg, prec)
    st = oracle.State(cfg)
    r.step(25)
    st.step(25)
    assert _field_relerr(r, st) < tol
    d, do = r.diag(), st.diag()
    assert d["n_particles"] == 0 == do["n_particles"]
    assert d["KE"] == 0.0
    for k in ("U_E", "U_B", "Ez_max"):
        assert d[k] == pytest.approx(do[k], rel=10 * tol, abs=1e-300)
    assert do["U_E"] > 0
    r.close()
    st.close()


def test_no_plasma_and_no_laser_edge_cases():
    cfg = workloads.config("c1", nz=32, nx=16, a0=0.0)
    r = pic.Run(cfg, "fp32")
    st = oracle.State(cfg, round_f32=True)
    assert r.diag()["n_particles"] == 32 * 16 * 4
    r.step(5)
    st.step(5)
    d = r.diag()
    # electrons leave through z = 0 and enter from the reservoir; E_z is the
    # field of the current noise of the randomly placed drifting electrons
    do = st.diag()
    assert d["n_particles"] == do["n_particles"]
    assert d["Ez_max"] == pytest.approx(do["Ez_max"], rel=1e-3)
    r.close()
    st.close()


@pytest.mark.parametrize("dims", [2, 3])
def test_boris_option_matches_oracle_boris(dims):
    """The Boris pusher selected in the step kernels (2D, and the 3D
    instantiations): FP64 matches the oracle's Boris, split precision keeps
    the FP32 momentum bound."""
    if dims == 2:
        cfg = workloads.config("c1", nz=32, nx=16, pusher="boris")
    else:
        cfg = _small3d(nz=24, pusher="boris")
    run = pic.Run(cfg, "fp64")
    st = oracle.State(cfg)
    run.step(5)
    st.step(5)
    g, o, m = _match(run.particles(), st.particles())
    assert m == st.particles()["id"].size
    assert _u_relerr(g, o).max() < 1e-10
    assert _field_relerr(run, st) < 1e-10
    run.close()
    st.close()
    run = pic.Run(cfg, "fp32")
    st = oracle.State(cfg, round_f32=True)
    run.step(5)
    st.step(5)
    g, o, m = _match(run.particles(), st.particles())
    assert m > 0.99 * st.particles()["id"].size
    assert _u_relerr(g, o).max() <= 1e-5
    run.close()
    st.close()


def test_invalid_parameters_rejected():
    cfg = workloads.config("c1", nx=20)
    with pytest.raises(pic.PicError) as e:
        pic.pic_state_bytes(pic.make_params(cfg))
    assert e.value.status == -1
    cfg = workloads.config("c1", cfl=1.2)
    with pytest.raises(pic.PicError) as e:
        pic.pic_state_bytes(pic.make_params(cfg))
    assert e.value.status == -4
    p = pic.make_params(workloads.config("c1"))
    buf = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(pic.PicError) as e:
        pic.pic_init_boosted(p, buf.data_ptr(), 1024, torch.cuda.current_stream().cuda_stream)
    assert e.value.status == -2


def _largest_nz(cfg):
    """Largest nz the library accepts for cfg (the z cell index, reservoir
    included, must fit the packed cell)."""
    lo, hi = 8, 4096
    while lo < hi:
        mid = (lo + hi + 1) // 2
        try:
            pic.pic_state_bytes(pic.make_params(dict(cfg, nz=mid)))
            lo = mid
        except pic.PicError:
            hi = mid - 1
    return lo


@pytest.mark.parametrize("case", ["2d_max_nz", "3d_max_nx", "3d_max_ny"])
def test_largest_accepted_sizes_match_oracle(case):
    """Boxes at the limits of the packed cell index (z with its reservoir,
    1024 cells across x or y): FP64 steps match the oracle to rounding."""
    if case == "2d_max_nz":
        cfg = workloads.config("c1", nx=16, ppc=1)
        cfg["nz"] = _largest_nz(cfg)
        with pytest.raises(pic.PicError):
            pic.pic_state_bytes(pic.make_params(dict(cfg, nz=cfg["nz"] + 1)))
    elif case == "3d_max_nx":
        cfg = _small3d(nz=8, nx=1024, ny=8, ppc=1)
    else:
        cfg = _small3d(nz=8, nx=8, ny=1024, ppc=1)
    run = pic.Run(cfg, "fp64")
    st = oracle.State(cfg)
    run.step(5)
    st.step(5)
    g, o, m = _match(run.particles(), st.particles())
    print(f"\n{case}: nz {cfg['nz']} nx {cfg['nx']} ny {cfg.get('ny')}: {m} particles")
    assert m == st.particles()["id"].size
    assert _u_relerr(g, o).max() < 1e-10
    for k in ("z", "x", "y"):
        assert np.abs(g[k] - o[k]).max() < 1e-10
    assert _field_relerr(run, st) < 1e-10
    run.close()
    st.close()
