"""Pins for the oracle's Yee field update and field gather (CPU only)."""
import math

import numpy as np
import pytest

from paper_0909_5603_amd import workloads


def _vacuum(dims, nz, nx, ny=1, bc="periodic", **over):
    cfg = workloads.config("c1", dims=dims, nz=nz, nx=nx, ny=ny, ppc=0, a0=0.0, bc_z=bc)
    cfg.update(over)
    return cfg


@pytest.mark.parametrize("dims", [2, 3])
def test_yee_standing_wave_dispersion(ora, dims):
    """Standing wave cos(kz z) cos(kx x) in a periodic box with B = 0: the
    leapfrog gives E^n = cos(n theta) E^0 exactly, with
    sin(theta/2) = dt sqrt(sum_d (sin(k_d d/2)/d)^2)."""
    nz, nx, ny = 32, 16, (8 if dims == 3 else 1)
    cfg = _vacuum(dims, nz, nx, ny)
    st = ora.State(cfg)
    dz = dx = cfg["dz"]
    kz, kx = 2 * math.pi * 3 / (nz * dz), 2 * math.pi * 2 / (nx * dx)
    comp = ora.EY if dims == 2 else ora.EY
    F = st.field(comp)
    # E_y at (x_i, y_{j+1/2}, z_k): depends only on z and x -> divergence free
    z = np.arange(F.shape[2]) * dz
    x = np.arange(F.shape[1]) * dx
    E0 = np.cos(kz * z)[None, None, :] * np.cos(kx * x)[None, :, None] * np.ones((F.shape[0], 1, 1))
    F[...] = E0
    st.reset_gauss_reference()
    dt = st.derived["dt"]
    s = dt * math.sqrt((math.sin(kz * dz / 2) / dz) ** 2 + (math.sin(kx * dx / 2) / dx) ** 2)
    theta = 2 * math.asin(s)
    for n in (1, 7, 40):
        st.step(n - st.step_index)
        np.testing.assert_allclose(st.field(comp), math.cos(n * theta) * E0, atol=1e-12)
    st.close()


def _div_b(B, d):
    """div B at cell centres of a periodic box; B arrays shaped (ny, nx, nz)."""
    bx, by, bz = B
    dz, dx, dy = d
    out = (np.roll(bx, -1, axis=1) - bx) / dx + (np.roll(bz, -1, axis=2) - bz) / dz
    if by.shape[0] > 1:
        out = out + (np.roll(by, -1, axis=0) - by) / dy
    return out


def test_div_b_preserved(ora):
    cfg = _vacuum(3, 8, 6, 5)
    st = ora.State(cfg)
    rng = np.random.default_rng(4)
    for c in (ora.EX, ora.EY, ora.EZ, ora.BX, ora.BY, ora.BZ):
        st.field(c)[...] = rng.normal(size=st.shape)
    d = (cfg["dz"], cfg["dx"], cfg["dy"])
    before = _div_b([st.field(c).copy() for c in (ora.BX, ora.BY, ora.BZ)], d)
    for _ in range(5):
        st.half_B()
        for c in (ora.EX, ora.EY, ora.EZ):
            st.field(c)[...] = rng.normal(size=st.shape)
    after = _div_b([st.field(c).copy() for c in (ora.BX, ora.BY, ora.BZ)], d)
    np.testing.assert_allclose(after, before, atol=1e-9 * np.abs(before).max())
    st.close()


def test_mur_absorbs_outgoing_pulse(ora):
    """Open z ends: a laser pulse leaves through the +z end.  With first-order
    Mur the reflected energy is a small fraction; a wrong sign of the Mur
    coefficient or a missing boundary update reflects most of it."""
    cfg = _vacuum(2, 256, 8, a0=1.0, bc="open", waist=1e9, gamma_boost=5.0)
    st = ora.State(cfg)
    d0 = st.diag()
    u0 = d0["U_E"] + d0["U_B"]
    assert u0 > 0
    nsteps = int(1.1 * 0.5 * cfg["nz"] * cfg["dz"] / st.derived["dt"]) + int(
        4 * st.derived["L_boost"] / st.derived["dt"])
    st.step(nsteps)
    d1 = st.diag()
    assert (d1["U_E"] + d1["U_B"]) / u0 < 1e-3
    st.close()


def test_laser_travels_forward_at_yee_group_velocity(ora):
    """The boosted laser pulse moves in +z at the Yee scheme's discrete group
    velocity for on-axis propagation,
    v_g = cos(k dz/2) / sqrt(1 - (dt/dz)^2 sin^2(k dz/2)),  k = 2 pi / lambda'."""
    cfg = _vacuum(2, 512, 4, a0=1.0, bc="periodic", waist=1e9, gamma_boost=5.0)
    st = ora.State(cfg)

    def centroid():
        e = st.field(ora.EY)[0].sum(axis=0) ** 2
        z = np.arange(e.size) * cfg["dz"]
        return (e * z).sum() / e.sum()

    c0 = centroid()
    n = 200
    st.step(n)
    v = (centroid() - c0) / (n * st.derived["dt"])
    d = st.derived
    k = 2 * math.pi / (d["dplus"] * cfg["lambda0_um"] / d["skin_um"])
    h = 0.5 * k * cfg["dz"]
    r = d["dt"] / cfg["dz"]
    vg = math.cos(h) / math.sqrt(1 - (r * math.sin(h)) ** 2)
    assert v == pytest.approx(vg, abs=2e-3)
    st.close()


@pytest.mark.parametrize("dims", [2, 3])
def test_gather_reproduces_affine_fields(ora, dims):
    """Linear interpolation at each component's own stagger reproduces any
    affine field exactly."""
    ny = 8 if dims == 3 else 1
    cfg = _vacuum(dims, 8, 8, ny, bc="open")
    st = ora.State(cfg)
    rng = np.random.default_rng(9)
    coefs = rng.normal(size=(6, 4))
    stag = {ora.EX: (0, 1, 0), ora.EY: (0, 0, 1), ora.EZ: (1, 0, 0),
            ora.BX: (1, 0, 1), ora.BY: (1, 1, 0), ora.BZ: (0, 1, 1)}
    dz, dx, dy = cfg["dz"], cfg["dx"], cfg["dy"]
    for c, (hz, hx, hy) in stag.items():
        F = st.field(c)
        z = (np.arange(F.shape[2]) + 0.5 * hz) * dz
        x = (np.arange(F.shape[1]) + 0.5 * hx) * dx
        y = (np.arange(F.shape[0]) + 0.5 * hy) * dy if dims == 3 else np.zeros(1)
        a = coefs[c]
        F[...] = a[0] + a[1] * z[None, None, :] + a[2] * x[None, :, None] + (a[3] * y[:, None, None] if dims == 3 else 0)
    for _ in range(50):
        pz, px = rng.uniform(1.5, 6.0) * dz, rng.uniform(1.5, 6.0) * dx
        py = rng.uniform(1.5, 6.0) * dy if dims == 3 else 0.0
        E, B = st.gather(pz, px, py)
        vals = np.concatenate([E, B])
        for c in range(6):
            a = coefs[c]
            ref = a[0] + a[1] * pz + a[2] * px + (a[3] * py if dims == 3 else 0.0)
            assert vals[c] == pytest.approx(ref, abs=1e-12)
    st.close()


def test_gather_outside_open_z_is_zero(ora):
    cfg = _vacuum(2, 8, 8, bc="open")
    st = ora.State(cfg)
    for c in range(6):
        st.field(c)[...] = 1.0
    E, B = st.gather(20 * cfg["dz"], 0.3)
    assert np.all(E == 0) and np.all(B == 0)
    st.close()
