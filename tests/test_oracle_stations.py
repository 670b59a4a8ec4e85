"""Pins for the oracle's laboratory-frame stations (CPU only).

A station is the plane z_lab = Z.  At boosted time t' = n dt it sits at
z' = Z/gamma_b - beta_b t' and samples the lab event of time
t_lab = t'/gamma_b + beta_b Z (inverse Lorentz transform of (z', t')).
Fixed by the mathematics: fields that Maxwell's equations leave static
(uniform transverse E and B, E_z and B_z linear in z) are recorded exactly
as their lab-frame transforms at z'(n), linear interpolation being exact for
linear fields; the sample count and lab times follow the closed form; and a
boosted laser recorded at a station shows the laboratory carrier frequency
omega0 (not the Doppler-shifted boosted one) and B = z x E.
"""
import math

import numpy as np
import pytest

from paper_0909_5603_amd import workloads


def _static_state(ora, **over):
    cfg = workloads.config("c1", nz=64, nx=16, ppc=0, a0=0.0, bc_z="periodic",
                           n_stations=3, station_stride=4, station_cap=64)
    cfg.update(over)
    st = ora.State(cfg)
    d = st.derived
    gam, beta = d["gamma_b"], d["beta_b"]
    Lz = cfg["nz"] * cfg["dz"]
    # stations whose boosted position crosses the middle of the box
    cfg["station_z0"] = gam * 0.7 * Lz
    cfg["station_dz"] = gam * 0.05 * Lz
    st.close()
    return cfg, gam, beta, Lz


def test_static_fields_are_recorded_as_their_lab_transform(ora):
    cfg, gam, beta, Lz = _static_state(ora)
    st = ora.State(cfg)
    dz = cfg["dz"]
    ny, nx, nzf = st.shape
    k = np.arange(nzf)
    ex, ey, bx, by = 0.3, -0.7, 0.45, 0.2
    a, b, c, e = 0.1, 0.02, -0.05, 0.03
    st.field(ora.EX)[...] = ex
    st.field(ora.EY)[...] = ey
    st.field(ora.BX)[...] = bx
    st.field(ora.BY)[...] = by
    st.field(ora.EZ)[...] = (a + b * (k + 0.5) * dz)[None, None, :]
    st.field(ora.BZ)[...] = (c + e * k * dz)[None, None, :]
    nsteps = 40
    st.step(nsteps)
    dt = st.derived["dt"]
    for q in range(cfg["n_stations"]):
        Z = cfg["station_z0"] + q * cfg["station_dz"]
        zp = Z / gam - beta * dt * np.arange(nsteps)
        inside = (zp >= 0) & (zp < Lz)
        times, data, count = st.station(q)
        assert count == inside.sum()
        n_in = np.nonzero(inside)[0]
        np.testing.assert_allclose(times, n_in * dt / gam + beta * Z, rtol=0, atol=1e-12)
        z = zp[n_in]
        expect = np.stack([
            np.full_like(z, gam * (ex + beta * by)), np.full_like(z, gam * (ey - beta * bx)),
            a + b * z,
            np.full_like(z, gam * (bx - beta * ey)), np.full_like(z, gam * (by + beta * ex)),
            c + e * z], 1)
        # away from the periodic seam, where a linear profile wraps
        ok = (z > 2 * dz) & (z < Lz - 2 * dz)
        assert ok.sum() > 10
        for comp in range(6):
            np.testing.assert_allclose(data[ok, comp], expect[ok, comp][:, None, None] * np.ones(data.shape[2:]),
                                       rtol=0, atol=1e-12)
    st.close()


def test_capacity_drops_but_counts(ora):
    cfg, gam, beta, Lz = _static_state(ora, station_cap=5)
    st = ora.State(cfg)
    st.step(30)
    times, data, count = st.station(0)
    assert count > 5 and times.size == 5 and data.shape[0] == 5
    st.close()


def test_station_sees_the_laboratory_laser():
    """Vacuum, open z: the boosted laser (Doppler-stretched by D+) passes a
    station; its lab-frame record has the laboratory carrier frequency k0
    (c = 1), lab amplitude E0_lab and B_x = -E_y (B = z x E)."""
    import oracle as ora

    cfg = workloads.config("c1", nz=256, nx=16, ppc=0, n_stations=1, station_stride=16,
                           station_cap=400)
    st0 = ora.State(cfg)
    d = st0.derived
    st0.close()
    gam, beta, dt = d["gamma_b"], d["beta_b"], d["dt"]
    zc = d["zc_boost"]
    # the pulse (+c) meets the station (-beta) after about 60 steps
    tm = 60 * dt
    cfg["station_z0"] = gam * (zc + (1 + beta) * tm)
    st = ora.State(cfg)
    st.step(140)
    times, data, count = st.station(0)
    assert count == times.size
    ey = data[:, 1, 0, 0]   # lab E_y on the axis row
    bx = data[:, 3, 0, 0]
    peak = np.abs(ey).max()
    assert peak == pytest.approx(d["E0_lab"], rel=0.1)
    assert np.abs(ey + bx).max() < 0.05 * peak
    # carrier frequency from zero crossings inside the pulse envelope
    strong = np.abs(ey) > 0.2 * peak
    i0, i1 = np.nonzero(strong)[0][[0, -1]]
    seg_t, seg = times[i0:i1 + 1], ey[i0:i1 + 1]
    s = np.sign(seg)
    idx = np.nonzero(np.diff(s) != 0)[0]
    tz = seg_t[idx] - seg[idx] * (seg_t[idx + 1] - seg_t[idx]) / (seg[idx + 1] - seg[idx])
    assert idx.size >= 3
    omega = math.pi / np.mean(np.diff(tz))
    assert omega == pytest.approx(d["k0_lab"], rel=0.05)
    st.close()
