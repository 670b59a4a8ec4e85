"""Pins for the oracle's laser antenna (CPU only).

The antenna is the lab plane z = Z_a, drifting at -beta_b in the boosted
frame; its sources make the grid carry the boosted incident wave above the
plane and nothing below (the discrete residual of H (E_i, B_i), H the unit
step above the plane).  What the mathematics fixes:
* above the plane the field is the boosted lab pulse (a vacuum solution for
  the flat-phase-front pulse) up to the Yee scheme's own error, which falls
  as dz^2 with dt / dz fixed, for any plane speed;
* below the plane there is no field (backward emission vanishes up to the
  mismatch between the analytic and the discrete wave);
* the emitted energy is the pulse's energy;
* in 2D with the polarisation out of plane the antenna current has zero
  divergence, so Gauss's law and the particle continuity stay at round-off
  with a plasma present;
* a pulse already crossing the plane at t' = 0 starts as H (E_i, B_i) and
  evolves the same way;
* closing the loop, a laboratory-frame station downstream of the plane
  records the laboratory pulse, converging at second order.
"""
import numpy as np
import pytest

from paper_0909_5603_amd import workloads


def _antenna_cfg(ora, nz, gamma=5.0, lam=2.0, z_frac=0.55, delay=3.0, ppc=0, **over):
    """2D vacuum (or plasma) box, open z, pulse of 1/12 the box (boosted
    length), antenna at z_frac of the box at t' = 0, envelope peak reaching
    the plane `delay` lab e-fold lengths after t' = 0."""
    dz = 12.8 / nz
    cfg = workloads.config("c1", nz=nz, nx=16, dz=dz, dx=dz, ppc=ppc, lambda0_um=lam,
                           gamma_boost=gamma, **over)
    st = ora.State(cfg)
    d = st.derived
    st.close()
    Lz = nz * dz
    Ll = Lz / 12 / d["dplus"]
    Za = d["gamma_b"] * z_frac * Lz
    cfg.update(laser_antenna=1, antenna_z_lab=Za, antenna_t_peak=d["beta_b"] * Za + delay * Ll,
               tau_lab=Ll)
    return cfg, Ll


def _run_and_compare(ora, cfg, nsteps):
    st = ora.State(cfg)
    d = st.derived
    g, b, dt = d["gamma_b"], d["beta_b"], d["dt"]
    st.step(nsteps)
    tp = nsteps * dt
    za = cfg["antenna_z_lab"] / g - b * tp
    ny, nx, nzf = st.shape
    E = st.field(ora.EY)[0, nx // 2]
    zs = np.arange(nzf) * cfg["dz"]
    x = (nx // 2) * cfg["dx"]
    ana = np.array([ora.boost_fields(b, *st.laser_lab(g * (z + b * tp), g * (tp + b * z), x))[0][1]
                    for z in zs])
    ana[zs <= za] = 0.0
    above, below = zs > za + 0.2, zs < za - 0.2
    pk = np.abs(ana).max()
    out = dict(err=np.abs(E - ana)[above].max() / pk, leak=np.abs(E[below]).max() / pk,
               energy=(E[above] ** 2).sum() / (ana[above] ** 2).sum(), pk=pk, diag=st.diag())
    st.close()
    return out


@pytest.mark.parametrize("gamma", [1.5, 5.0])
def test_emitted_wave_is_the_boosted_pulse_to_second_order(ora, gamma):
    lam = 10.0 if gamma < 2 else 2.0  # about 30 cells per boosted wavelength at nz = 256
    res = []
    for nz in (256, 512):
        cfg, Ll = _antenna_cfg(ora, nz, gamma=gamma, lam=lam)
        st = ora.State(cfg)
        d = st.derived
        st.close()
        nsteps = int(6 * Ll * d["gamma_b"] / d["dt"]) + 5  # the whole pulse has passed the plane
        res.append(_run_and_compare(ora, cfg, nsteps))
    e1, e2 = res[0]["err"], res[1]["err"]
    print(f"\ngamma {gamma}: error {e1:.3e} -> {e2:.3e}, leak {res[1]['leak']:.2e}, energy {res[1]['energy']:.5f}")
    assert e2 < 0.3 * e1          # second order: a factor 4 per halving
    assert e2 < 1e-2
    assert res[1]["leak"] < 1e-4  # no backward emission
    assert abs(res[1]["energy"] - 1.0) < 5e-3


def test_pulse_already_crossing_the_plane_at_start(ora):
    """Envelope peak at the plane at t' = 0: the box starts with the upper
    half of the pulse (H times the incident wave) and the antenna emits the
    rest."""
    cfg, Ll = _antenna_cfg(ora, 512, delay=0.0, z_frac=0.45)
    st = ora.State(cfg)
    d = st.derived
    ey0 = st.field(ora.EY)[0, 8].copy()
    st.close()
    za0 = cfg["antenna_z_lab"] / d["gamma_b"]
    zs = np.arange(ey0.size) * cfg["dz"]
    assert np.abs(ey0[zs <= za0]).max() == 0.0
    assert np.abs(ey0[zs > za0]).max() > 0.5 * d["E0_lab"] * d["dminus"]
    nsteps = int(3 * Ll * d["gamma_b"] / d["dt"]) + 5
    r = _run_and_compare(ora, cfg, nsteps)
    print(f"\nerror {r['err']:.3e} leak {r['leak']:.2e}")
    assert r["err"] < 1e-2 and r["leak"] < 1e-4


def test_antenna_outside_the_box_or_zero_amplitude_emits_nothing(ora):
    cfg, Ll = _antenna_cfg(ora, 128, z_frac=1.3)  # the plane is above the box throughout
    st = ora.State(cfg)
    st.step(40)
    assert np.abs(st.field(ora.EY)).max() == 0.0
    st.close()
    cfg, Ll = _antenna_cfg(ora, 128, a0=0.0)
    st = ora.State(cfg)
    st.step(60)
    assert all(np.abs(st.field(c)).max() == 0.0 for c in range(6))
    st.close()


def test_gauss_law_and_continuity_with_plasma_2d(ora):
    """Polarisation out of the (z, x) plane: the antenna current is along y
    and has zero divergence."""
    cfg, Ll = _antenna_cfg(ora, 128, lam=0.8, delay=0.5, ppc=2)
    st = ora.State(cfg)
    cont = st.step(40, check_continuity=True)
    d = st.diag()
    assert cont < 1e-12
    assert d["gauss_drift"] < 1e-12
    assert d["U_E"] > 0
    st.close()


def test_downstream_station_records_the_laboratory_pulse(ora):
    """The whole lab -> boosted -> lab loop inside the oracle: the pulse given
    in the laboratory is emitted by the drifting antenna, evolved in the
    boosted frame, and recorded by a station 0.1 L_z gamma_b downstream of
    the plane; the station's lab-frame E_y(t_lab) is the lab pulse at the
    station's z, up to the Yee and interpolation errors (second order)."""
    errs = []
    for nz in (256, 512):
        cfg, Ll = _antenna_cfg(ora, nz)
        st0 = ora.State(dict(cfg, ppc=0))
        d = st0.derived
        g, b, Lz = d["gamma_b"], d["beta_b"], cfg["nz"] * cfg["dz"]
        Zs = cfg["antenna_z_lab"] + 0.1 * g * Lz
        st = ora.State(dict(cfg, n_stations=1, station_z0=Zs, station_dz=0.0,
                            station_stride=cfg["nx"], station_cap=4000))
        st.step(int(0.5 * Lz / (b * d["dt"])))
        t, data, n = st.station(0)
        ey = data[:, 1, 0, 0]
        ana = np.array([st0.laser_lab(Zs, tl, 0.0)[0][1] for tl in t])
        pk = np.abs(ana).max()
        assert pk > 0.9 * d["E0_lab"]  # the whole pulse went past
        errs.append(np.abs(ey - ana).max() / pk)
        st.close()
        st0.close()
    print(f"\nlab pulse at the station: {errs[0]:.2e} -> {errs[1]:.2e}")
    assert errs[1] < 0.35 * errs[0] and errs[1] < 5e-3
