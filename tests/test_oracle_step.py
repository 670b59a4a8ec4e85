"""Pins for the oracle's full PIC step (CPU only): the coupling constants via
the cold plasma frequency, Gauss's law and continuity through whole steps,
and the open-z plasma flow of the parity configuration."""
import math

import numpy as np
import pytest

from paper_0909_5603_amd import workloads


def _lattice(cfg, per_dim):
    """Electrons on a regular in-cell lattice (per_dim^2 per cell, 2D)."""
    nz, nx = cfg["nz"], cfg["nx"]
    o = (np.arange(per_dim) + 0.5) / per_dim
    K, I, A, B = np.meshgrid(np.arange(nz), np.arange(nx), o, o, indexing="ij")
    z = ((K + A) * cfg["dz"]).ravel()
    x = ((I + B) * cfg["dx"]).ravel()
    return z, x


def test_cold_plasma_oscillates_at_plasma_frequency(ora):
    """Lab frame (gamma_b = 1), cold uniform plasma, long-wavelength velocity
    perturbation: E_z oscillates at omega_p = 1 in these units (leapfrog and
    grid corrections are below 1e-3 here).  A wrong charge, weight, current
    sign or unit would change the frequency or stop the oscillation."""
    cfg = workloads.config("c1", nz=64, nx=4, ppc=16, gamma_boost=1.0, a0=0.0, u_th=0.0,
                           bc_z="periodic")
    st = ora.State(cfg)
    z, x = _lattice(cfg, 4)
    n = z.size
    Lz = cfg["nz"] * cfg["dz"]
    k = 2 * math.pi / Lz
    uz = 1e-3 * np.sin(k * z)
    st.set_particles(z, x, np.zeros(n), np.zeros(n), np.zeros(n), uz)
    st.reset_gauss_reference()
    dt = st.derived["dt"]
    nsteps = int(3.2 * 2 * math.pi / dt)
    probe = []
    for _ in range(nsteps):
        st.step(1)
        probe.append(st.field(ora.EZ)[0, 1, cfg["nz"] // 4])
    probe = np.array(probe)
    s = np.sign(probe)
    idx = np.where(np.diff(s) != 0)[0]
    t = np.array([(i + 1 - probe[i] / (probe[i + 1] - probe[i]) + 1) * dt for i in idx])
    period = 2 * np.mean(np.diff(t))
    omega = 2 * math.pi / period
    assert omega == pytest.approx(1.0, abs=2e-3)
    assert np.abs(probe).max() > 1e-4
    st.close()


@pytest.mark.parametrize("dims", [2, 3])
def test_gauss_and_continuity_through_full_steps(ora, dims):
    """With a boosted laser, drifting thermal plasma and the ion background,
    (div E - rho) is conserved step to step and the continuity residual stays
    at round-off (periodic box)."""
    if dims == 3:
        cfg = workloads.config("c5", nz=24, nx=8, ny=8, ppc=2, bc_z="periodic", waist=0.2)
    else:
        cfg = workloads.config("c1", nz=48, nx=16, bc_z="periodic", waist=0.4)
    st = ora.State(cfg)
    cont = st.step(6, check_continuity=True)
    d = st.diag()
    assert cont < 1e-12
    assert d["gauss_drift"] < 1e-11
    assert d["Ez_max"] > 0
    st.close()


def test_parity_config_open_boundaries(ora):
    """Parity configuration, first 20 steps: the plasma streams through the
    open z ends (reservoir columns replace the electrons that leave), Gauss
    and continuity hold at round-off in the interior."""
    cfg = workloads.config("c1")
    st = ora.State(cfg)
    n0 = st.diag()["n_particles"]
    assert n0 == cfg["nz"] * cfg["nx"] * cfg["ppc"]
    cont = st.step(20, check_continuity=True)
    d = st.diag()
    assert cont < 1e-12
    assert d["gauss_drift"] < 1e-12
    # inflow balances outflow to within one lattice column
    assert abs(d["n_particles"] - n0) <= cfg["nx"] * cfg["ppc"]
    p = st.particles()
    assert p["z"].min() >= 0.0
    st.close()


def test_step_is_deterministic(ora):
    cfg = workloads.config("c1", nz=32, nx=16)
    a = ora.State(cfg)
    b = ora.State(cfg)
    a.step(15)
    b.step(15)
    pa, pb = a.particles(), b.particles()
    for k in ("z", "x", "uz", "ux", "uy"):
        np.testing.assert_array_equal(pa[k], pb[k])
    np.testing.assert_array_equal(a.field(ora.EZ), b.field(ora.EZ))
