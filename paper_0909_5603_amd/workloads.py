"""Seeded synthetic workload descriptions.

These are the inputs both the GPU library and the CPU oracle are given: plain
parameter dictionaries (grid, cell size, particles per cell, seed, boost,
laser and plasma parameters in laboratory units) and seeded numpy generators
for the pusher microbenchmark and the serving request stream.  Nothing here
computes any part of the PIC method itself.

The paper's workloads are laser-wakefield stages specified by physical
parameters (laboratory density, laser a0, wavelength and waist, boost factor),
so synthetic inputs of those shapes stand in for them; there is no dataset.
"""
from __future__ import annotations

import numpy as np

_BASE_2D = dict(
    dims=2, nx=64, ny=1, dz=0.05, dx=0.05, dy=0.05, cfl=0.95, ppc=4, seed=1,
    gamma_boost=5.0, n_lab_cm3=1e17, u_th=1e-3, a0=1.0, lambda0_um=0.8, waist=8.0,
    tau_lab=0.0, pol_axis=2, bc_z="open", pusher="vay", sort_every=20,
)

# 30 um waist expressed in c/omega_p at 1e17 cm^-3 (c/omega_p = 16.8046 um)
_WAIST_30UM_1E17 = 30.0 / 16.804638405152193

CONFIGS = {
    # 2D3V plain method, parity configuration: 128(z) x 64(x), 4 e-/cell,
    # gamma_boost 5, a0 1, 0.8 um laser, waist 8 c/omega_p, 200 steps.
    "c1": dict(_BASE_2D, nz=128, nx=64, steps=200),
    # 3D3V LWFA 256x128x128, 8 e-/cell (33.5M), gamma_boost 13, a0 2, 2000 steps.
    "c3": dict(_BASE_2D, dims=3, nz=256, nx=128, ny=128, ppc=8, seed=4, gamma_boost=13.0,
               a0=2.0, waist=_WAIST_30UM_1E17, pol_axis=1, steps=2000),
    # 3D3V LWFA 512x256x256, 16 e-/cell (537M), gamma_boost 30, 1000 steps,
    # sort every 20 steps.
    "c5": dict(_BASE_2D, dims=3, nz=512, nx=256, ny=256, ppc=16, seed=6, gamma_boost=30.0,
               a0=2.0, waist=_WAIST_30UM_1E17, pol_axis=1, steps=1000),
}


def config(name: str, **overrides) -> dict:
    cfg = dict(CONFIGS[name])
    cfg.update(overrides)
    return cfg


def scaled_3d(nz: int, nx: int, ny: int, ppc: int, base: str = "c5", **over) -> dict:
    """A 3D box of the given size with every other parameter of ``base``."""
    cfg = config(base, nz=nz, nx=nx, ny=ny, ppc=ppc)
    cfg.update(over)
    return cfg


# ------------------------------------------------------------------ pusher set
PUSH_DT = 0.1


def pusher_set(n: int, kind: str, seed: int):
    """Pusher microbenchmark particles (2^27 in the full benchmark).

    kind == "crossed": momenta along +z with gamma log-uniform in [1e2, 1e6],
    B = 1 along y and a per-particle E = -v x B (so E_x = v_z).
    kind == "gyration": B = 1 along z, E = 0, momentum perpendicular to B at a
    random azimuth with the same gamma law.

    Returns (u (n,3) f64, Ex (n,) f64, B (3,) f64, cell (n,3) i32, off (n,3) f64)
    with positions as an integer cell plus an offset in [0,1) on a unit grid.
    """
    rng = np.random.default_rng(seed)
    gam = 10.0 ** rng.uniform(2.0, 6.0, size=n)
    umag = np.sqrt(gam * gam - 1.0)
    u = np.zeros((n, 3))
    if kind == "crossed":
        u[:, 2] = umag
        Ex = umag / np.sqrt(1.0 + umag * umag)
        B = np.array([0.0, 1.0, 0.0])
    elif kind == "gyration":
        phi = rng.uniform(0.0, 2 * np.pi, size=n)
        u[:, 0] = umag * np.cos(phi)
        u[:, 1] = umag * np.sin(phi)
        Ex = np.zeros(n)
        B = np.array([0.0, 0.0, 1.0])
    else:
        raise ValueError(kind)
    cell = rng.integers(0, 1 << 20, size=(n, 3)).astype(np.int32)
    off = rng.uniform(0.0, 1.0, size=(n, 3))
    return u, Ex, B, cell, off


# ------------------------------------------------------------------ serving
def serving_stream(n_requests: int, seed: int = 5, rate_per_s: float = 20.0,
                   z_range=(64, 1024), x_range=(32, 512), ppc_range=(1, 16),
                   gamma_range=(2.0, 30.0), a0_range=(0.5, 3.0), steps_range=(100, 2000)):
    """Poisson stream of 2D3V boosted-frame runs (the serving workload):
    grid z and x uniform over powers of two, ppc uniform, gamma_boost
    log-uniform, a0 uniform, step count uniform; every other parameter as in
    the 2D parity configuration.  Returns a list of (arrival_time_s, cfg)."""
    rng = np.random.default_rng(seed)
    zs = [1 << k for k in range(int(np.log2(z_range[0])), int(np.log2(z_range[1])) + 1)]
    xs = [1 << k for k in range(int(np.log2(x_range[0])), int(np.log2(x_range[1])) + 1)]
    t = 0.0
    out = []
    for r in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        cfg = dict(_BASE_2D)
        cfg.update(
            nz=int(rng.choice(zs)), nx=int(rng.choice(xs)),
            ppc=int(rng.integers(ppc_range[0], ppc_range[1] + 1)),
            gamma_boost=float(np.exp(rng.uniform(np.log(gamma_range[0]), np.log(gamma_range[1])))),
            a0=float(rng.uniform(*a0_range)),
            steps=int(rng.integers(steps_range[0], steps_range[1] + 1)),
            seed=int(1000 + r),
        )
        out.append((t, cfg))
    return out
