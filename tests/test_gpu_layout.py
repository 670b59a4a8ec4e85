"""Particle order in storage, after the initial sort and after later ones.

Not a result of the method but a property the step kernel's speed relies on.
Plasma columns are created in groups of 64 consecutive slots: one lattice
slot of one tile's transverse plane (8x8 = 64 cells in 3D split precision;
where a plane is smaller, 8x4 in FP64 and 16 in 2D, consecutive columns are
interleaved), so a group covers 64 different cells.  The step kernel gives a
wavefront 64 consecutive slots of a tile starting at a multiple of 64; the
sort pads every tile's range to a multiple of 64 and places whole groups at
such offsets, the particles of groups split by a tile boundary behind them.
So most aligned 64-slot ranges hold one whole group, whose lanes add their
currents to 64 different LDS cells, also after the plasma has drifted
through several tiles and been sorted again.
"""
import numpy as np
import pytest

from paper_0909_5603_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_0909_5603_amd import pic  # noqa: E402

# drifting plasma without a laser: the sort's grouping alone is tested (a
# laser's transverse kicks move electrons across tile and cell boundaries)
CASES = {
    # name: (config, precision, tile-plane group size)
    "3d_split": (lambda: workloads.config("c5", nz=48, nx=32, ny=16, ppc=3, gamma_boost=13.0, a0=0.0),
                 "fp32", 64),
    "3d_fp64": (lambda: workloads.config("c5", nz=40, nx=16, ny=24, ppc=2, gamma_boost=13.0, a0=0.0),
                "fp64", 32),
    "2d_split": (lambda: workloads.config("c1", nz=64, nx=48, ppc=4, a0=0.0), "fp32", 16),
}


def _ranges(run, cfg, group):
    """For every aligned 64-slot range: number of live particles, whether
    they are one lattice slot of consecutive columns, and whether their cells
    are all different."""
    slots, live = pic.pic_particle_count(run.handle)
    assert slots % 64 == 0
    nperp = cfg["nx"] * (cfg["ny"] if cfg["dims"] == 3 else 1)
    ppc = cfg["ppc"]
    out = []
    for first in range(0, slots, 64):
        p = run.particles(first, 64)
        n = p["id"].size
        ids = p["id"].astype(np.int64)
        col, slot = ids // (nperp * ppc), ids % ppc
        k = np.floor(p["z"] / cfg["dz"]).astype(np.int64)
        i = np.floor(p["x"] / cfg["dx"]).astype(np.int64)
        j = np.floor(p["y"] / cfg["dy"]).astype(np.int64) if cfg["dims"] == 3 else np.zeros_like(k)
        cell = (k * 4096 + i) * 4096 + j
        # one lattice slot; one column, or 64 // group consecutive ones
        one_group = n == 64 and bool((slot == slot[0]).all()) and int(col.max() - col.min()) < 64 // group
        distinct = np.unique(cell).size == n
        out.append((n, one_group, distinct))
    return slots, live, out


@pytest.mark.parametrize("case", list(CASES))
def test_wavefront_ranges_hold_whole_groups(case):
    make, prec, group = CASES[case]
    cfg = make()
    run = pic.Run(cfg, prec)
    slots, live, r = _ranges(run, cfg, group)
    n_full = sum(1 for n, g, d in r if g)
    # after the initial sort: the tiles' ranges are padded (fewer than 64
    # empty slots each) and nearly every range is one whole group in 64 cells
    assert live <= slots < live + 64 * len(r)
    assert all(d for n, g, d in r if g)
    assert n_full * 64 > 0.9 * live, (n_full * 64, live)
    # two more sorts after the plasma has drifted through more than a tile:
    # whole groups stay aligned (groups split by a tile boundary are not)
    run.step(2 * cfg.get("sort_every", 20) + 1)
    slots2, live2, r2 = _ranges(run, cfg, group)
    run.close()
    n_full2 = sum(1 for n, g, d in r2 if g)
    n_dist2 = sum(1 for n, g, d in r2 if g and d)
    print(f"\n{case}: {live} particles, {n_full} whole-group ranges; after two sorts {live2}, "
          f"{n_full2} ({n_dist2} in 64 different cells)")
    if case == "3d_split":
        # a group is one column: the sort places it in the tile of its
        # lowest cell, so the drift does not split it (91 % of the slots
        # measured); its cells still differ unless a transverse kick (the
        # space-charge field where the plasma leaves through z = 0) moved a
        # member into a neighbour's cell
        assert n_full2 * 64 > 0.8 * live2, (n_full2 * 64, live2)
        assert n_dist2 > 0.6 * n_full2
    # where a group interleaves columns (FP64, 2D) it spans more z cells,
    # and groups that span more than the tile's slack are sorted by cell
