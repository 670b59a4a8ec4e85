"""Particle order in storage after the initial sort.

Not a result of the method but a property the step kernel's speed relies on:
plasma columns are created with the lattice slot outermost and the transverse
cells enumerated tile by tile, and the sort keeps each wavefront's particles
in order, so every aligned group of one tile plane's worth of slots (8x8 = 64
cells in 3D split precision, 8x4 = 32 in FP64, 16 in 2D) holds one lattice
slot of one column, and where a plane is smaller than a wavefront the columns
are interleaved, so every aligned group of 64 slots covers 64 different
cells: the lanes of a step-kernel wavefront do not add their currents to the
same LDS addresses.
"""
import numpy as np
import pytest

from paper_0909_5603_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_0909_5603_amd import pic  # noqa: E402

CASES = {
    # name: (config, precision, group size)
    "3d_split": (lambda: workloads.config("c5", nz=48, nx=32, ny=16, ppc=3, gamma_boost=13.0, waist=0.3),
                 "fp32", 64),
    "3d_fp64": (lambda: workloads.config("c5", nz=40, nx=16, ny=24, ppc=2, gamma_boost=13.0, waist=0.3),
                "fp64", 32),
    "2d_split": (lambda: workloads.config("c1", nz=64, nx=48, ppc=4), "fp32", 16),
}


@pytest.mark.parametrize("case", list(CASES))
def test_aligned_groups_are_one_slot_of_one_tile_plane(case):
    make, prec, group = CASES[case]
    cfg = make()
    run = pic.Run(cfg, prec)
    slots, live = pic.pic_particle_count(run.handle)
    p = run.particles()
    run.close()
    n = p["id"].size
    assert n == live == slots  # a fresh sort leaves no removed slots
    assert n % group == 0
    nperp = cfg["nx"] * (cfg["ny"] if cfg["dims"] == 3 else 1)
    ppc = cfg["ppc"]
    ids = p["id"].astype(np.int64)
    col = ids // (nperp * ppc)
    slot = ids % ppc
    k = np.floor(p["z"] / cfg["dz"]).astype(np.int64)
    i = np.floor(p["x"] / cfg["dx"]).astype(np.int64)
    j = np.floor(p["y"] / cfg["dy"]).astype(np.int64) if cfg["dims"] == 3 else np.zeros_like(k)
    cell = (k * 4096 + i) * 4096 + j
    g = n // group
    for name, v in (("column", col), ("slot", slot)):
        v = v.reshape(g, group)
        assert (v == v[:, :1]).all(), f"a group mixes lattice {name}s"
    # wavefront-sized groups: one slot, consecutive columns, 64 distinct cells
    w = n // 64
    assert n % 64 == 0
    ws, wc = slot.reshape(w, 64), col.reshape(w, 64)
    ncw = 64 // group
    # the columns left over when their count is not a multiple of ncw keep
    # one column per wavefront; they are the topmost ones
    ncol = int(col.max()) + 1
    full = wc.max(axis=1) < ncol - ncol % ncw
    assert full.mean() > 0.9
    assert (ws == ws[:, :1])[full].all()
    assert ((wc.max(axis=1) - wc.min(axis=1))[full] <= ncw - 1).all()
    cells = np.sort(cell.reshape(w, 64), axis=1)
    dup = (cells[:, 1:] == cells[:, :-1]).any(axis=1)
    print(f"\n{case}: {n} particles, {w} wavefront groups ({full.sum()} from interleaved columns), "
          f"with a repeated cell: {dup[full].sum()}")
    assert not dup[full].any()
