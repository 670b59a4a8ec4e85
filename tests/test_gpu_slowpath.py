"""The particle kernel's out-of-window path (k_particles_hbm) against the
oracle.

A hot plasma (lab thermal spread 0.5, boosted at gamma_b = 2, periodic box,
sort cadence 50 steps) spreads the particles of a tile over more cells than
its LDS window holds within a few steps; those particles are gathered from
and deposited into HBM directly, and the run re-sorts its tiles at the next
step.  The results must not depend on which path a
particle took: FP64 matches the oracle to rounding, split precision keeps
the momentum and continuity bounds, and the diagnostics report that the
path was taken."""
import numpy as np
import pytest

import oracle
from paper_0909_5603_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_0909_5603_amd import pic  # noqa: E402


def _cfg():
    return workloads.config("c5", nz=32, nx=16, ny=16, ppc=2, gamma_boost=2.0, u_th=0.5, a0=0.0,
                            bc_z="periodic", sort_every=50)


def _match(a, b):
    oa, ob = np.argsort(a["id"]), np.argsort(b["id"])
    ids, ia, ib = np.intersect1d(a["id"][oa], b["id"][ob], assume_unique=True, return_indices=True)
    return ({k: v[oa][ia] for k, v in a.items()}, {k: v[ob][ib] for k, v in b.items()}, ids.size)


def _urel(g, o):
    ug = np.stack([g["ux"], g["uy"], g["uz"]], 1)
    uo = np.stack([o["ux"], o["uy"], o["uz"]], 1)
    return np.linalg.norm(ug - uo, axis=1) / np.linalg.norm(uo, axis=1)


def _wrapdiff(a, b, L):
    return np.abs((a - b + 0.5 * L) % L - 0.5 * L)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_out_of_window_particles_match_oracle(prec):
    cfg = _cfg()
    run = pic.Run(cfg, prec, continuity=(prec == "fp32"))
    st = oracle.State(cfg, round_f32=(prec == "fp32"))
    slow, worst, cont = 0, 0.0, 0.0
    for _ in range(8):
        run.step(1)
        st.step(1)
        d = run.diag(pic.PIC_DIAG_FIELDS | pic.PIC_DIAG_PARTICLES)
        slow += d["n_slow"]
        if prec == "fp32":
            cont = max(cont, d["cont_resid"])
    g, o, m = _match(run.particles(), st.particles())
    assert m == st.particles()["id"].size
    worst = _urel(g, o).max()
    L = {"z": cfg["nz"] * cfg["dz"], "x": cfg["nx"] * cfg["dx"], "y": cfg["ny"] * cfg["dy"]}
    perr = max(_wrapdiff(g[k], o[k], L[k]).max() for k in ("z", "x", "y"))
    n = st.particles()["id"].size
    print(f"\n{prec}: {slow} out-of-window pushes over 8 steps ({slow / (8 * n):.1%}), "
          f"max du/u {worst:.3e}, max dx {perr:.3e}, continuity {cont:.2e}")
    # the path is taken (re-sorting after a step with more than 1/128 of the
    # particles out of their windows keeps it from growing further)
    assert slow > 0
    if prec == "fp64":
        assert worst < 1e-10 and perr < 1e-10
    else:
        assert worst < 1e-5 and cont <= 1e-6
    run.close()
    st.close()
