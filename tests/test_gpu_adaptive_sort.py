"""Tile re-sorts requested by the out-of-window path, in an open-z run with
plasma injection.

A hot plasma (lab thermal spread 0.5 at gamma_b = 2) streams through an
open box: its tiles spread beyond their windows between the cadence sorts,
so the run re-sorts on request in between.  Those sorts inject nothing;
only the cadence steps create plasma columns, as in the oracle, so the FP64
run must match the oracle particle by particle and in the fields (storage
order is the only thing the extra sorts change)."""
import numpy as np
import pytest

import oracle
from paper_0909_5603_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_0909_5603_amd import pic  # noqa: E402


def test_requested_sorts_keep_the_injection_schedule():
    cfg = workloads.config("c1", ppc=2, u_th=0.5, gamma_boost=2.0, sort_every=20)
    run = pic.Run(cfg, "fp64")
    st = oracle.State(cfg)
    slow = 0
    for _ in range(9):
        run.step(5)
        st.step(5)
        slow += run.diag(pic.PIC_DIAG_PARTICLES)["n_slow"]
    g, o = run.particles(), st.particles()
    og, oo = np.argsort(g["id"]), np.argsort(o["id"])
    assert np.array_equal(g["id"][og], o["id"][oo])
    ug = np.stack([g[k][og] for k in ("ux", "uy", "uz")], 1)
    uo = np.stack([o[k][oo] for k in ("ux", "uy", "uz")], 1)
    urel = (np.linalg.norm(ug - uo, axis=1) / np.linalg.norm(uo, axis=1)).max()
    Lx = cfg["nx"] * cfg["dx"]
    dz = np.abs(g["z"][og] - o["z"][oo]).max()
    dx = np.abs((g["x"][og] - o["x"][oo] + 0.5 * Lx) % Lx - 0.5 * Lx).max()
    fr = max(np.abs(run.field(c) - st.field(c)).max() for c in range(6)) / \
        max(np.abs(st.field(c)).max() for c in range(6))
    print(f"\n{g['id'].size} particles, {slow} out-of-window pushes, du/u {urel:.2e}, "
          f"dz {dz:.2e}, dx {dx:.2e}, fields {fr:.2e}")
    assert slow > 0
    assert urel < 1e-9 and dz < 1e-9 and dx < 1e-9 and fr < 1e-9
    run.close()
    st.close()
