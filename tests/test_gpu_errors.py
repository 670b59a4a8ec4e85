"""Device-side error reporting, forced from the host with an input that the
kernels handle in bounds.

A thermal spread of 1e30 (the momenta stay finite in FP32, their squares do
not) makes 1 + u^2 overflow in the split-precision step: such a particle
does not move (its velocity factor 1/sqrt(1 + u^2) is 0, every offset and
cell stays in range) and the step sets the non-finite-momentum bit, which
pic_diag reports as PIC_ESTATE with a message.  A run with ordinary inputs
on the same device afterwards is unaffected."""
import numpy as np
import pytest

from paper_0909_5603_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_0909_5603_amd import pic  # noqa: E402


def test_non_finite_momentum_is_reported():
    cfg = workloads.config("c1", nz=32, nx=16, ppc=1, u_th=1e30)
    run = pic.Run(cfg, "fp32")
    run.step(2)
    with pytest.raises(pic.PicError) as e:
        run.diag()
    assert e.value.status == -7  # PIC_ESTATE
    assert "non-finite" in pic.pic_last_error()
    # the particles stayed where they were created
    p = run.particles()
    assert p["z"].size > 0 and np.isfinite(p["z"]).all() and np.isfinite(p["x"]).all()
    run.close()
    ok = pic.Run(workloads.config("c1", nz=32, nx=16, ppc=1), "fp32")
    ok.step(2)
    assert ok.diag()["err_bits"] == 0
    ok.close()
