"""pic_step_batch_noalloc (batch table in the library's device array, no
allocation) against pic_step_batch on the same runs: every electron's
momentum and position and the fields agree exactly (the current is summed in
integers and the per-electron arithmetic does not depend on the batch), on
two calls in a row, the second with a smaller batch."""
import numpy as np
import pytest

from paper_0909_5603_amd import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_0909_5603_amd import pic  # noqa: E402


def _cfgs():
    return [workloads.config("c1", nz=64, nx=32, ppc=3, seed=21, a0=2.0),
            workloads.config("c1", nz=128, nx=16, gamma_boost=3.0, seed=22),
            workloads.config("c1", nz=32, nx=64, ppc=2, seed=23),
            workloads.config("c1", nz=96, nx=32, ppc=5, gamma_boost=12.0, seed=24)]


def _same(ra, rb):
    pa, pb = ra.particles(), rb.particles()
    oa, ob = np.argsort(pa["id"]), np.argsort(pb["id"])
    assert np.array_equal(pa["id"][oa], pb["id"][ob])
    for k in ("z", "x", "ux", "uy", "uz"):
        assert np.array_equal(pa[k][oa], pb[k][ob]), k
    for c in range(6):
        assert np.array_equal(ra.field(c), rb.field(c)), c
    assert ra.diag(0)["step"] == rb.diag(0)["step"]


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_batch_matches_the_batch_entry_point(precision):
    cfgs = _cfgs()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    ref = [pic.Run(c, precision, stream=sa) for c in cfgs]
    new = [pic.Run(c, precision, stream=sb) for c in cfgs]
    # first call: the whole batch, runs of different lengths drop out
    steps1 = [30, 12, 25, 7]
    pic.pic_step_batch([r.handle for r in ref], steps1)
    pic.pic_step_batch_noalloc([r.handle for r in new], steps1)
    sa.synchronize()
    sb.synchronize()
    for a, b in zip(ref, new):
        _same(a, b)
    # second call: a smaller batch (two runs, fewer steps)
    steps2 = [9, 4]
    pic.pic_step_batch([ref[2].handle, ref[0].handle], steps2)
    pic.pic_step_batch_noalloc([new[2].handle, new[0].handle], steps2)
    sa.synchronize()
    sb.synchronize()
    for a, b in zip(ref, new):
        _same(a, b)
    for r in ref + new:
        r.close()


def test_noalloc_batch_with_filter_antenna_and_stations():
    """Runs with the current filter, a laser antenna and lab-frame stations in
    the batch (the launches those options add) give the same results."""
    cfgs = [workloads.config("c1", nz=64, nx=32, ppc=2, seed=31),
            workloads.config("c1", nz=64, nx=32, ppc=2, seed=32, filter_passes=2, filter_compensate=1),
            workloads.config("c1", seed=33, filter_passes=1, n_stations=3, station_z0=30.0, station_dz=5.0,
                             station_stride=4, station_cap=200, laser_antenna=1, antenna_z_lab=25.0,
                             antenna_t_peak=25.0)]
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    ref = [pic.Run(c, "fp32", stream=sa) for c in cfgs]
    new = [pic.Run(c, "fp32", stream=sb) for c in cfgs]
    for steps in ([20, 35, 40], [0, 6, 11]):
        pic.pic_step_batch([r.handle for r in ref], steps)
        pic.pic_step_batch_noalloc([r.handle for r in new], steps)
        sa.synchronize()
        sb.synchronize()
        for a, b in zip(ref, new):
            _same(a, b)
        for q in range(3):
            ta, fa, na = ref[2].station(q)
            tb, fb, nb = new[2].station(q)
            assert na == nb and np.array_equal(ta, tb) and np.array_equal(fa, fb), q
    for r in ref + new:
        r.close()


def test_noalloc_batch_rejects_more_runs_than_the_table_holds():
    run = pic.Run(workloads.config("c1", nz=32, nx=16, ppc=1), "fp32")
    with pytest.raises(pic.PicError):
        pic.pic_step_batch_noalloc([run.handle] * 257, [1] * 257)
    run.close()
