"""The C-ABI library loads, exports every function include/pic.h declares,
and its pure host calls (sizing, validation) work without a GPU."""
import os
import re

import pytest

from paper_0909_5603_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def pic():
    from paper_0909_5603_amd import pic as m

    if not os.path.exists(m.LIB_PATH):
        from paper_0909_5603_amd import build

        build.build()
    m.lib()
    return m


def _declared():
    src = open(os.path.join(ROOT, "include", "pic.h")).read()
    return sorted(set(re.findall(r"^(?:pic_status|const char\*)\s+(pic_\w+)\(", src, re.M)))


def test_exports_every_declared_symbol(pic):
    names = _declared()
    assert len(names) >= 12
    L = pic.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(pic.EXPORTS) == names


def test_state_bytes_scale_with_the_workload(pic):
    small = pic.pic_state_bytes(pic.make_params(workloads.config("c1")))
    big = pic.pic_state_bytes(pic.make_params(workloads.config("c5")))
    fp64 = pic.pic_state_bytes(pic.make_params(workloads.config("c5"), "fp64"))
    assert 1e6 < small < 1e8
    # 537M particles x 2 buffers x 32 B plus fields
    assert 3.0e10 < big < 6.0e10
    assert fp64 > 1.5 * big


@pytest.mark.parametrize("over,status", [
    (dict(nx=20), -1), (dict(dims=4), -1), (dict(cfl=1.0), -4), (dict(cfl=0.0), -4),
    (dict(gamma_boost=0.5), -1), (dict(ppc=-1), -1), (dict(sort_every=0), -1),
    (dict(nz=4000), -1), (dict(pol_axis=3), -1), (dict(filter_passes=17), -1),
    (dict(filter_passes=-1), -1), (dict(filter_passes=1, filter_compensate=2), -1),
    (dict(laser_antenna=2), -1), (dict(laser_antenna=1, antenna_z_lab=float("nan")), -1),
    (dict(laser_antenna=1, antenna_t_peak=float("inf")), -1),
])
def test_invalid_parameters(pic, over, status):
    cfg = workloads.config("c1", **over)
    with pytest.raises(pic.PicError) as e:
        pic.pic_state_bytes(pic.make_params(cfg))
    assert e.value.status == status
    assert pic.pic_last_error()


def test_null_arguments(pic):
    import ctypes

    L = pic.lib()
    assert L.pic_free(None) == 0
    assert L.pic_state_bytes(None, None) == -1
    assert L.pic_step(None, 1) == -1
    assert L.pic_diag(None, 0, None) == -1
    out = ctypes.c_void_p()
    p = pic.make_params(workloads.config("c1"))
    assert L.pic_init_boosted(ctypes.byref(p), None, 0, None, ctypes.byref(out)) == -1
    # the batched steps reject an empty, oversized or NULL-holding batch
    # before touching a device
    runs = (ctypes.c_void_p * 257)()
    steps = (ctypes.c_int * 257)(*([1] * 257))
    for fn in (L.pic_step_batch, L.pic_step_batch_noalloc):
        assert fn(None, None, 0) == -1
        assert fn(runs, steps, 0) == -1
        assert fn(runs, steps, 257) == -1
        assert fn(runs, steps, 2) == -1  # NULL runs


def test_copy_bench_rejects_bad_sizes_before_any_launch(pic):
    L = pic.lib()
    assert L.pic_copy_bench(None, None, 0, None) == 0  # empty copy: nothing to do
    assert L.pic_copy_bench(None, None, -16, None) == -1
    assert L.pic_copy_bench(None, None, 24, None) == -1  # not a multiple of 16
    assert L.pic_copy_bench(None, None, 32, None) == -1  # NULL buffers
    assert L.pic_copy_bench(8, 40, 32, None) == -1  # misaligned addresses: rejected before a launch
    assert L.pic_stream_bench(0, None, None, 0, None) == 0
    assert L.pic_stream_bench(3, None, None, 32, None) == -1  # unknown mode
    assert L.pic_stream_bench(0, None, None, 24, None) == -1  # not a multiple of 16
    assert L.pic_stream_bench(1, None, None, 32, None) == -1  # NULL buffers
    assert L.pic_stream_bench(2, 0, 40, 32, None) == -1  # misaligned destination


def test_filter_buffers_are_allocated_only_when_used(pic):
    base = pic.pic_state_bytes(pic.make_params(workloads.config("c1")))
    filt = pic.pic_state_bytes(pic.make_params(workloads.config("c1", filter_passes=2)))
    npts = (workloads.config("c1")["nz"] + 1) * workloads.config("c1")["nx"]
    # two R-typed current sets (3 components) and two double node arrays
    assert filt - base >= 2 * 3 * 4 * npts + 2 * 8 * npts


@pytest.mark.parametrize("over", [
    dict(n_stations=-1), dict(n_stations=65537), dict(n_stations=2, station_stride=0, station_cap=4),
    dict(n_stations=2, station_stride=10_000, station_cap=4), dict(n_stations=2, station_stride=1, station_cap=0),
    dict(n_stations=2, station_stride=1, station_cap=4, station_z0=float("nan")),
    dict(n_stations=2, station_stride=1, station_cap=4, station_dz=float("inf")),
    dict(n_stations=65536, station_stride=1, station_cap=1 << 20),  # record beyond 64 GiB
])
def test_invalid_station_parameters(pic, over):
    with pytest.raises(pic.PicError) as e:
        pic.pic_state_bytes(pic.make_params(workloads.config("c1", **over)))
    assert e.value.status == -1
    assert "station" in pic.pic_last_error()


def test_station_record_size(pic):
    cfg = workloads.config("c5", nz=32, nx=16, ny=16, ppc=1)
    base = pic.pic_state_bytes(pic.make_params(cfg))
    S, stride, cap = 3, 4, 50
    withst = pic.pic_state_bytes(pic.make_params(dict(cfg, n_stations=S, station_stride=stride,
                                                      station_cap=cap)))
    p = pic.make_params(dict(cfg, n_stations=S, station_stride=stride, station_cap=cap))
    nys, nxs = pic.station_shape(p)
    assert (nys, nxs) == (4, 4)
    rec = S * cap * (6 * nys * nxs + 1) * 8 + S * 8
    assert rec <= withst - base <= rec + 4 * 256
    # 2D: one transverse row
    p2 = pic.make_params(workloads.config("c1", n_stations=1, station_stride=2, station_cap=3))
    assert pic.station_shape(p2) == (1, workloads.config("c1")["nx"] // 2)


def test_read_station_argument_checks(pic):
    import ctypes

    L = pic.lib()
    n = ctypes.c_int64()
    assert L.pic_read_station(None, 0, ctypes.byref(n), None, None, 0) == -1
