"""Thin ctypes binding of libpic (include/pic.h): argument marshalling only.

Every step of the PIC path runs in the HIP kernels of ``libpic.so``; PyTorch
supplies device memory (one ``torch.uint8`` buffer per run) and the stream.
Importing this module on a machine without the built library raises
``ImportError``: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpic.so")

PIC_OK = 0
PIC_BC_OPEN, PIC_BC_PERIODIC = 0, 1
PIC_VAY, PIC_BORIS = 0, 1
PIC_FP32_SPLIT, PIC_FP64 = 0, 1
PIC_DIAGF_CONTINUITY = 1
PIC_DIAG_FIELDS, PIC_DIAG_PARTICLES, PIC_DIAG_GAUSS, PIC_DIAG_ALL = 1, 2, 4, 7
PIC_F_EX, PIC_F_EY, PIC_F_EZ, PIC_F_BX, PIC_F_BY, PIC_F_BZ, PIC_F_JX_LAST, PIC_F_JY_LAST, PIC_F_JZ_LAST = range(9)
PIC_OPT_GRAPH = 1

STATUS = {0: "PIC_OK", -1: "PIC_EINVAL", -2: "PIC_EBUDGET", -3: "PIC_EHIP", -4: "PIC_ECFL",
          -5: "PIC_ENAN", -6: "PIC_ECAPACITY", -7: "PIC_ESTATE"}


class PicError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class pic_lab_params(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int), ("nz", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("dz", ctypes.c_double), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("cfl", ctypes.c_double), ("ppc", ctypes.c_int), ("seed", ctypes.c_uint64),
        ("gamma_boost", ctypes.c_double), ("n_lab_cm3", ctypes.c_double), ("u_th", ctypes.c_double),
        ("a0", ctypes.c_double), ("lambda0_um", ctypes.c_double), ("waist", ctypes.c_double),
        ("tau_lab", ctypes.c_double), ("pol_axis", ctypes.c_int), ("bc_z", ctypes.c_int),
        ("pusher", ctypes.c_int), ("precision", ctypes.c_int), ("sort_every", ctypes.c_int),
        ("diag_flags", ctypes.c_uint), ("filter_passes", ctypes.c_int),
        ("filter_compensate", ctypes.c_int), ("n_stations", ctypes.c_int),
        ("station_z0", ctypes.c_double), ("station_dz", ctypes.c_double),
        ("station_stride", ctypes.c_int), ("station_cap", ctypes.c_int),
        ("laser_antenna", ctypes.c_int), ("antenna_z_lab", ctypes.c_double),
        ("antenna_t_peak", ctypes.c_double),
    ]


class pic_diag_out(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("t", ctypes.c_double), ("U_E", ctypes.c_double),
                ("U_B", ctypes.c_double), ("Ez_max", ctypes.c_double), ("KE", ctypes.c_double),
                ("n_particles", ctypes.c_int64), ("cont_resid", ctypes.c_double),
                ("gauss_drift", ctypes.c_double), ("err_bits", ctypes.c_uint32),
                ("n_slow", ctypes.c_int64)]


class pic_derived(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "dt", "beta_b", "gamma_b", "dminus", "dplus", "skin_um", "k0_lab", "E0_lab",
        "L_lab", "L_boost", "zc_boost", "weight", "dV")] + [
        ("reservoir", ctypes.c_int), ("nzf", ctypes.c_int), ("capacity", ctypes.c_int64),
        ("ntiles", ctypes.c_int)]


# names declared in include/pic.h, in order
EXPORTS = ["pic_state_bytes", "pic_init_boosted", "pic_step", "pic_step_timed", "pic_step_batch",
           "pic_step_batch_noalloc", "pic_diag",
           "pic_particle_count", "pic_read_particles", "pic_read_fields", "pic_read_station", "pic_get_derived",
           "pic_set_option", "pic_free", "pic_last_error", "pic_push_bench", "pic_copy_bench",
           "pic_stream_bench"]

_lib = None


def lib():
    """Load libpic.so (raises ImportError when it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    P = ctypes.POINTER(pic_lab_params)
    L.pic_state_bytes.argtypes = [P, ctypes.POINTER(ctypes.c_size_t)]
    L.pic_init_boosted.argtypes = [P, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
    L.pic_step.argtypes = [vp, ctypes.c_int]
    L.pic_step_timed.argtypes = [vp, ctypes.c_int, dp]
    L.pic_step_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int), ctypes.c_int]
    L.pic_step_batch_noalloc.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(ctypes.c_int), ctypes.c_int]
    L.pic_diag.argtypes = [vp, ctypes.c_uint, ctypes.POINTER(pic_diag_out)]
    L.pic_particle_count.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.pic_read_particles.argtypes = [vp, i64, i64] + [dp] * 6 + [ctypes.POINTER(ctypes.c_uint32),
                                                              ctypes.POINTER(i64)]
    L.pic_read_fields.argtypes = [vp, ctypes.c_int, dp, i64]
    L.pic_read_station.argtypes = [vp, ctypes.c_int, ctypes.POINTER(i64), dp, dp, i64]
    L.pic_get_derived.argtypes = [vp, ctypes.POINTER(pic_derived)]
    L.pic_set_option.argtypes = [vp, ctypes.c_int, ctypes.c_int]
    L.pic_free.argtypes = [vp]
    L.pic_last_error.argtypes = []
    L.pic_last_error.restype = ctypes.c_char_p
    L.pic_copy_bench.argtypes = [ctypes.c_void_p, ctypes.c_void_p, i64, ctypes.c_void_p]
    L.pic_copy_bench.restype = ctypes.c_int
    L.pic_stream_bench.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, i64, ctypes.c_void_p]
    L.pic_push_bench.argtypes = [ctypes.c_int, ctypes.c_int, i64, ctypes.c_int, ctypes.c_double, dp,
                                 vp, vp, vp, vp, vp]
    for n in EXPORTS:
        if n != "pic_last_error":
            getattr(L, n).restype = ctypes.c_int
    _lib = L
    return L


def _check(status: int):
    if status != PIC_OK:
        raise PicError(status, lib().pic_last_error().decode())


# ------------------------------------------------------------------ C-ABI mirrors
def pic_last_error() -> str:
    return lib().pic_last_error().decode()


def make_params(cfg: dict, precision: str = "fp32", continuity: bool = False) -> pic_lab_params:
    """pic_lab_params from a workload description (a plain dict)."""
    p = pic_lab_params()
    p.dims = int(cfg["dims"]); p.nz = int(cfg["nz"]); p.nx = int(cfg["nx"])
    p.ny = int(cfg.get("ny", 1)) if int(cfg["dims"]) == 3 else 1
    p.dz = float(cfg["dz"]); p.dx = float(cfg["dx"]); p.dy = float(cfg.get("dy", cfg["dx"]))
    p.cfl = float(cfg["cfl"]); p.ppc = int(cfg["ppc"]); p.seed = int(cfg["seed"])
    p.gamma_boost = float(cfg["gamma_boost"]); p.n_lab_cm3 = float(cfg["n_lab_cm3"])
    p.u_th = float(cfg["u_th"]); p.a0 = float(cfg["a0"]); p.lambda0_um = float(cfg["lambda0_um"])
    p.waist = float(cfg["waist"]); p.tau_lab = float(cfg.get("tau_lab", 0.0))
    p.pol_axis = int(cfg["pol_axis"])
    p.bc_z = PIC_BC_PERIODIC if cfg.get("bc_z", "open") == "periodic" else PIC_BC_OPEN
    p.pusher = PIC_BORIS if cfg.get("pusher", "vay") == "boris" else PIC_VAY
    p.precision = PIC_FP64 if precision == "fp64" else PIC_FP32_SPLIT
    p.sort_every = int(cfg.get("sort_every", 20))
    p.diag_flags = PIC_DIAGF_CONTINUITY if continuity else 0
    p.filter_passes = int(cfg.get("filter_passes", 0))
    p.filter_compensate = int(cfg.get("filter_compensate", 0))
    p.n_stations = int(cfg.get("n_stations", 0))
    p.station_z0 = float(cfg.get("station_z0", 0.0)); p.station_dz = float(cfg.get("station_dz", 0.0))
    p.station_stride = int(cfg.get("station_stride", 1)); p.station_cap = int(cfg.get("station_cap", 0))
    p.laser_antenna = int(cfg.get("laser_antenna", 0))
    p.antenna_z_lab = float(cfg.get("antenna_z_lab", 0.0))
    p.antenna_t_peak = float(cfg.get("antenna_t_peak", 0.0))
    return p


def pic_state_bytes(params: pic_lab_params) -> int:
    n = ctypes.c_size_t(0)
    _check(lib().pic_state_bytes(ctypes.byref(params), ctypes.byref(n)))
    return int(n.value)


def pic_init_boosted(params: pic_lab_params, dev_ptr: int, nbytes: int, stream: int) -> int:
    h = ctypes.c_void_p()
    _check(lib().pic_init_boosted(ctypes.byref(params), ctypes.c_void_p(dev_ptr), nbytes,
                                  ctypes.c_void_p(stream), ctypes.byref(h)))
    return h.value


def pic_step(run: int, nsteps: int):
    _check(lib().pic_step(ctypes.c_void_p(run), int(nsteps)))


def pic_step_timed(run: int, nsteps: int) -> dict:
    """Mean device milliseconds per step of each stage (HIP events)."""
    ms = (ctypes.c_double * 4)()
    _check(lib().pic_step_timed(ctypes.c_void_p(run), int(nsteps), ms))
    return {"sort": ms[0], "particles": ms[1], "fields": ms[2], "step": ms[3]}


def pic_step_batch(runs, nsteps):
    n = len(runs)
    arr = (ctypes.c_void_p * n)(*runs)
    st = (ctypes.c_int * n)(*[int(s) for s in nsteps])
    _check(lib().pic_step_batch(arr, st, n))


def pic_step_batch_noalloc(runs, nsteps):
    n = len(runs)
    arr = (ctypes.c_void_p * n)(*runs)
    st = (ctypes.c_int * n)(*[int(s) for s in nsteps])
    _check(lib().pic_step_batch_noalloc(arr, st, n))


def pic_diag(run: int, what: int = PIC_DIAG_ALL) -> dict:
    o = pic_diag_out()
    _check(lib().pic_diag(ctypes.c_void_p(run), what, ctypes.byref(o)))
    return {n: getattr(o, n) for n, _ in pic_diag_out._fields_}


def pic_particle_count(run: int):
    s, l = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().pic_particle_count(ctypes.c_void_p(run), ctypes.byref(s), ctypes.byref(l)))
    return int(s.value), int(l.value)


def pic_read_particles(run: int, first: int = 0, count: int | None = None) -> dict:
    if count is None:
        count = pic_particle_count(run)[0] - first
    count = max(int(count), 0)
    arr = {k: np.zeros(count) for k in ("z", "x", "y", "ux", "uy", "uz")}
    ids = np.zeros(count, dtype=np.uint32)
    n = ctypes.c_int64()
    dpp = ctypes.POINTER(ctypes.c_double)
    _check(lib().pic_read_particles(
        ctypes.c_void_p(run), int(first), count,
        *[arr[k].ctypes.data_as(dpp) for k in ("z", "x", "y", "ux", "uy", "uz")],
        ids.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), ctypes.byref(n)))
    m = int(n.value)
    out = {k: v[:m] for k, v in arr.items()}
    out["id"] = ids[:m]
    return out


def pic_read_fields(run: int, comp: int, npts: int) -> np.ndarray:
    out = np.zeros(npts)
    _check(lib().pic_read_fields(ctypes.c_void_p(run), int(comp),
                                 out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), npts))
    return out


def station_shape(params: pic_lab_params):
    """(nys, nxs): transverse samples of one station record."""
    st = max(int(params.station_stride), 1)
    return (params.ny // st if params.dims == 3 else 1), params.nx // st


def pic_read_station(run: int, params: pic_lab_params, station: int, max_samples: int | None = None):
    """(lab times[m], data[m, 6, nys, nxs], samples taken) of one station."""
    nys, nxs = station_shape(params)
    m = int(params.station_cap if max_samples is None else max_samples)
    times = np.zeros(max(m, 1))
    data = np.zeros(max(m, 1) * 6 * nys * nxs)
    n = ctypes.c_int64()
    dpp = ctypes.POINTER(ctypes.c_double)
    _check(lib().pic_read_station(ctypes.c_void_p(run), int(station), ctypes.byref(n),
                                  times.ctypes.data_as(dpp), data.ctypes.data_as(dpp), m))
    k = min(int(n.value), int(params.station_cap), m)
    return times[:k].copy(), data[:k * 6 * nys * nxs].reshape(k, 6, nys, nxs).copy(), int(n.value)


def pic_get_derived(run: int) -> dict:
    d = pic_derived()
    _check(lib().pic_get_derived(ctypes.c_void_p(run), ctypes.byref(d)))
    return {n: getattr(d, n) for n, _ in pic_derived._fields_}


def pic_set_option(run: int, opt: int, value: int):
    _check(lib().pic_set_option(ctypes.c_void_p(run), int(opt), int(value)))


def pic_free(run: int):
    _check(lib().pic_free(ctypes.c_void_p(run)))


def pic_push_bench(precision: int, pusher: int, n: int, nsteps: int, dt: float, B, Ex_ptr: int,
                   u_ptr: int, cell_ptr: int, off_ptr: int, stream: int):
    b = (ctypes.c_double * 3)(*[float(v) for v in B])
    _check(lib().pic_push_bench(int(precision), int(pusher), int(n), int(nsteps), float(dt), b,
                                ctypes.c_void_p(Ex_ptr), ctypes.c_void_p(u_ptr),
                                ctypes.c_void_p(cell_ptr), ctypes.c_void_p(off_ptr),
                                ctypes.c_void_p(stream)))


def pic_stream_bench(mode: int, src_ptr: int, dst_ptr: int, nbytes: int, stream: int):
    _check(lib().pic_stream_bench(int(mode), ctypes.c_void_p(src_ptr), ctypes.c_void_p(dst_ptr), int(nbytes),
                                  ctypes.c_void_p(stream)))


def pic_copy_bench(src_ptr: int, dst_ptr: int, nbytes: int, stream: int):
    _check(lib().pic_copy_bench(ctypes.c_void_p(src_ptr), ctypes.c_void_p(dst_ptr), int(nbytes),
                                ctypes.c_void_p(stream)))


# ------------------------------------------------------------------ convenience
class Run:
    """One boosted-frame run: a torch device buffer plus the library handle."""

    def __init__(self, cfg: dict, precision: str = "fp32", continuity: bool = False,
                 device: str = "cuda:0", stream=None, graph: bool = True):
        import torch

        lib()
        self.cfg = dict(cfg)
        self.params = make_params(cfg, precision, continuity)
        self.nbytes = pic_state_bytes(self.params)
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=device)
        # a stream of its own (default priority): the legacy null stream
        # cannot be captured into a HIP graph
        self.stream = stream if stream is not None else torch.cuda.Stream(self.buf.device)
        self.handle = pic_init_boosted(self.params, self.buf.data_ptr(), self.nbytes,
                                       self.stream.cuda_stream)
        if not graph:
            pic_set_option(self.handle, PIC_OPT_GRAPH, 0)
        self.derived = pic_get_derived(self.handle)
        ny = self.params.ny if self.params.dims == 3 else 1
        self.shape = (ny, self.params.nx, self.derived["nzf"])
        self.npts = int(np.prod(self.shape))

    def step(self, n: int = 1):
        pic_step(self.handle, n)

    def diag(self, what: int = PIC_DIAG_ALL) -> dict:
        return pic_diag(self.handle, what)

    def particles(self, first: int = 0, count: int | None = None) -> dict:
        return pic_read_particles(self.handle, first, count)

    def field(self, comp: int) -> np.ndarray:
        return pic_read_fields(self.handle, comp, self.npts).reshape(self.shape)

    def station(self, q: int, max_samples: int | None = None):
        return pic_read_station(self.handle, self.params, q, max_samples)

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if self.handle:
            self.stream.synchronize()
            pic_free(self.handle)
            self.handle = None
        self.buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
