"""ctypes binding of the FP64 CPU oracle (``pic_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the GPU product
path never does.  The oracle shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pic_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

BC_OPEN, BC_PERIODIC = 0, 1
VAY, BORIS = 0, 1
EX, EY, EZ, BX, BY, BZ, JX, JY, JZ = range(9)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liboracle.so."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(ctypes.Structure):
    _fields_ = [
        ("dims", ctypes.c_int), ("nz", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("dz", ctypes.c_double), ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("cfl", ctypes.c_double), ("ppc", ctypes.c_int), ("seed", ctypes.c_uint64),
        ("gamma_boost", ctypes.c_double), ("n_lab_cm3", ctypes.c_double), ("u_th", ctypes.c_double),
        ("a0", ctypes.c_double), ("lambda0_um", ctypes.c_double), ("waist", ctypes.c_double),
        ("tau_lab", ctypes.c_double), ("pol_axis", ctypes.c_int), ("bc_z", ctypes.c_int),
        ("pusher", ctypes.c_int), ("inject_every", ctypes.c_int), ("round_f32", ctypes.c_int),
        ("filter_passes", ctypes.c_int), ("filter_compensate", ctypes.c_int),
        ("n_stations", ctypes.c_int), ("station_z0", ctypes.c_double),
        ("station_dz", ctypes.c_double), ("station_stride", ctypes.c_int),
        ("station_cap", ctypes.c_int), ("laser_antenna", ctypes.c_int),
        ("antenna_z_lab", ctypes.c_double), ("antenna_t_peak", ctypes.c_double),
    ]


class Derived(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "dt", "beta_b", "gamma_b", "dminus", "dplus", "skin_um", "k0_lab", "E0_lab",
        "L_lab", "L_boost", "zc_boost", "weight", "dV")] + [
        ("reservoir", ctypes.c_int), ("nzf", ctypes.c_int)]


class DiagOut(ctypes.Structure):
    _fields_ = [("step", ctypes.c_int64), ("t", ctypes.c_double), ("U_E", ctypes.c_double),
                ("U_B", ctypes.c_double), ("Ez_max", ctypes.c_double), ("KE", ctypes.c_double),
                ("n_particles", ctypes.c_int64), ("gauss_drift", ctypes.c_double)]


_lib = None
_D = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        L.ora_create.restype = vp
        L.ora_create.argtypes = [ctypes.POINTER(Params)]
        L.ora_destroy.argtypes = [vp]
        L.ora_get_derived.argtypes = [vp, ctypes.POINTER(Derived)]
        L.ora_step.argtypes = [vp, ctypes.c_int, _D]
        L.ora_diag.argtypes = [vp, ctypes.POINTER(DiagOut)]
        L.ora_num_particles.restype = ctypes.c_int64
        L.ora_num_particles.argtypes = [vp]
        L.ora_field_points.restype = ctypes.c_int64
        L.ora_field_points.argtypes = [vp]
        L.ora_field.restype = _D
        L.ora_field.argtypes = [vp, ctypes.c_int]
        L.ora_step_index.restype = ctypes.c_int64
        L.ora_step_index.argtypes = [vp]
        L.ora_get_particles.argtypes = [vp] + [_D] * 6 + [ctypes.POINTER(ctypes.c_uint32)]
        L.ora_set_particles.argtypes = [vp, ctypes.c_int64] + [_D] * 6 + [ctypes.POINTER(ctypes.c_uint32)]
        L.ora_reset_gauss_reference.argtypes = [vp]
        L.ora_philox4x64_10.argtypes = [ctypes.POINTER(ctypes.c_uint64)] * 3
        for fn in ("ora_push_vay", "ora_push_boris"):
            getattr(L, fn).argtypes = [_D, _D, _D, ctypes.c_double]
        L.ora_boost_fields.argtypes = [ctypes.c_double, _D, _D, _D, _D]
        L.ora_boost_momentum.argtypes = [ctypes.c_double, _D, _D]
        L.ora_gather.argtypes = [vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, _D, _D]
        L.ora_deposit.argtypes = [vp, _D, _D, ctypes.c_double]
        L.ora_rho.argtypes = [vp, _D]
        L.ora_field_half_B.argtypes = [vp]
        L.ora_field_full_E.argtypes = [vp]
        L.ora_laser_lab.argtypes = [vp] + [ctypes.c_double] * 4 + [_D, _D]
        L.ora_filter_current.argtypes = [vp]
        L.ora_station.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(_D), ctypes.POINTER(_D)]
        L.ora_filter_nodes.argtypes = [vp, _D]
        L.ora_push_many.argtypes = [ctypes.c_int64, _D, _D, _D, _D, ctypes.c_double, ctypes.c_int, ctypes.c_int]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_D)


# ---------------------------------------------------------------- building blocks
def philox4x64_10(ctr, key):
    c = (ctypes.c_uint64 * 4)(*[int(v) & (2**64 - 1) for v in ctr])
    k = (ctypes.c_uint64 * 2)(*[int(v) & (2**64 - 1) for v in key])
    o = (ctypes.c_uint64 * 4)()
    lib().ora_philox4x64_10(c, k, o)
    return [int(v) for v in o]


def push(u, E, B, eps, pusher=VAY):
    u = np.array(u, dtype=np.float64)
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    fn = lib().ora_push_boris if pusher == BORIS else lib().ora_push_vay
    fn(_dp(u), _dp(E), _dp(B), float(eps))
    return u


def boost_fields(beta, E, B):
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    Eo, Bo = np.zeros(3), np.zeros(3)
    lib().ora_boost_fields(float(beta), _dp(E), _dp(B), _dp(Eo), _dp(Bo))
    return Eo, Bo


def boost_momentum(beta, u):
    u = np.ascontiguousarray(u, dtype=np.float64)
    uo = np.zeros(3)
    lib().ora_boost_momentum(float(beta), _dp(u), _dp(uo))
    return uo


def push_many(u, E, B, pos, dt, nsteps, pusher=VAY):
    """Advance particles in per-particle uniform fields; arrays are (n,3)."""
    u = np.ascontiguousarray(u, dtype=np.float64).copy()
    pos = np.ascontiguousarray(pos, dtype=np.float64).copy()
    E = np.ascontiguousarray(E, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    n = u.shape[0]
    lib().ora_push_many(n, _dp(u), _dp(E), _dp(B), _dp(pos), float(dt), int(nsteps), int(pusher))
    return u, pos


# ---------------------------------------------------------------- full state
def make_params(cfg: dict, round_f32: bool = False) -> Params:
    """Build oracle parameters from a workload description (a plain dict)."""
    p = Params()
    p.dims = int(cfg["dims"]); p.nz = int(cfg["nz"]); p.nx = int(cfg["nx"])
    p.ny = int(cfg.get("ny", 1)); p.dz = float(cfg["dz"]); p.dx = float(cfg["dx"])
    p.dy = float(cfg.get("dy", cfg["dx"])); p.cfl = float(cfg["cfl"]); p.ppc = int(cfg["ppc"])
    p.seed = int(cfg["seed"]); p.gamma_boost = float(cfg["gamma_boost"])
    p.n_lab_cm3 = float(cfg["n_lab_cm3"]); p.u_th = float(cfg["u_th"]); p.a0 = float(cfg["a0"])
    p.lambda0_um = float(cfg["lambda0_um"]); p.waist = float(cfg["waist"])
    p.tau_lab = float(cfg.get("tau_lab", 0.0)); p.pol_axis = int(cfg["pol_axis"])
    p.bc_z = BC_PERIODIC if cfg.get("bc_z", "open") == "periodic" else BC_OPEN
    p.pusher = BORIS if cfg.get("pusher", "vay") == "boris" else VAY
    p.inject_every = int(cfg.get("sort_every", 20)); p.round_f32 = 1 if round_f32 else 0
    p.filter_passes = int(cfg.get("filter_passes", 0))
    p.filter_compensate = int(cfg.get("filter_compensate", 0))
    p.n_stations = int(cfg.get("n_stations", 0))
    p.station_z0 = float(cfg.get("station_z0", 0.0)); p.station_dz = float(cfg.get("station_dz", 0.0))
    p.station_stride = int(cfg.get("station_stride", 1)); p.station_cap = int(cfg.get("station_cap", 0))
    p.laser_antenna = int(cfg.get("laser_antenna", 0))
    p.antenna_z_lab = float(cfg.get("antenna_z_lab", 0.0))
    p.antenna_t_peak = float(cfg.get("antenna_t_peak", 0.0))
    return p


class State:
    """Owning wrapper around an oracle state."""

    def __init__(self, cfg: dict, round_f32: bool = False):
        self.cfg = dict(cfg)
        self.params = make_params(cfg, round_f32)
        self._h = lib().ora_create(ctypes.byref(self.params))
        if not self._h:
            raise RuntimeError("ora_create failed")
        d = Derived()
        lib().ora_get_derived(self._h, ctypes.byref(d))
        self.derived = {n: getattr(d, n) for n, _ in Derived._fields_}

    def close(self):
        if self._h:
            lib().ora_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def step_index(self) -> int:
        return int(lib().ora_step_index(self._h))

    def step(self, n: int = 1, check_continuity: bool = False):
        if check_continuity:
            c = ctypes.c_double(0.0)
            lib().ora_step(self._h, int(n), ctypes.byref(c))
            return c.value
        lib().ora_step(self._h, int(n), None)
        return None

    def diag(self) -> dict:
        o = DiagOut()
        lib().ora_diag(self._h, ctypes.byref(o))
        return {n: getattr(o, n) for n, _ in DiagOut._fields_}

    @property
    def shape(self):
        nzf = self.derived["nzf"]
        return (self.params.ny, self.params.nx, nzf)

    def field(self, comp: int) -> np.ndarray:
        """Writable view of a field component, shape (ny, nx, nzf)."""
        ptr = lib().ora_field(self._h, int(comp))
        n = int(lib().ora_field_points(self._h))
        return np.ctypeslib.as_array(ptr, shape=(n,)).reshape(self.shape)

    def particles(self) -> dict:
        n = int(lib().ora_num_particles(self._h))
        arr = {k: np.zeros(n) for k in ("z", "x", "y", "ux", "uy", "uz")}
        ids = np.zeros(n, dtype=np.uint32)
        lib().ora_get_particles(self._h, *[_dp(arr[k]) for k in ("z", "x", "y", "ux", "uy", "uz")],
                                ids.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))
        arr["id"] = ids
        return arr

    def set_particles(self, z, x, y, ux, uy, uz, ids=None):
        cols = [np.ascontiguousarray(a, dtype=np.float64) for a in (z, x, y, ux, uy, uz)]
        n = cols[0].shape[0]
        ids = np.arange(n, dtype=np.uint32) if ids is None else np.ascontiguousarray(ids, dtype=np.uint32)
        lib().ora_set_particles(self._h, n, *[_dp(a) for a in cols],
                                ids.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)))

    def reset_gauss_reference(self):
        lib().ora_reset_gauss_reference(self._h)

    def gather(self, z, x, y=0.0):
        E, B = np.zeros(3), np.zeros(3)
        lib().ora_gather(self._h, float(z), float(x), float(y), _dp(E), _dp(B))
        return E, B

    def deposit(self, p0, p1, vy=0.0):
        a = np.ascontiguousarray(p0, dtype=np.float64)
        b = np.ascontiguousarray(p1, dtype=np.float64)
        lib().ora_deposit(self._h, _dp(a), _dp(b), float(vy))

    def rho(self) -> np.ndarray:
        out = np.zeros(int(lib().ora_field_points(self._h)))
        lib().ora_rho(self._h, _dp(out))
        return out.reshape(self.shape)

    def half_B(self):
        lib().ora_field_half_B(self._h)

    def full_E(self):
        lib().ora_field_full_E(self._h)

    def station(self, q: int):
        """(lab times, data[sample, comp, ny/stride, nx/stride], samples taken)"""
        n = ctypes.c_int64()
        t, d = _D(), _D()
        lib().ora_station(self._h, int(q), ctypes.byref(n), ctypes.byref(t), ctypes.byref(d))
        p = self.params
        st = max(p.station_stride, 1)
        nys, nxs = (p.ny // st if p.dims == 3 else 1), p.nx // st
        m = min(int(n.value), p.station_cap)
        times = np.ctypeslib.as_array(t, shape=(max(p.station_cap, 1),))[:m].copy()
        data = np.ctypeslib.as_array(d, shape=(max(p.station_cap, 1) * 6 * nys * nxs,))
        data = data[:m * 6 * nys * nxs].reshape(m, 6, nys, nxs).copy()
        return times, data, int(n.value)

    def filter_current(self):
        lib().ora_filter_current(self._h)

    def filter_nodes(self, a: np.ndarray) -> np.ndarray:
        out = np.ascontiguousarray(a, dtype=np.float64).reshape(-1).copy()
        lib().ora_filter_nodes(self._h, _dp(out))
        return out.reshape(self.shape)

    def laser_lab(self, z, t, x, y=0.0):
        E, B = np.zeros(3), np.zeros(3)
        lib().ora_laser_lab(self._h, float(z), float(t), float(x), float(y), _dp(E), _dp(B))
        return E, B
