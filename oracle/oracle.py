"""ctypes binding of the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liborc.so")
LIB_OMP = os.path.join(HERE, "liborc_omp.so")
SRC = os.path.join(HERE, "mts_oracle.c")


def build_oracle(force: bool = False, openmp: bool = False) -> str:
    """Compile the oracle with plain gcc, FP contraction off.  openmp: the same
    source with its per-node loops of the PD substep spread over threads
    (identical results; used only to time the oracle on all host cores)."""
    lib = LIB_OMP if openmp else LIB
    if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(SRC):
        extra = ["-fopenmp"] if openmp else []
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", *extra,
                               "-shared", "-o", lib + ".tmp", SRC, "-lm"])
        os.replace(lib + ".tmp", lib)
    return lib


class _Problem(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("mode", C.c_int32), ("breaking", C.c_int32),
        ("weight_kind", C.c_int32), ("kernel", C.c_int32), ("m", C.c_int32),
        ("n_cracks", C.c_int32), ("fe_n", C.c_int32 * 3),
        ("n_pd", C.c_int64), ("pos", C.POINTER(C.c_double)),
        ("dx", C.c_double), ("horizon_factor", C.c_double),
        ("pd_lo", C.c_double * 3), ("pd_hi", C.c_double * 3),
        ("dom_lo", C.c_double * 3), ("dom_hi", C.c_double * 3),
        ("fe_h", C.c_double), ("overlap", C.c_double),
        ("cracks", (C.c_double * 3) * 8),
        ("E", C.c_double), ("rho", C.c_double), ("G0", C.c_double),
        ("thickness", C.c_double), ("s_crit", C.c_double), ("l_over_delta", C.c_double),
        ("traction", C.c_double), ("vel_bc", C.c_double), ("dt_pd", C.c_double),
        ("setup_only", C.c_int32),
        ("fe_beta", C.c_double),
        ("traction_x", C.c_double),
        ("clamp_x0", C.c_int32),
        ("pd_beta", C.c_double),
    ]


class _Info(C.Structure):
    _fields_ = [
        ("delta", C.c_double), ("volume", C.c_double), ("c0", C.c_double),
        ("s_crit", C.c_double), ("nu", C.c_double), ("dt_pd", C.c_double), ("dt_fe", C.c_double),
        ("n_pd", C.c_int64), ("nnz", C.c_int64), ("n_fe_nodes", C.c_int64),
        ("n_fe_elems", C.c_int64), ("n_constraints", C.c_int64), ("n_region", C.c_int64),
        ("pd_steps", C.c_int64), ("macro_steps", C.c_int64), ("n_rebuilds", C.c_int64),
        ("n_broken", C.c_int64),
        ("e_kin", C.c_double), ("e_pd", C.c_double), ("e_fe", C.c_double), ("w_ext", C.c_double),
    ]


PD_U, PD_V, PD_A, FE_U, FE_V, FE_A, DAMAGE, LAMBDA, PD_ALPHA, PD_MASS, FE_MASS, FE_X, H, \
    CONSTRAINT_NODES, FE_P, PD_P, GF, REGION, GF_NODES = range(19)

_libs = {}


def _L(openmp: bool = False):
    if openmp not in _libs:
        _lib = C.CDLL(build_oracle(openmp=openmp))
        P = C.POINTER
        _lib.orc_create.restype = C.c_void_p
        _lib.orc_create.argtypes = [P(_Problem)]
        _lib.orc_destroy.argtypes = [C.c_void_p]
        _lib.orc_advance.argtypes = [C.c_void_p, C.c_int64]
        _lib.orc_info_get.argtypes = [C.c_void_p, P(_Info)]
        _lib.orc_get.restype = C.c_int64
        _lib.orc_get.argtypes = [C.c_void_p, C.c_int, P(C.c_double), C.c_int64]
        _lib.orc_set.argtypes = [C.c_void_p, C.c_int, P(C.c_double), C.c_int64]
        _lib.orc_get_bonds.restype = C.c_int64
        _lib.orc_get_bonds.argtypes = [C.c_void_p, P(C.c_int64), P(C.c_int32), P(C.c_uint8), C.c_int64]
        _lib.orc_pd_force.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double)]
        _lib.orc_pd_energy.restype = C.c_double
        _lib.orc_pd_energy.argtypes = [C.c_void_p, P(C.c_double)]
        _lib.orc_fe_force.argtypes = [C.c_void_p, P(C.c_double), P(C.c_double)]
        _lib.orc_constraint_residual.argtypes = [C.c_void_p, P(C.c_double)]
        _lib.orc_dt_bound.restype = C.c_double
        _lib.orc_dt_bound.argtypes = [C.c_void_p, C.c_int]
        _lib.orc_last_error.restype = C.c_char_p
        for fn in ("orc_neighbors_brute", "orc_neighbors_grid"):
            f = getattr(_lib, fn)
            f.restype = C.c_int64
            f.argtypes = [C.c_int, C.c_int64, P(C.c_double), C.c_double, P(C.c_int64),
                          P(C.c_int32), C.c_int64]
        _lib.orc_exp_moment.restype = C.c_double
        _lib.orc_exp_moment.argtypes = [C.c_int, C.c_double, C.c_double]
        _libs[openmp] = _lib
    return _libs[openmp]


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _nb(fn, pos, delta):
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    n, dim = pos.shape
    cap = max(16, n * 64 if dim == 2 else n * 160)
    rp = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(cap, dtype=np.int32)
    nnz = fn(dim, n, _dp(pos), delta, rp.ctypes.data_as(C.POINTER(C.c_int64)),
             col.ctypes.data_as(C.POINTER(C.c_int32)), cap)
    if nnz < 0:
        raise RuntimeError("neighbour capacity exceeded")
    return rp, col[:nnz].copy()


def neighbors_brute(pos, delta):
    return _nb(_L().orc_neighbors_brute, pos, delta)


def neighbors_grid(pos, delta):
    return _nb(_L().orc_neighbors_grid, pos, delta)


def exp_moment(n, delta, l):
    return _L().orc_exp_moment(n, delta, l)


_MODE = {"coupled": 0, "pure_pd": 1, "pure_fe": 2}
_WEIGHT = {"cubic": 0, "linear": 1, "constant": 2}
_KERNEL = {"pmb": 0, "exp": 1}


def make_problem(inst: dict, setup_only: bool = False):
    pos = np.ascontiguousarray(inst["pos"], dtype=np.float64)
    p = _Problem()
    dim = int(inst["dim"])
    p.dim = dim
    p.mode = _MODE[inst.get("mode", "coupled")]
    p.breaking = 1 if inst.get("breaking", True) else 0
    p.weight_kind = _WEIGHT[inst.get("weight", "cubic")]
    p.kernel = _KERNEL[inst.get("kernel", "pmb")]
    p.m = int(inst["m"])
    cr = inst.get("cracks", [])
    p.n_cracks = len(cr)
    for i, c in enumerate(cr):
        for j in range(3):
            p.cracks[i][j] = float(c[j])
    fe_n = inst.get("fe_n", (0, 0, 0))
    for a in range(3):
        p.fe_n[a] = int(fe_n[a]) if a < len(fe_n) else 0
    p.n_pd = pos.shape[0]
    p.pos = _dp(pos)
    p.dx = float(inst["dx"])
    p.horizon_factor = float(inst.get("horizon_factor", 3.015))
    for name in ("pd_lo", "pd_hi", "dom_lo", "dom_hi"):
        arr = getattr(p, name)
        v = inst[name]
        for a in range(dim):
            arr[a] = float(v[a])
    p.fe_h = float(inst.get("fe_h", 0.0))
    p.overlap = float(inst.get("overlap", 0.0))
    for k in ("E", "rho", "G0", "thickness", "l_over_delta", "traction", "vel_bc", "dt_pd"):
        setattr(p, k, float(inst.get(k, 0.0)))
    p.s_crit = float(inst.get("s_crit", 0.0))
    p.setup_only = 1 if setup_only else 0
    p.fe_beta = float(inst.get("fe_beta", 0.0))
    p.traction_x = float(inst.get("traction_x", 0.0))
    p.clamp_x0 = 1 if inst.get("clamp_x0", False) else 0
    p.pd_beta = float(inst.get("pd_beta", 0.0))
    return p, pos


class Oracle:
    """One oracle solve of an instance dict (from mts_inputs)."""

    def __init__(self, inst: dict, setup_only: bool = False, openmp: bool = False):
        """setup_only: build weights, masses, FE mesh and the constraint set but
        not the unit-load responses (for checks of large runs); cannot advance.
        openmp: run on the OpenMP build (threads from OMP_NUM_THREADS)."""
        self.lib = _L(openmp)
        self.inst = inst
        self._p, self._pos = make_problem(inst, setup_only)
        self.h = self.lib.orc_create(C.byref(self._p))
        if not self.h:
            raise RuntimeError("oracle create failed: " + self.lib.orc_last_error().decode())
        self.dim = int(inst["dim"])

    def close(self):
        if self.h:
            self.lib.orc_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def info(self) -> dict:
        o = _Info()
        self.lib.orc_info_get(self.h, C.byref(o))
        return {k: getattr(o, k) for k, _ in _Info._fields_}

    def advance(self, n: int):
        if self.lib.orc_advance(self.h, int(n)) != 0:
            raise RuntimeError("oracle advance failed: " + self.lib.orc_last_error().decode())

    def get(self, what: int) -> np.ndarray:
        info = self.info()
        n = {PD_U: info["n_pd"] * self.dim, PD_V: info["n_pd"] * self.dim,
             PD_A: info["n_pd"] * self.dim, PD_P: info["n_pd"] * self.dim,
             FE_U: info["n_fe_nodes"] * self.dim, FE_V: info["n_fe_nodes"] * self.dim,
             FE_A: info["n_fe_nodes"] * self.dim, FE_X: info["n_fe_nodes"] * self.dim,
             FE_P: info["n_fe_nodes"] * self.dim,
             DAMAGE: info["n_pd"], PD_ALPHA: info["n_pd"], PD_MASS: info["n_pd"],
             FE_MASS: info["n_fe_nodes"], LAMBDA: info["n_constraints"] * self.dim,
             H: (info["n_constraints"] * self.dim) ** 2,
             CONSTRAINT_NODES: info["n_constraints"], GF: info["n_constraints"] * (2 ** self.dim),
             REGION: info["n_pd"], GF_NODES: info["n_constraints"] * (2 ** self.dim)}[what]
        out = np.zeros(max(n, 1), dtype=np.float64)
        got = self.lib.orc_get(self.h, what, _dp(out), out.size)
        if got < 0:
            raise RuntimeError("oracle get failed")
        out = out[:got]
        if what in (PD_U, PD_V, PD_A, PD_P, FE_U, FE_V, FE_A, FE_X, FE_P, LAMBDA):
            out = out.reshape(-1, self.dim)
        if what == H:
            k = int(round(np.sqrt(got)))
            out = out.reshape(k, k)
        return out

    def set(self, what: int, arr):
        arr = np.ascontiguousarray(arr, dtype=np.float64).ravel()
        if self.lib.orc_set(self.h, what, _dp(arr), arr.size) != 0:
            raise RuntimeError("oracle set failed")

    def bonds(self):
        info = self.info()
        rp = np.zeros(info["n_pd"] + 1, dtype=np.int64)
        col = np.zeros(info["nnz"], dtype=np.int32)
        mu = np.zeros(info["nnz"], dtype=np.uint8)
        self.lib.orc_get_bonds(self.h, rp.ctypes.data_as(C.POINTER(C.c_int64)),
                               col.ctypes.data_as(C.POINTER(C.c_int32)),
                               mu.ctypes.data_as(C.POINTER(C.c_uint8)), info["nnz"])
        return rp, col, mu

    def pd_force(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        f = np.zeros_like(u)
        self.lib.orc_pd_force(self.h, _dp(u), _dp(f))
        return f

    def pd_energy(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        return self.lib.orc_pd_energy(self.h, _dp(u))

    def fe_force(self, u):
        u = np.ascontiguousarray(u, dtype=np.float64)
        f = np.zeros_like(u)
        self.lib.orc_fe_force(self.h, _dp(u), _dp(f))
        return f

    def constraint_residual(self):
        n = self.info()["n_constraints"] * self.dim
        out = np.zeros(max(n, 1))
        self.lib.orc_constraint_residual(self.h, _dp(out))
        return out[:n].reshape(-1, self.dim)

    def dt_bound(self, which: int) -> float:
        return self.lib.orc_dt_bound(self.h, which)
