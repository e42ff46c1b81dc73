"""ctypes binding of libmtspd (the C-ABI in include/mtspd.h).  Argument
marshalling only: every step of the solver runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmtspd.so")

OK, EINVAL, ENOMEM, EDEVICE, EUNSTABLE, EAGAIN, ETOOBIG, ESTATE = range(8)
COUPLED, PURE_PD = 0, 1
FP64, MIXED = 0, 1
PD_U, PD_V, PD_A, FE_U, FE_V, FE_A, DAMAGE, LAMBDA, PD_ALPHA, PD_MASS, FE_MASS, FE_X, \
    CONSTRAINT_NODES, H = range(14)
KT_PD_SUBSTEP, KT_LINK, KT_FE, KT_LAMBDA, KT_REBUILD = range(5)
REQ_ACTIVE, REQ_DONE = 1, 2
WEIGHT = {"cubic": 0, "linear": 1, "constant": 2}
KERNEL = {"pmb": 0, "exp": 1}


class MtsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"mtspd status {status}: {msg}")
        self.status = status


class Problem(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("mode", C.c_int32), ("precision", C.c_int32), ("breaking", C.c_int32),
        ("weight_kind", C.c_int32), ("kernel", C.c_int32), ("m", C.c_int32), ("n_cracks", C.c_int32),
        ("fe_n", C.c_int32 * 3), ("n_pd", C.c_int64), ("host_pd_pos", C.POINTER(C.c_double)),
        ("dx", C.c_double), ("horizon_factor", C.c_double),
        ("pd_lo", C.c_double * 3), ("pd_hi", C.c_double * 3),
        ("dom_lo", C.c_double * 3), ("dom_hi", C.c_double * 3),
        ("fe_h", C.c_double), ("overlap", C.c_double), ("cracks", (C.c_double * 3) * 8),
        ("E", C.c_double), ("rho", C.c_double), ("G0", C.c_double), ("thickness", C.c_double),
        ("s_crit", C.c_double), ("l_over_delta", C.c_double),
        ("traction", C.c_double), ("vel_bc", C.c_double), ("dt_pd", C.c_double),
        ("fe_beta", C.c_double),
        ("traction_x", C.c_double),
        ("clamp_x0", C.c_int32),
        ("pd_beta", C.c_double),
    ]


class Info(C.Structure):
    _fields_ = [
        ("delta", C.c_double), ("volume", C.c_double), ("c0", C.c_double), ("s_crit", C.c_double),
        ("dt_pd", C.c_double), ("dt_fe", C.c_double),
        ("n_pd", C.c_int64), ("nnz", C.c_int64), ("n_fe_nodes", C.c_int64), ("n_fe_elems", C.c_int64),
        ("n_constraints", C.c_int64), ("n_region", C.c_int64),
        ("pd_steps", C.c_int64), ("macro_steps", C.c_int64), ("n_rebuilds", C.c_int64), ("n_colors", C.c_int64),
        ("device_bytes", C.c_int64), ("dim", C.c_int32), ("precision", C.c_int32),
        ("dt_bound_pd", C.c_double), ("inverse_bytes", C.c_int64),
        ("slot_bytes", C.c_double), ("n_rebuild_columns", C.c_int64),
    ]


class EnergyInfo(C.Structure):
    _fields_ = [("kinetic", C.c_double), ("strain_pd", C.c_double), ("strain_fe", C.c_double),
                ("external_work", C.c_double), ("n_broken", C.c_int64)]


class PlanInfo(C.Structure):
    _fields_ = [("n_pd", C.c_int64), ("nnz_estimate", C.c_int64), ("n_fe_nodes", C.c_int64),
                ("n_constraints_estimate", C.c_int64), ("device_bytes_estimate", C.c_int64)]


class PoolInfo(C.Structure):
    _fields_ = [("budget_bytes", C.c_int64), ("used_bytes", C.c_int64), ("ticks", C.c_int64),
                ("graph_captures", C.c_int64), ("graph_replays", C.c_int64),
                ("n_running", C.c_int32), ("n_ready", C.c_int32), ("max_slots", C.c_int32), ("lanes", C.c_int32)]


EXPORTS = ["mts_plan", "mts_create", "mts_create_in", "mts_advance", "mts_sync", "mts_read", "mts_read_device", "mts_write", "mts_read_bonds",
           "mts_query", "mts_energy", "mts_energy_noalloc", "mts_profile", "mts_kernel_time", "mts_destroy", "mts_status_str", "mts_last_error",
           "mts_pool_create", "mts_pool_submit", "mts_pool_step", "mts_pool_poll", "mts_pool_read",
           "mts_pool_release", "mts_pool_query", "mts_pool_destroy"]

_lib = None


def load():
    """Load the in-tree library; fail loudly if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2403_03605_amd.build`")
    try:  # torch (streams, device memory) brings the HIP runtime: load it first so there is one
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    P = C.POINTER
    lib.mts_plan.argtypes = [P(Problem), P(PlanInfo)]
    lib.mts_create.argtypes = [P(Problem), C.c_void_p, P(C.c_void_p)]
    lib.mts_create_in.argtypes = [P(Problem), C.c_void_p, C.c_int64, C.c_void_p, P(C.c_void_p)]
    lib.mts_advance.argtypes = [C.c_void_p, C.c_int64]
    lib.mts_sync.argtypes = [C.c_void_p]
    lib.mts_read.argtypes = [C.c_void_p, C.c_int32, P(C.c_double), C.c_int64, P(C.c_int64)]
    lib.mts_read_device.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_int64, P(C.c_int64)]
    lib.mts_write.argtypes = [C.c_void_p, C.c_int32, P(C.c_double), C.c_int64]
    lib.mts_read_bonds.argtypes = [C.c_void_p, P(C.c_int64), P(C.c_int32), P(C.c_uint8), C.c_int64, P(C.c_int64)]
    lib.mts_query.argtypes = [C.c_void_p, P(Info)]
    lib.mts_energy.argtypes = [C.c_void_p, P(EnergyInfo)]
    lib.mts_energy_noalloc.argtypes = [C.c_void_p, C.c_void_p]
    lib.mts_profile.argtypes = [C.c_void_p, C.c_int32]
    lib.mts_kernel_time.argtypes = [C.c_void_p, C.c_int32, P(C.c_int64), P(C.c_double)]
    lib.mts_destroy.argtypes = [C.c_void_p]
    lib.mts_destroy.restype = None
    lib.mts_status_str.restype = C.c_char_p
    lib.mts_status_str.argtypes = [C.c_int]
    lib.mts_last_error.restype = C.c_char_p
    lib.mts_pool_create.argtypes = [C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_void_p,
                                    P(C.c_void_p)]
    lib.mts_pool_submit.argtypes = [C.c_void_p, P(Problem), C.c_int64, P(C.c_uint64)]
    lib.mts_pool_step.argtypes = [C.c_void_p, P(C.c_int32), P(C.c_uint64), C.c_int32, P(C.c_int32)]
    lib.mts_pool_poll.argtypes = [C.c_void_p, C.c_uint64, P(C.c_int32), P(C.c_int64), P(Info)]
    lib.mts_pool_read.argtypes = [C.c_void_p, C.c_uint64, C.c_int32, P(C.c_double), C.c_int64, P(C.c_int64)]
    lib.mts_pool_release.argtypes = [C.c_void_p, C.c_uint64]
    lib.mts_pool_query.argtypes = [C.c_void_p, P(PoolInfo)]
    lib.mts_pool_destroy.argtypes = [C.c_void_p]
    lib.mts_pool_destroy.restype = None
    for f in ("mts_plan", "mts_create", "mts_create_in", "mts_advance", "mts_sync", "mts_read", "mts_read_device", "mts_write", "mts_read_bonds",
              "mts_query", "mts_energy", "mts_energy_noalloc", "mts_profile", "mts_kernel_time", "mts_pool_create",
              "mts_pool_submit",
              "mts_pool_step", "mts_pool_poll", "mts_pool_read", "mts_pool_release", "mts_pool_query"):
        getattr(lib, f).restype = C.c_int
    _lib = lib
    return lib


def _check(st):
    if st != OK:
        raise MtsError(st, _lib.mts_last_error().decode(errors="replace"))


def make_problem(inst: dict):
    """Marshal an instance dict (mts_inputs) into the C struct."""
    pos = np.ascontiguousarray(inst["pos"], dtype=np.float64)
    p = Problem()
    dim = int(inst["dim"])
    p.dim = dim
    p.mode = PURE_PD if inst.get("mode", "coupled") == "pure_pd" else COUPLED
    p.precision = MIXED if inst.get("precision", "fp64") == "mixed" else FP64
    p.breaking = 1 if inst.get("breaking", True) else 0
    p.weight_kind = WEIGHT[inst.get("weight", "cubic")]
    p.kernel = KERNEL[inst.get("kernel", "pmb")]
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
    p.host_pd_pos = pos.ctypes.data_as(C.POINTER(C.c_double))
    p.dx = float(inst["dx"])
    p.horizon_factor = float(inst.get("horizon_factor", 3.015))
    for name in ("pd_lo", "pd_hi", "dom_lo", "dom_hi"):
        arr = getattr(p, name)
        for a in range(min(dim, 3, len(inst[name]))):
            arr[a] = float(inst[name][a])
    p.fe_h = float(inst.get("fe_h", 0.0))
    p.overlap = float(inst.get("overlap", 0.0))
    for k in ("E", "rho", "G0", "thickness", "l_over_delta", "traction", "vel_bc", "dt_pd", "fe_beta"):
        setattr(p, k, float(inst.get(k, 0.0)))
    p.s_crit = float(inst.get("s_crit", 0.0))
    p.traction_x = float(inst.get("traction_x", 0.0))
    p.clamp_x0 = 1 if inst.get("clamp_x0", False) else 0
    p.pd_beta = float(inst.get("pd_beta", 0.0))
    return p, pos


def plan(inst: dict) -> dict:
    lib = load()
    p, _pos = make_problem(inst)
    out = PlanInfo()
    _check(lib.mts_plan(C.byref(p), C.byref(out)))
    return {k: getattr(out, k) for k, _ in PlanInfo._fields_}


def _sizes(info, what):
    d = info["dim"]
    return {PD_U: info["n_pd"] * d, PD_V: info["n_pd"] * d, PD_A: info["n_pd"] * d,
            FE_U: info["n_fe_nodes"] * d, FE_V: info["n_fe_nodes"] * d, FE_A: info["n_fe_nodes"] * d,
            FE_X: info["n_fe_nodes"] * d, DAMAGE: info["n_pd"], PD_ALPHA: info["n_pd"], PD_MASS: info["n_pd"],
            FE_MASS: info["n_fe_nodes"], LAMBDA: info["n_constraints"] * d,
            CONSTRAINT_NODES: info["n_constraints"], H: (info["n_constraints"] * d) ** 2}[what]


class Solver:
    """One solver instance (mts_create ... mts_destroy)."""

    def __init__(self, inst: dict, stream=None, arena=None):
        """arena: optional contiguous uint8 device tensor that holds all of the
        solver's device memory (mts_create_in); kept referenced until close()."""
        self.lib = load()
        p, self._pos = make_problem(inst)
        if stream is None:
            try:
                import torch
                stream = torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else 0
            except Exception:
                stream = 0
        self.stream = int(stream)
        h = C.c_void_p()
        self.arena = arena
        if arena is None:
            _check(self.lib.mts_create(C.byref(p), C.c_void_p(self.stream), C.byref(h)))
        else:
            if not arena.is_cuda or not arena.is_contiguous():
                raise ValueError("arena must be a contiguous device tensor")
            nbytes = arena.numel() * arena.element_size()
            _check(self.lib.mts_create_in(C.byref(p), C.c_void_p(arena.data_ptr()), nbytes,
                                          C.c_void_p(self.stream), C.byref(h)))
        self.h = h
        self.dim = int(inst["dim"])

    def close(self):
        if getattr(self, "h", None):
            self.lib.mts_destroy(self.h)
            self.h = None
        self.arena = None

    def __del__(self):
        self.close()

    def advance(self, n: int):
        _check(self.lib.mts_advance(self.h, int(n)))

    def sync(self):
        _check(self.lib.mts_sync(self.h))

    def query(self) -> dict:
        o = Info()
        _check(self.lib.mts_query(self.h, C.byref(o)))
        return {k: getattr(o, k) for k, _ in Info._fields_}

    def energy(self) -> dict:
        o = EnergyInfo()
        _check(self.lib.mts_energy(self.h, C.byref(o)))
        return {k: getattr(o, k) for k, _ in EnergyInfo._fields_}

    def energy_noalloc(self, out):
        """mts_energy_noalloc: the five energy values written into `out`, a
        float64 device tensor of at least 5 elements, on the solver's stream
        (no allocation, no wait)."""
        import torch
        if out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous() or out.numel() < 5:
            raise ValueError("out must be a contiguous float64 device tensor of >= 5 elements")
        _check(self.lib.mts_energy_noalloc(self.h, C.c_void_p(out.data_ptr())))
        return out

    def read(self, what: int) -> np.ndarray:
        info = self.query()
        n = _sizes(info, what)
        out = np.zeros(max(n, 1), dtype=np.float64)
        got = C.c_int64()
        _check(self.lib.mts_read(self.h, what, out.ctypes.data_as(C.POINTER(C.c_double)), out.size, C.byref(got)))
        out = out[:got.value]
        if what in (PD_U, PD_V, PD_A, FE_U, FE_V, FE_A, FE_X, LAMBDA):
            out = out.reshape(-1, self.dim)
        if what == H:
            k = int(round(np.sqrt(out.size)))
            out = out.reshape(k, k)
        return out

    def read_device(self, what: int, out=None):
        """The quantity written into a float64 CUDA/HIP tensor on the solver's
        stream (no host round trip); `out` is allocated when not given.  Same
        shape as read(); synchronize the solver's stream before using `out`
        on another stream."""
        import torch
        info = self.query()
        n = _sizes(info, what)
        if out is None:
            out = torch.empty(max(n, 1), dtype=torch.float64, device="cuda")
        if out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 device tensor")
        got = C.c_int64()
        _check(self.lib.mts_read_device(self.h, what, C.c_void_p(out.data_ptr()), out.numel(), C.byref(got)))
        out = out[:got.value]
        if what in (PD_U, PD_V, PD_A, FE_U, FE_V, FE_A, FE_X, LAMBDA):
            out = out.view(-1, self.dim)
        if what == H:
            k = int(round(got.value ** 0.5))
            out = out.view(k, k)
        return out

    def write(self, what: int, arr):
        a = np.ascontiguousarray(arr, dtype=np.float64).ravel()
        _check(self.lib.mts_write(self.h, what, a.ctypes.data_as(C.POINTER(C.c_double)), a.size))

    def bonds(self):
        info = self.query()
        rp = np.zeros(info["n_pd"] + 1, dtype=np.int64)
        col = np.zeros(info["nnz"], dtype=np.int32)
        mu = np.zeros(info["nnz"], dtype=np.uint8)
        nnz = C.c_int64()
        _check(self.lib.mts_read_bonds(self.h, rp.ctypes.data_as(C.POINTER(C.c_int64)),
                                       col.ctypes.data_as(C.POINTER(C.c_int32)),
                                       mu.ctypes.data_as(C.POINTER(C.c_uint8)), info["nnz"], C.byref(nnz)))
        return rp, col, mu

    def profile(self, enable: bool):
        _check(self.lib.mts_profile(self.h, 1 if enable else 0))

    def kernel_time(self, kernel: int):
        n = C.c_int64()
        ms = C.c_double()
        _check(self.lib.mts_kernel_time(self.h, kernel, C.byref(n), C.byref(ms)))
        return n.value, ms.value


class Pool:
    """Serving pool (mts_pool_*): requests of one dimension and precision,
    admitted against a device-memory budget and advanced together."""

    def __init__(self, budget_bytes: int, max_slots: int = 64, dim: int = 2, precision: str = "mixed",
                 use_graphs: bool = True, stream=None):
        self.lib = load()
        if stream is None:
            stream = 0  # the pool creates a stream of its own
        h = C.c_void_p()
        _check(self.lib.mts_pool_create(int(budget_bytes), int(max_slots), int(dim),
                                        MIXED if precision == "mixed" else FP64, 1 if use_graphs else 0,
                                        C.c_void_p(int(stream)), C.byref(h)))
        self.h = h
        self.dim = dim
        self._ids = (C.c_uint64 * 1024)()

    def close(self):
        if getattr(self, "h", None):
            self.lib.mts_pool_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def submit(self, inst: dict, n_macro: int):
        """Build the request; returns its id, or None when the pool is full now
        (EAGAIN).  Raises MtsError otherwise."""
        p, _pos = make_problem(inst)
        rid = C.c_uint64()
        st = self.lib.mts_pool_submit(self.h, C.byref(p), int(n_macro), C.byref(rid))
        if st == EAGAIN:
            return None
        _check(st)
        return rid.value

    def step(self):
        """One pool step; returns (running after it, ids of requests that finished)."""
        na, nd = C.c_int32(), C.c_int32()
        _check(self.lib.mts_pool_step(self.h, C.byref(na), self._ids, len(self._ids), C.byref(nd)))
        return na.value, [self._ids[i] for i in range(min(nd.value, len(self._ids)))]

    def poll(self, rid: int):
        """(state, macro steps enqueued, the request's query record)"""
        st, done, info = C.c_int32(), C.c_int64(), Info()
        _check(self.lib.mts_pool_poll(self.h, C.c_uint64(rid), C.byref(st), C.byref(done), C.byref(info)))
        return st.value, done.value, {k: getattr(info, k) for k, _ in Info._fields_}

    def read(self, rid: int, what: int, size: int) -> np.ndarray:
        out = np.zeros(max(size, 1), dtype=np.float64)
        got = C.c_int64()
        _check(self.lib.mts_pool_read(self.h, C.c_uint64(rid), what, out.ctypes.data_as(C.POINTER(C.c_double)),
                                      out.size, C.byref(got)))
        out = out[:got.value]
        if what in (PD_U, PD_V, PD_A, FE_U, FE_V, FE_A, FE_X, LAMBDA):
            out = out.reshape(-1, self.dim)
        return out

    def release(self, rid: int):
        _check(self.lib.mts_pool_release(self.h, C.c_uint64(rid)))

    def query(self) -> dict:
        o = PoolInfo()
        _check(self.lib.mts_pool_query(self.h, C.byref(o)))
        return {k: getattr(o, k) for k, _ in PoolInfo._fields_}
