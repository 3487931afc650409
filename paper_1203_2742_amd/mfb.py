"""Python binding of the C ABI in include/mfb.h (argument marshalling only).

Every numeric step runs in the HIP kernels of libmfb.so.  If the library is
missing this module raises at import time; there is no CPU fallback.

Functions carry the C names without the ``mfb_`` prefix and take torch
tensors (device memory, streams) where the C ABI takes device pointers:

    plan = plan_symbolic(n, colptr, rowind)            # host numpy/torch arrays
    info = plan_info(plan)
    f = factor_create(plan, workspace)                 # uint8 cuda tensor
    factor(f, x); logdet(f, out); projected_inverse(f, s)
    hessian(f, y, t, arena); inv_hessian(f, t, y, arena)
    completion(f, s); cholesky_product(f, x); factor_export_ldl(f, ldl)
    get_status(f) -> (code, bad_column)

``SparseBarrier`` bundles a plan, a factor handle and their device buffers.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmfb.so")
HEADER_PATH = os.path.join(_HERE, "..", "include", "mfb.h")

OK, EINVAL, ENOTCHORDAL, ENOTPD, ENOCOMPLETION, ENOMEM, EHIP, ESTATE, ESCRATCH = range(9)
NAMES = {0: "OK", 1: "EINVAL", 2: "ENOTCHORDAL", 3: "ENOTPD", 4: "ENOCOMPLETION",
         5: "ENOMEM", 6: "EHIP", 7: "ESTATE", 8: "ESCRATCH"}
STATIC_SCRATCH_BYTES = 256 << 20
PLAN_TIE_LAST = 1
PLAN_NO_GATHER_MAP = 2
PLAN_WIDE_LOW = 4


class MfbError(RuntimeError):
    def __init__(self, code: int, where: str = ""):
        self.code = int(code)
        self.name = NAMES.get(self.code, str(code))
        super().__init__(f"{where}: {self.name}" if where else self.name)


KERNELS = ("k_factor", "k_projinv", "k_hess_up", "k_hess_down", "k_ihess_down", "k_ihess_up",
           "k_completion", "k_vinv", "k_product", "k_gather", "k_gamma", "k_hfactor", "k_hfactor_adj",
           "k_bigv")


class ProfileEntry(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("level", ctypes.c_int32), ("nsuper", ctypes.c_int32),
                ("k", ctypes.c_int32), ("ms", ctypes.c_double), ("bytes", ctypes.c_double),
                ("flops", ctypes.c_double)]


class PlanInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in
                ("n", "nnz", "nsuper", "nlevels_up", "nlevels_down", "max_front", "max_ncols",
                 "max_nanc", "update_doubles")] + \
               [("factor_workspace_bytes", ctypes.c_size_t), ("rhs_arena_bytes", ctypes.c_size_t)] + \
               [(n, ctypes.c_double) for n in
                ("flops_factor", "flops_projinv", "flops_hessian", "flops_inv_hessian",
                 "flops_inv_hessian_x", "flops_completion", "flops_product",
                 "bytes_factor", "bytes_projinv", "bytes_hessian", "bytes_inv_hessian",
                 "bytes_completion", "bytes_product")] + \
               [("nnz_relaxed", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class PlanOpts(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("max_zero_frac", ctypes.c_double), ("wide_j", ctypes.c_int32),
                ("big_a", ctypes.c_int32)]


class StepArgs(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("logdet", ctypes.c_void_p), ("s", ctypes.c_void_p),
                ("k", ctypes.c_int32), ("y", ctypes.c_void_p), ("t", ctypes.c_void_p),
                ("t_in", ctypes.c_void_p), ("y_out", ctypes.c_void_p), ("arena", ctypes.c_void_p),
                ("arena_bytes", ctypes.c_size_t)]


STEP_FACTOR, STEP_LOGDET, STEP_PROJINV, STEP_HESSIAN, STEP_INV_HESSIAN = 1, 2, 4, 8, 16


def _load():
    # torch ships its own HIP runtime; loading it first makes the library bind
    # to that runtime instead of bringing a second one (from the system ROCm)
    # into the process, where device allocations of one runtime are not the
    # other's
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1203_2742_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "mfb_plan_symbolic": (I32, [I64, P, P, ctypes.c_uint32, ctypes.POINTER(P)]),
        "mfb_plan_symbolic_opts": (I32, [I64, P, P, ctypes.POINTER(PlanOpts), ctypes.POINTER(P)]),
        "mfb_plan_pattern": (I32, [P, P, P]),
        "mfb_plan_info": (I32, [P, ctypes.POINTER(PlanInfo)]),
        "mfb_plan_supernodes": (I32, [P, P, P, P]),
        "mfb_plan_destroy": (None, [P]),
        "mfb_factor_create": (I32, [P, P, SZ, ctypes.POINTER(P)]),
        "mfb_factor_destroy": (None, [P]),
        "mfb_factor": (I32, [P, P, P]),
        "mfb_logdet": (I32, [P, P, P]),
        "mfb_projected_inverse": (I32, [P, P, P]),
        "mfb_hessian": (I32, [P, I32, P, P, P, SZ, P]),
        "mfb_inv_hessian": (I32, [P, I32, P, P, P, SZ, P]),
        "mfb_hessian_static": (I32, [P, I32, P, P, P]),
        "mfb_hessian_factor": (I32, [P, I32, P, P, P, SZ, P]),
        "mfb_hessian_factor_adj": (I32, [P, I32, P, P, P, SZ, P]),
        "mfb_gram_arena_bytes": (SZ, [P, I32]),
        "mfb_step_graph_create": (I32, [P, ctypes.c_uint32, ctypes.POINTER(StepArgs), ctypes.POINTER(P)]),
        "mfb_graph_launch": (I32, [P, P]),
        "mfb_graph_destroy": (None, [P]),
        "mfb_gram": (I32, [P, I32, P, P, P, SZ, P]),
        "mfb_completion": (I32, [P, P, P]),
        "mfb_completion_factored": (I32, [P, P, P]),
        "mfb_inv_hessian_factored": (I32, [P, I32, P, P, P, SZ, P]),
        "mfb_cholesky_product": (I32, [P, P, P]),
        "mfb_factor_export_ldl": (I32, [P, P, P]),
        "mfb_get_status": (I32, [P, ctypes.POINTER(I64)]),
        "mfb_strerror": (ctypes.c_char_p, [I32]),
        "mfb_profile_enable": (I32, [P, I32]),
        "mfb_profile_read": (I32, [P, P, I64, ctypes.POINTER(I64)]),
        "mfb_kernel_name": (ctypes.c_char_p, [I32]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


_lib = _load()


def header_symbols():
    """Names of the functions declared in include/mfb.h."""
    text = open(HEADER_PATH).read()
    return sorted(set(re.findall(r"\b(mfb_[a-z_]+)\s*\(", text)))


def _chk(rc, where):
    if rc != 0:
        raise MfbError(rc, where)


def _stream(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _dev_f64(t, n, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 cuda tensor")
    if t.numel() < n:
        raise ValueError(f"{name} holds {t.numel()} values, needs {n}")
    return t


# --------------------------------------------------------------------- plan

class Plan:
    def __init__(self, handle, n, nnz):
        self.handle = handle
        self.n = n
        self.nnz = nnz
        self.info = plan_info(self)

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:  # the module may already be torn down at exit
            _lib.mfb_plan_destroy(h)


def plan_symbolic(n, colptr, rowind, flags: int = 0, relax=None, wide_j: int = 0, big_a: int = 0) -> Plan:
    """mfb_plan_symbolic, or mfb_plan_symbolic_opts when any option is given
    (relax: max_zero_frac of relaxed supernodes; wide_j, big_a: the two front
    thresholds, 0 for the default).  Plan.nnz is the caller's pattern's."""
    cp = np.ascontiguousarray(np.asarray(colptr), dtype=np.int64)
    ri = np.ascontiguousarray(np.asarray(rowind), dtype=np.int32)
    if cp.shape != (int(n) + 1,):
        raise MfbError(EINVAL, "plan_symbolic: colptr length")
    h = ctypes.c_void_p()
    if relax is None and not wide_j and not big_a:
        _chk(_lib.mfb_plan_symbolic(int(n), cp.ctypes.data, ri.ctypes.data, flags, ctypes.byref(h)),
             "plan_symbolic")
    else:
        o = PlanOpts(int(flags), -1.0 if relax is None else float(relax), int(wide_j), int(big_a))
        _chk(_lib.mfb_plan_symbolic_opts(int(n), cp.ctypes.data, ri.ctypes.data, ctypes.byref(o), ctypes.byref(h)),
             "plan_symbolic_opts")
    return Plan(h, int(n), int(cp[-1]) if n else 0)


def plan_pattern(plan: Plan):
    """The pattern the sweeps run on, (colptr int64[n+1], rowind int32[nnz_relaxed])."""
    cp = np.empty(plan.n + 1, np.int64)
    ri = np.empty(max(1, plan.info["nnz_relaxed"]), np.int32)
    _chk(_lib.mfb_plan_pattern(plan.handle, cp.ctypes.data, ri.ctypes.data), "plan_pattern")
    return cp, ri[:plan.info["nnz_relaxed"]]


def plan_info(plan: Plan) -> dict:
    info = PlanInfo()
    _chk(_lib.mfb_plan_info(plan.handle, ctypes.byref(info)), "plan_info")
    return info.as_dict()


def plan_supernodes(plan: Plan):
    """(snode_of[n], sparent[nsuper], srep[nsuper]) as int32 numpy arrays."""
    ns = plan.info["nsuper"]
    a = np.empty(max(plan.n, 1), np.int32)
    b = np.empty(max(ns, 1), np.int32)
    c = np.empty(max(ns, 1), np.int32)
    _chk(_lib.mfb_plan_supernodes(plan.handle, a.ctypes.data, b.ctypes.data, c.ctypes.data),
         "plan_supernodes")
    return a[:plan.n], b[:ns], c[:ns]


# ------------------------------------------------------------------- factor

class Factor:
    def __init__(self, handle, plan, workspace):
        self.handle = handle
        self.plan = plan
        self.workspace = workspace  # keep the device buffer alive

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:  # the module may already be torn down at exit
            _lib.mfb_factor_destroy(h)


def factor_create(plan: Plan, workspace) -> Factor:
    h = ctypes.c_void_p()
    _chk(_lib.mfb_factor_create(plan.handle, _ptr(workspace), workspace.numel() * workspace.element_size(),
                                ctypes.byref(h)), "factor_create")
    return Factor(h, plan, workspace)


def factor(f: Factor, x, stream=None):
    _chk(_lib.mfb_factor(f.handle, _ptr(_dev_f64(x, f.plan.nnz, "x")), _stream(stream)), "factor")


def logdet(f: Factor, out, stream=None):
    _chk(_lib.mfb_logdet(f.handle, _ptr(_dev_f64(out, 1, "out")), _stream(stream)), "logdet")


def projected_inverse(f: Factor, s=None, stream=None):
    sp = _ptr(_dev_f64(s, f.plan.nnz, "s")) if s is not None else None
    _chk(_lib.mfb_projected_inverse(f.handle, sp, _stream(stream)), "projected_inverse")


def _k_of(t, nnz):
    if nnz == 0:
        return 0
    return t.numel() // nnz


def hessian(f: Factor, y, t, arena, k=None, stream=None):
    nnz = f.plan.nnz
    k = _k_of(y, nnz) if k is None else int(k)
    _dev_f64(y, k * nnz, "y")
    _dev_f64(t, k * nnz, "t")
    _chk(_lib.mfb_hessian(f.handle, k, _ptr(y), _ptr(t), _ptr(arena),
                          arena.numel() * arena.element_size(), _stream(stream)), "hessian")


def hessian_static(f: Factor, y, t, k=None, stream=None):
    """mfb_hessian_static: the Hessian with the library's static scratch."""
    nnz = f.plan.nnz
    k = _k_of(y, nnz) if k is None else int(k)
    _dev_f64(y, k * nnz, "y")
    _dev_f64(t, k * nnz, "t")
    _chk(_lib.mfb_hessian_static(f.handle, k, _ptr(y), _ptr(t), _stream(stream)), "hessian_static")


def inv_hessian(f: Factor, t, y, arena, k=None, stream=None):
    nnz = f.plan.nnz
    k = _k_of(t, nnz) if k is None else int(k)
    _dev_f64(t, k * nnz, "t")
    _dev_f64(y, k * nnz, "y")
    _chk(_lib.mfb_inv_hessian(f.handle, k, _ptr(t), _ptr(y), _ptr(arena),
                              arena.numel() * arena.element_size(), _stream(stream)), "inv_hessian")


def hessian_factor(f: Factor, y, w, arena, k=None, stream=None):
    """mfb_hessian_factor: w_r = R(y_r) (Algorithm 5.3)."""
    nnz = f.plan.nnz
    k = _k_of(y, nnz) if k is None else int(k)
    _dev_f64(y, k * nnz, "y")
    _dev_f64(w, k * nnz, "w")
    _chk(_lib.mfb_hessian_factor(f.handle, k, _ptr(y), _ptr(w), _ptr(arena),
                                 arena.numel() * arena.element_size(), _stream(stream)), "hessian_factor")


def hessian_factor_adj(f: Factor, w, t, arena, k=None, stream=None):
    """mfb_hessian_factor_adj: t_r = R^adj(w_r) (Algorithm 5.4)."""
    nnz = f.plan.nnz
    k = _k_of(w, nnz) if k is None else int(k)
    _dev_f64(w, k * nnz, "w")
    _dev_f64(t, k * nnz, "t")
    _chk(_lib.mfb_hessian_factor_adj(f.handle, k, _ptr(w), _ptr(t), _ptr(arena),
                                     arena.numel() * arena.element_size(), _stream(stream)),
         "hessian_factor_adj")


def gram_arena_bytes(plan: Plan, m):
    return int(_lib.mfb_gram_arena_bytes(plan.handle, int(m)))


def gram(plan: Plan, w, g, arena, m=None, stream=None):
    """mfb_gram: g(i, j) = w_i . w_j (trace inner product on S^n_V)."""
    m = _k_of(w, plan.nnz) if m is None else int(m)
    _dev_f64(w, m * plan.nnz, "w")
    _dev_f64(g, m * m, "g")
    _chk(_lib.mfb_gram(plan.handle, m, _ptr(w), _ptr(g), _ptr(arena),
                       arena.numel() * arena.element_size(), _stream(stream)), "gram")


class Graph:
    """A captured step (mfb_step_graph_create); keeps its buffers alive."""

    def __init__(self, handle, keep):
        self.handle = handle
        self.keep = keep

    def launch(self, stream=None):
        _chk(_lib.mfb_graph_launch(self.handle, _stream(stream)), "graph_launch")

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.mfb_graph_destroy(h)


def step_graph(f: Factor, ops, x, logdet=None, s=None, k=0, y=None, t=None, t_in=None, y_out=None,
               arena=None):
    """Capture factor(x) followed by the operations set in `ops` (STEP_*
    flags; STEP_FACTOR is required) into one replayable graph.  The buffers
    are bound at capture: a launch reads and writes these same tensors."""
    nnz = f.plan.nnz
    need = {"x": (x, nnz, STEP_FACTOR), "logdet": (logdet, 1, STEP_LOGDET), "s": (s, nnz, STEP_PROJINV),
            "y": (y, k * nnz, STEP_HESSIAN), "t": (t, k * nnz, STEP_HESSIAN),
            "t_in": (t_in, k * nnz, STEP_INV_HESSIAN), "y_out": (y_out, k * nnz, STEP_INV_HESSIAN)}
    for name, (v, n, bit) in need.items():
        if ops & bit:
            _dev_f64(v, n, name)

    def ad(v):
        return v.data_ptr() if v is not None else None
    a = StepArgs(ad(x), ad(logdet), ad(s), int(k), ad(y), ad(t), ad(t_in), ad(y_out), ad(arena),
                 arena.numel() * arena.element_size() if arena is not None else 0)
    h = ctypes.c_void_p()
    _chk(_lib.mfb_step_graph_create(f.handle, int(ops), ctypes.byref(a), ctypes.byref(h)), "step_graph_create")
    return Graph(h, (f, x, logdet, s, y, t, t_in, y_out, arena))


def completion(f: Factor, s, stream=None):
    _chk(_lib.mfb_completion(f.handle, _ptr(_dev_f64(s, f.plan.nnz, "s")), _stream(stream)),
         "completion")


def inv_hessian_factored(f: Factor, t, y, arena, k=None, stream=None):
    nnz = f.plan.nnz
    k = _k_of(t, nnz) if k is None else int(k)
    _dev_f64(t, k * nnz, "t")
    _dev_f64(y, k * nnz, "y")
    _chk(_lib.mfb_inv_hessian_factored(f.handle, k, _ptr(t), _ptr(y), _ptr(arena),
                                       arena.numel() * arena.element_size(), _stream(stream)),
         "inv_hessian_factored")


def completion_factored(f: Factor, s, stream=None):
    _chk(_lib.mfb_completion_factored(f.handle, _ptr(_dev_f64(s, f.plan.nnz, "s")), _stream(stream)),
         "completion_factored")


def cholesky_product(f: Factor, x, stream=None):
    _chk(_lib.mfb_cholesky_product(f.handle, _ptr(_dev_f64(x, f.plan.nnz, "x")), _stream(stream)),
         "cholesky_product")


def factor_export_ldl(f: Factor, ldl, stream=None):
    _chk(_lib.mfb_factor_export_ldl(f.handle, _ptr(_dev_f64(ldl, f.plan.nnz, "ldl")),
                                    _stream(stream)), "factor_export_ldl")


def get_status(f: Factor):
    bad = ctypes.c_int64(-1)
    rc = _lib.mfb_get_status(f.handle, ctypes.byref(bad))
    if rc == EHIP:
        raise MfbError(rc, "get_status")
    return rc, int(bad.value)


def strerror(code: int) -> str:
    return _lib.mfb_strerror(int(code)).decode()


def profile_enable(f: Factor, enable: bool = True):
    _chk(_lib.mfb_profile_enable(f.handle, 1 if enable else 0), "profile_enable")


def profile_read(f: Factor):
    """Recorded launches as a list of dicts (and clears the record)."""
    count = ctypes.c_int64(0)
    _chk(_lib.mfb_profile_read(f.handle, None, 0, ctypes.byref(count)), "profile_read")
    return _profile_take(f, int(count.value))


def _profile_take(f, n):
    if n == 0:
        return []
    buf = (ProfileEntry * n)()
    count = ctypes.c_int64(0)
    _chk(_lib.mfb_profile_read(f.handle, ctypes.cast(buf, ctypes.c_void_p), n, ctypes.byref(count)),
         "profile_read")
    return [{"kernel": KERNELS[e.kernel], "level": e.level, "nsuper": e.nsuper, "k": e.k,
             "ms": e.ms, "bytes": e.bytes, "flops": e.flops} for e in buf[:min(n, count.value)]]


def kernel_name(kernel: int) -> str:
    return _lib.mfb_kernel_name(int(kernel)).decode()


# ----------------------------------------------------------- convenience

class SparseBarrier:
    """A plan plus a factor handle with torch-allocated device buffers."""

    def __init__(self, pattern, device="cuda", flags=0, relax=None, wide_j=0, big_a=0):
        import torch
        n, cp, ri = pattern
        self.plan = plan_symbolic(n, cp, ri, flags, relax, wide_j, big_a)
        self.info = self.plan.info
        self.nnz = self.plan.nnz
        self.device = torch.device(device)
        self.workspace = torch.empty(self.info["factor_workspace_bytes"], dtype=torch.uint8,
                                     device=self.device)
        self.f = factor_create(self.plan, self.workspace)
        self._arena = None

    def arena(self, k):
        import torch
        need = max(1, k) * self.info["rhs_arena_bytes"]
        if self._arena is None or self._arena.numel() < need:
            self._arena = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._arena

    def _new(self, k=None):
        import torch
        shape = (self.nnz,) if k is None else (k, self.nnz)
        return torch.empty(shape, dtype=torch.float64, device=self.device)

    def factor(self, x):
        factor(self.f, x)

    def logdet(self):
        import torch
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        logdet(self.f, out)
        return out

    def projected_inverse(self):
        s = self._new()
        projected_inverse(self.f, s)
        return s

    def hessian(self, y):
        k = 1 if y.dim() == 1 else y.shape[0]
        t = torch_empty_like(y)
        hessian(self.f, y, t, self.arena(k), k=k)
        return t

    def inv_hessian(self, t):
        k = 1 if t.dim() == 1 else t.shape[0]
        y = torch_empty_like(t)
        inv_hessian(self.f, t, y, self.arena(k), k=k)
        return y

    def inv_hessian_factored(self, t):
        k = 1 if t.dim() == 1 else t.shape[0]
        y = torch_empty_like(t)
        inv_hessian_factored(self.f, t, y, self.arena(k), k=k)
        return y

    def hessian_factor(self, y):
        k = 1 if y.dim() == 1 else y.shape[0]
        w = torch_empty_like(y)
        hessian_factor(self.f, y, w, self.arena(k), k=k)
        return w

    def hessian_factor_adj(self, w):
        k = 1 if w.dim() == 1 else w.shape[0]
        t = torch_empty_like(w)
        hessian_factor_adj(self.f, w, t, self.arena(k), k=k)
        return t

    def gram(self, w):
        import torch
        m = 1 if w.dim() == 1 else w.shape[0]
        g = torch.empty((m, m), dtype=torch.float64, device=self.device)
        arena = torch.empty(max(1, gram_arena_bytes(self.f.plan, m)), dtype=torch.uint8, device=self.device)
        gram(self.f.plan, w, g, arena, m=m)
        return g

    def completion(self, s):
        completion(self.f, s)

    def completion_factored(self, s):
        completion_factored(self.f, s)

    def cholesky_product(self):
        x = self._new()
        cholesky_product(self.f, x)
        return x

    def export_ldl(self):
        ldl = self._new()
        factor_export_ldl(self.f, ldl)
        return ldl

    def status(self):
        return get_status(self.f)


def torch_empty_like(t):
    import torch
    return torch.empty_like(t, memory_format=torch.contiguous_format)
