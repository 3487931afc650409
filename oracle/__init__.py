"""CPU oracle for the multifrontal barrier recursions (TEST INFRASTRUCTURE).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg
may import this package.  The GPU library never does; the two share no
code.  The arithmetic lives in ``mf_oracle.c`` (plain C, double precision,
scalar column-by-column algorithms of the paper); this module only loads
it and marshals numpy arrays.

Functions (all values float64 in the CCS order of the pattern):

* ``factor(pat, x) -> ldl``            Algorithm 3.1 (D on the diagonal slots,
                                       L strictly below)
* ``logdet(pat, ldl) -> float``         log det X (f(X) = -logdet)
* ``product(pat, ldl) -> x``            Algorithm 3.2
* ``projinv(pat, ldl) -> s``            Algorithm 4.1, S = P(X^-1)
* ``completion(pat, s) -> ldl``         Algorithm 4.2 (factor of X-hat)
* ``completion_factored(pat, s, with_r=False)``  Algorithm 4.3: the same
                                       factor, computed with the update
                                       matrices held as V_j = R_j R_j^T;
                                       with_r also returns every R_j
* ``hessian(pat, ldl, s, y) -> t``      Algorithm 5.1
* ``inv_hessian(pat, ldl, s, t) -> y``  Algorithm 5.2
* ``hessian_factor(pat, ldl, s, y)``    Algorithm 5.3 (W = R(Y))
* ``hessian_factor_adj(pat, ldl, s, w)`` Algorithm 5.4 (T = R^adj(W))
* ``etree(pat) -> (parent, degree)``

``pat`` is ``(n, colptr, rowind)``.  Errors raise ``OracleError`` with the
code and, for pivot failures, the failing column.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libmforacle.so")
_SRC = os.path.join(_HERE, "mf_oracle.c")
_LIB = None
_LOCK = threading.Lock()

CODES = {0: "OK", 1: "EINVAL", 2: "ENOTCHORDAL", 3: "ENOTPD", 4: "ENOCOMPLETION", 5: "ENOMEM"}


class OracleError(RuntimeError):
    def __init__(self, code, bad=-1):
        self.code = CODES.get(code, str(code))
        self.bad = bad
        super().__init__(f"oracle error {self.code} (column {bad})")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no FMA contraction)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", _SO, _SRC, "-lm"])
    return _SO


def _lib():
    global _LIB
    with _LOCK:
        if _LIB is None:
            if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
                build()
            lib = ctypes.CDLL(_SO)
            P = ctypes.c_void_p
            I64 = ctypes.c_int64
            for name, args in {
                "orc_factor": [I64, P, P, P, P, P],
                "orc_logdet": [I64, P, P, P],
                "orc_product": [I64, P, P, P, P],
                "orc_projinv": [I64, P, P, P, P],
                "orc_completion": [I64, P, P, P, P, P],
                "orc_completion_factored": [I64, P, P, P, P, P, P],
                "orc_hessian": [I64, P, P, P, P, P, P],
                "orc_inv_hessian": [I64, P, P, P, P, P, P],
                "orc_hessian_factor": [I64, P, P, P, P, P, P],
                "orc_hessian_factor_adj": [I64, P, P, P, P, P, P],
                "orc_etree": [I64, P, P, P, P],
            }.items():
                f = getattr(lib, name)
                f.argtypes = args
                f.restype = ctypes.c_int
            _LIB = lib
    return _LIB


def _pat(pat):
    n, cp, ri = pat
    cp = np.ascontiguousarray(cp, dtype=np.int64)
    ri = np.ascontiguousarray(ri, dtype=np.int32)
    return int(n), cp, ri


def _vec(v, nnz):
    v = np.ascontiguousarray(v, dtype=np.float64)
    if v.shape != (nnz,):
        raise ValueError(f"expected {nnz} values, got {v.shape}")
    return v


def _check(rc, bad=None):
    if rc != 0:
        raise OracleError(rc, int(bad.value) if bad is not None else -1)


def factor(pat, x):
    n, cp, ri = _pat(pat)
    x = _vec(x, cp[-1])
    out = np.empty_like(x)
    bad = ctypes.c_int64(-1)
    _check(_lib().orc_factor(n, cp.ctypes.data, ri.ctypes.data, x.ctypes.data, out.ctypes.data,
                             ctypes.addressof(bad)), bad)
    return out


def logdet(pat, ldl):
    n, cp, ri = _pat(pat)
    ldl = _vec(ldl, cp[-1])
    out = ctypes.c_double(0.0)
    _check(_lib().orc_logdet(n, cp.ctypes.data, ldl.ctypes.data, ctypes.addressof(out)))
    return out.value


def product(pat, ldl):
    n, cp, ri = _pat(pat)
    ldl = _vec(ldl, cp[-1])
    out = np.empty_like(ldl)
    _check(_lib().orc_product(n, cp.ctypes.data, ri.ctypes.data, ldl.ctypes.data, out.ctypes.data))
    return out


def projinv(pat, ldl):
    n, cp, ri = _pat(pat)
    ldl = _vec(ldl, cp[-1])
    out = np.empty_like(ldl)
    _check(_lib().orc_projinv(n, cp.ctypes.data, ri.ctypes.data, ldl.ctypes.data, out.ctypes.data))
    return out


def completion(pat, s):
    n, cp, ri = _pat(pat)
    s = _vec(s, cp[-1])
    out = np.empty_like(s)
    bad = ctypes.c_int64(-1)
    _check(_lib().orc_completion(n, cp.ctypes.data, ri.ctypes.data, s.ctypes.data, out.ctypes.data,
                                 ctypes.addressof(bad)), bad)
    return out


def completion_factored(pat, s, with_r=False):
    """Algorithm 4.3.  Returns ldl, or (ldl, r) with r[j] the upper
    triangular R_j (|I_j| x |I_j|, positive diagonal), V_j = R_j R_j^T."""
    n, cp, ri = _pat(pat)
    s = _vec(s, cp[-1])
    out = np.empty_like(s)
    mi = np.diff(cp) - 1
    roff = np.concatenate([[0], np.cumsum(mi * (mi + 1) // 2)])
    rbuf = np.zeros(max(1, int(roff[-1])), dtype=np.float64) if with_r else None
    bad = ctypes.c_int64(-1)
    _check(_lib().orc_completion_factored(n, cp.ctypes.data, ri.ctypes.data, s.ctypes.data, out.ctypes.data,
                                          rbuf.ctypes.data if with_r else None, ctypes.addressof(bad)), bad)
    if not with_r:
        return out
    rs = []
    for j in range(n):
        m = int(mi[j])
        r = np.zeros((m, m))
        r[np.triu_indices(m)] = rbuf[roff[j]:roff[j + 1]]
        rs.append(r)
    return out, rs


def _three(fn, pat, ldl, s, v):
    n, cp, ri = _pat(pat)
    nnz = cp[-1]
    ldl, s, v = _vec(ldl, nnz), _vec(s, nnz), _vec(v, nnz)
    out = np.empty_like(v)
    _check(fn(n, cp.ctypes.data, ri.ctypes.data, ldl.ctypes.data, s.ctypes.data, v.ctypes.data,
              out.ctypes.data))
    return out


def hessian(pat, ldl, s, y):
    return _three(_lib().orc_hessian, pat, ldl, s, y)


def inv_hessian(pat, ldl, s, t):
    return _three(_lib().orc_inv_hessian, pat, ldl, s, t)


def hessian_factor(pat, ldl, s, y):
    return _three(_lib().orc_hessian_factor, pat, ldl, s, y)


def hessian_factor_adj(pat, ldl, s, w):
    return _three(_lib().orc_hessian_factor_adj, pat, ldl, s, w)


def etree(pat):
    n, cp, ri = _pat(pat)
    parent = np.empty(n, dtype=np.int64)
    degree = np.empty(n, dtype=np.int64)
    _check(_lib().orc_etree(n, cp.ctypes.data, ri.ctypes.data, parent.ctypes.data,
                            degree.ctypes.data))
    return parent, degree
