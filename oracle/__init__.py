"""CPU oracle for radix-tree-forest inverse-CDF sampling (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``rtf_oracle.c`` (plain C, built
with gcc) through ctypes and shares nothing with the HIP library.

Every function works on numpy arrays on the host and follows the passage of
Binder & Keller (arXiv:1901.05423) named in the C source.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rtf_oracle.c")
_LIB = os.path.join(_HERE, "librtf_oracle.so")

ORC_OK, ORC_ERR_ARG, ORC_ERR_ZERO_TOTAL, ORC_ERR_VALUE = 0, 1, 2, 3
SENT = 65


def compile_oracle() -> str:
    """Build librtf_oracle.so with gcc (no fast-math, no FP contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off",
           "-fno-fast-math", "-fPIC", "-shared", "-o", _LIB, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if (not os.path.exists(_LIB)
                or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            compile_oracle()
        _lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        _lib.oracle_quantize.argtypes = [P, I64, P, P]
        _lib.oracle_prefix.argtypes = [P, I64, P]
        _lib.oracle_search.argtypes = [P, I64, P, I64, P, P]
        _lib.oracle_linear_search.argtypes = [P, I64, P, I64, P]
        _lib.oracle_forest.argtypes = [P, P, P, ctypes.c_int32, P, P, P, P]
        _lib.oracle_descend.argtypes = [P, P, P, I64, I64, I64, P, I64, P]
        _lib.oracle_levels.argtypes = [P, I64, I64, P]
        _lib.oracle_balance.argtypes = [P, P, ctypes.c_int32, P, P, P, P]
        _lib.oracle_alg1.argtypes = [P, I64, I64, ctypes.c_uint64, P, P]
        _lib.oracle_grad.argtypes = [P, I64, ctypes.c_double, P, P, I64, P]
        _lib.oracle_alias_build.argtypes = [P, I64, P, P, P]
        _lib.oracle_alias_sample.argtypes = [P, P, I64, ctypes.c_uint64, P, I64, P]
        for f in ("oracle_quantize", "oracle_search", "oracle_linear_search",
                  "oracle_forest", "oracle_levels", "oracle_alg1", "oracle_grad", "oracle_balance",
                  "oracle_alias_build"):
            getattr(_lib, f).restype = ctypes.c_int
        _lib.oracle_prefix.restype = None
        _lib.oracle_descend.restype = None
        _lib.oracle_alias_sample.restype = None
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__(f"oracle error code {code}")
        self.code = code


def quantize(v, elem_off=None):
    """Per-distribution uint32 quantisation; returns (q uint32[n], scale f64[D])."""
    v = _c(v, np.float32)
    if elem_off is None:
        elem_off = np.array([0, v.size], np.int64)
    elem_off = _c(elem_off, np.int64)
    D = elem_off.size - 1
    q = np.zeros(v.size, np.uint32)
    scale = np.zeros(D, np.float64)
    for d in range(D):
        a, b = int(elem_off[d]), int(elem_off[d + 1])
        seg_q = np.zeros(b - a, np.uint32)
        sc = np.zeros(1, np.float64)
        rc = lib().oracle_quantize(_p(v[a:b]), b - a, _p(seg_q), _p(sc))
        if rc != ORC_OK:
            raise OracleError(rc)
        q[a:b] = seg_q
        scale[d] = sc[0]
    return q, scale


def prefix(w):
    """C[0..n]: C[0] = 0, C[i+1] = C[i] + w[i] (uint64)."""
    w = _c(w, np.uint32)
    C = np.zeros(w.size + 1, np.uint64)
    lib().oracle_prefix(_p(w), w.size, _p(C))
    return C


def search(w, u, want_x=True, C=None):
    """Binary-search inverse CDF: (idx int32[S], x f64[S] or None)."""
    if C is None:
        C = prefix(w)
    C = _c(C, np.uint64)
    u = _c(u, np.uint64)
    n = C.size - 1
    idx = np.zeros(u.size, np.int32)
    x = np.zeros(u.size, np.float64) if want_x else None
    rc = lib().oracle_search(_p(C), n, _p(u), u.size, _p(idx),
                             _p(x) if want_x else None)
    if rc != ORC_OK:
        raise OracleError(rc)
    return idx, x


def linear_search(w, u):
    C = prefix(w)
    u = _c(u, np.uint64)
    idx = np.zeros(u.size, np.int32)
    rc = lib().oracle_linear_search(_p(C), C.size - 1, _p(u), u.size, _p(idx))
    if rc != ORC_OK:
        raise OracleError(rc)
    return idx


class Forest:
    """Host copy of a forest: key u64[n], child i32[n,2], table i32[m], W u64[D]."""

    def __init__(self, key, child, table, W, elem_off, cell_off):
        self.key, self.child, self.table, self.W = key, child, table, W
        self.elem_off, self.cell_off = elem_off, cell_off


def forest(w, m=None, elem_off=None, cell_off=None):
    """Reference forest from the definition (single or batched)."""
    w = _c(w, np.uint32)
    if elem_off is None:
        elem_off = np.array([0, w.size], np.int64)
        cell_off = np.array([0, int(m)], np.int64)
    elem_off = _c(elem_off, np.int64)
    cell_off = _c(cell_off, np.int64)
    D = elem_off.size - 1
    n, mt = int(elem_off[-1]), int(cell_off[-1])
    key = np.zeros(n, np.uint64)
    child = np.zeros((n, 2), np.int32)
    table = np.zeros(mt, np.int32)
    W = np.zeros(D, np.uint64)
    rc = lib().oracle_forest(_p(w), _p(elem_off), _p(cell_off), D, _p(key),
                             _p(child), _p(table), _p(W))
    if rc != ORC_OK:
        raise OracleError(rc)
    return Forest(key, child, table, W, elem_off, cell_off)


def balance(f: Forest):
    """The depth fallback (Sec. 3): a copy of f whose degenerate cell trees
    (a positive-weight leaf more than 2 ceil(log2 c) internal nodes deep in a
    cell of c leaves) are replaced by balanced ones; returns (forest, rebuilt)."""
    child = f.child.copy()
    rebuilt = np.zeros(1, np.int64)
    D = f.elem_off.size - 1
    rc = lib().oracle_balance(_p(f.elem_off), _p(f.cell_off), D, _p(f.key), _p(child),
                              _p(f.table), _p(rebuilt))
    if rc != ORC_OK:
        raise OracleError(rc)
    return Forest(f.key, child, f.table, f.W, f.elem_off, f.cell_off), int(rebuilt[0])


def descend(f: Forest, u, d=0):
    """Alg. 2 on a forest for distribution d; indices local to d."""
    u = _c(u, np.uint64)
    idx = np.zeros(u.size, np.int32)
    eo, co = int(f.elem_off[d]), int(f.cell_off[d])
    m = int(f.cell_off[d + 1]) - co
    lib().oracle_descend(_p(f.key), _p(f.child), _p(f.table), eo, co, m,
                         _p(u), u.size, _p(idx))
    return idx


def levels(w, m):
    w = _c(w, np.uint32)
    lvl = np.zeros(max(w.size - 1, 0), np.int32)
    rc = lib().oracle_levels(_p(w), w.size, int(m), _p(lvl))
    if rc != ORC_OK:
        raise OracleError(rc)
    return lvl


def alg1(w, m, seed):
    """Alg. 1 simulated under a seeded random schedule: (key, child)."""
    w = _c(w, np.uint32)
    key = np.zeros(w.size, np.uint64)
    child = np.zeros((w.size, 2), np.int32)
    rc = lib().oracle_alg1(_p(w), w.size, int(m), int(seed), _p(key), _p(child))
    if rc != ORC_OK:
        raise OracleError(rc)
    return key, child


def grad(q, scale, u, g):
    """FP64 reference dL/dv for one distribution (index held fixed)."""
    q = _c(q, np.uint32)
    u = _c(u, np.uint64)
    g = _c(g, np.float64)
    out = np.zeros(q.size, np.float64)
    rc = lib().oracle_grad(_p(q), q.size, float(scale), _p(u), _p(g), u.size,
                           _p(out))
    if rc != ORC_OK:
        raise OracleError(rc)
    return out


class Alias:
    """An alias table (Sec. 2.6): per cell j the part thr[j] of the cell's
    capacity W kept by item j, and the item alias[j] that takes the rest."""

    def __init__(self, thr, alias, W):
        self.thr, self.alias, self.W = thr, alias, int(W)


def alias_build(w):
    """Walker's alias table by Vose's two-worklist construction, in exact
    integers (item mass w_i * n, cell capacity W = sum w)."""
    w = _c(w, np.uint32)
    n = w.size
    thr = np.zeros(n, np.uint64)
    alias = np.zeros(n, np.int32)
    work = np.zeros(2 * n, np.int64)
    rc = lib().oracle_alias_build(_p(w), n, _p(thr), _p(alias), _p(work))
    if rc != ORC_OK:
        raise OracleError(rc)
    return Alias(thr, alias, int(w.astype(np.uint64).sum()))


def alias_sample(t: Alias, u):
    """Indices the alias table maps the uniforms u (uint64) to."""
    u = _c(u, np.uint64)
    idx = np.zeros(u.size, np.int32)
    lib().oracle_alias_sample(_p(t.thr), _p(t.alias), t.thr.size, t.W, _p(u), u.size, _p(idx))
    return idx


def quadratic_error(p, counts, N):
    """The quadratic error of Fig. convergence: the sum over the values i of
    (p_i - c_i / N)^2, c_i the number of the N samples that realised i."""
    p = np.asarray(p, np.float64)
    c = np.asarray(counts, np.float64)
    return float(np.sum((p - c / float(N)) ** 2))
