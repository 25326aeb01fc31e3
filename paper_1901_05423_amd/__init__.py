"""MI355X-native radix tree forests for monotone inverse-CDF sampling.

Python binding of ``librtforest.so`` (C ABI in ``include/rtforest.h``).  It only
marshals arguments: every step of the method runs in the library's HIP
kernels.  PyTorch supplies device memory and the current stream.  Importing
this package does not load the library; the first call does, and raises
``RuntimeError`` if the built library is missing (there is no CPU fallback).

Method: Binder & Keller, "Massively Parallel Construction of Radix Tree
Forests for the Efficient Sampling of Discrete or Piecewise Constant
Probability Distributions" (arXiv:1901.05423).
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librtforest.so")

RTF_OK = 0
RTF_ERR_INVALID_ARG = 1
RTF_ERR_SIZE = 2
RTF_ERR_WORKSPACE = 3
RTF_ERR_HIP = 4
RTF_ERR_ZERO_TOTAL = 5
RTF_ERR_VALUE = 6

NODE_BYTES = 16
CELL_BYTES = 64
CELL_KEYS = 7  # keys per cell record; the last int64 word holds (ref, aux)


class RtfError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        name = lib().rtf_status_string(code).decode() if _lib is not None else str(code)
        super().__init__(f"{what}: {name}" if what else name)
        self.code = code


class rtf_forest(ctypes.Structure):
    _fields_ = [
        ("D", ctypes.c_int32),
        ("tile", ctypes.c_int32),
        ("n_total", ctypes.c_int64),
        ("m_total", ctypes.c_int64),
        ("nodes", ctypes.c_void_p),
        ("cells", ctypes.c_void_p),
        ("dists", ctypes.c_void_p),
        ("elem_off", ctypes.c_void_p),
        ("cell_off", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
        ("scratch", ctypes.c_void_p),
        ("scratch_bytes", ctypes.c_size_t),
        ("wide", ctypes.c_void_p),
    ]


class rtf_alias_table(ctypes.Structure):
    _fields_ = [
        ("D", ctypes.c_int32),
        ("n_total", ctypes.c_int64),
        ("recs", ctypes.c_void_p),
        ("W", ctypes.c_void_p),
        ("elem_off", ctypes.c_void_p),
        ("status", ctypes.c_void_p),
    ]


_lib = None

# name -> (restype, argtypes)
_P, _I32, _I64, _SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
_FP = ctypes.POINTER(rtf_forest)
_AP = ctypes.POINTER(rtf_alias_table)
SIGNATURES = {
    "rtf_workspace_bytes": (_SZ, [_I64, _I64]),
    "rtf_workspace_bytes_batched": (_SZ, [_I32, _I64, _I64]),
    "rtf_build": (ctypes.c_int, [_P, _I64, _I64, _P, _SZ, _P, _FP]),
    "rtf_build_batched": (ctypes.c_int, [_P, _P, _P, _I32, _I64, _I64, _P, _SZ, _P, _FP]),
    "rtf_build_tiled": (ctypes.c_int, [_P, _I64, _I64, _I32, _P, _SZ, _P, _FP]),
    "rtf_build_batched_tiled": (ctypes.c_int, [_P, _P, _P, _I32, _I64, _I64, _I32, _P, _SZ, _P, _FP]),
    "rtf_wide_workspace_bytes": (_SZ, [_I64]),
    "rtf_forest_widen": (ctypes.c_int, [_FP, _P, _SZ, _P]),
    "rtf_balance_workspace_bytes": (_SZ, [_I64]),
    "rtf_forest_balance": (ctypes.c_int, [_FP, _P, _SZ, _P, _P]),
    "rtf_sample": (ctypes.c_int, [_FP, _P, _I64, _P, _P, _P]),
    "rtf_sample_batched": (ctypes.c_int, [_FP, _P, _P, _I64, _P, _P, _P]),
    "rtf_sample_2d": (ctypes.c_int, [_FP, _P, _I64, _P, _P, _P]),
    "rtf_sample_bsearch": (ctypes.c_int, [_FP, _P, _I64, _P, _P, _P]),
    "rtf_sample_cutpoint_bsearch": (ctypes.c_int, [_FP, _P, _I64, _P, _P, _P]),
    "rtf_quantize_f32": (ctypes.c_int, [_P, _P, _I32, _I64, _P, _P, _P, _P]),
    "rtf_backward_workspace_bytes": (_SZ, [_I32, _I64]),
    "rtf_backward": (ctypes.c_int, [_FP, _P, _P, _P, _P, _I64, _P, _P, _P, _SZ, _P]),
    "rtf_backward_static": (ctypes.c_int, [_FP, _P, _P, _P, _P, _I64, _P, _P, _P]),
    "rtf_check": (ctypes.c_int, [_FP, _P]),
    "rtf_forest_depth": (ctypes.c_int, [_FP, _P, _P]),
    "rtf_forest_export": (ctypes.c_int, [_FP, _P, _P, _P, _P]),
    "rtf_forest_import": (ctypes.c_int, [_P, _P, _P, _P, _P, _I32, _I64, _I64, _P, _SZ, _P, _FP]),
    "rtf_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "rtf_alias_workspace_bytes": (_SZ, [_I32, _I64]),
    "rtf_alias_build": (ctypes.c_int, [_P, _P, _I32, _I64, _P, _SZ, _P, _AP]),
    "rtf_alias_sample": (ctypes.c_int, [_AP, _P, _P, _I64, _P, _P]),
    "rtf_alias_sample_2d": (ctypes.c_int, [_AP, _P, _I64, _P, _P]),
    "rtf_alias_export": (ctypes.c_int, [_AP, _P, _P, _P, _P]),
}


def lib():
    """Load librtforest.so (built by ``__graft_entry__.build()``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build the HIP library first "
                "(python -c 'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _check(code: int, what: str):
    if code != RTF_OK:
        raise RtfError(code, what)


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev(t, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Forest:
    """A built forest: owns its workspace tensor and the C descriptor."""

    def __init__(self, ws, desc: rtf_forest, device):
        self.ws = ws
        self.desc = desc
        self.device = device

    @property
    def D(self):
        return self.desc.D

    @property
    def n_total(self):
        return self.desc.n_total

    @property
    def m_total(self):
        return self.desc.m_total

    def widen(self, ws=None, stream=None):
        """Collapsed 4-ary records for the descended cells (rtf_forest_widen);
        later sampling calls on this forest read them.  Returns self."""
        nb = lib().rtf_wide_workspace_bytes(self.n_total)
        if nb == 0:
            raise RtfError(RTF_ERR_SIZE, "rtf_wide_workspace_bytes")
        if ws is None or ws.numel() < nb:
            ws = _workspace(nb, self.device)
        _check(lib().rtf_forest_widen(ctypes.byref(self.desc), _ptr(ws), nb, _stream(stream)),
               "rtf_forest_widen")
        self.wide_ws = ws
        return self

    def balance(self, ws=None, stream=None) -> int:
        """The depth fallback (rtf_forest_balance): degenerate cell trees are
        replaced by balanced ones; returns the number of cells rebuilt
        (synchronises).  Collapsed records are dropped (widen() again)."""
        nb = lib().rtf_balance_workspace_bytes(self.m_total)
        if nb == 0:
            raise RtfError(RTF_ERR_SIZE, "rtf_balance_workspace_bytes")
        if ws is None or ws.numel() < nb:
            ws = _workspace(nb, self.device)
        count = ctypes.c_int64(0)
        _check(lib().rtf_forest_balance(ctypes.byref(self.desc), _ptr(ws), nb,
                                        ctypes.byref(count), _stream(stream)),
               "rtf_forest_balance")
        self.wide_ws = None
        return int(count.value)

    def wide_view(self):
        """Device view of the collapsed records: int64 [n_total, 8] (k, kc0,
        kc1, r0|r1, r2|r3, unused x3), or None before widen()."""
        if getattr(self, "wide_ws", None) is None or not self.desc.wide:
            return None
        torch = _torch()
        return self.wide_ws[:64 * self.n_total].view(torch.int64).view(self.n_total, 8)

    def depth(self, stream=None) -> int:
        """The deepest search (guide entry + nodes, as Alg. 2 counts reads)
        any uniform makes in this forest (rtf_forest_depth); synchronises."""
        d = ctypes.c_int32(0)
        _check(lib().rtf_forest_depth(ctypes.byref(self.desc), ctypes.byref(d), _stream(stream)),
               "rtf_forest_depth")
        return int(d.value)

    def check(self, stream=None):
        """Synchronise and raise on a device-detected data error."""
        _check(lib().rtf_check(ctypes.byref(self.desc), _stream(stream)), "rtf_check")

    def node_view(self):
        """Device view of the node records: int64 [n_total, 2] holding the key
        bits and the two int32 child references."""
        torch = _torch()
        n = self.n_total
        off = self.desc.nodes - self.ws.data_ptr()
        return self.ws[off:off + NODE_BYTES * n].view(torch.int64).view(n, 2)

    def cell_view(self):
        """Device view of the guide cell records: int64 [m_total, 8] holding
        the keys k[0..6] and the (ref, aux) int32 pair."""
        torch = _torch()
        off = self.desc.cells - self.ws.data_ptr()
        return self.ws[off:off + CELL_BYTES * self.m_total].view(torch.int64).view(
            self.m_total, CELL_KEYS + 1)

    def export_raw(self, stream=None):
        """Host copies of the records as stored: node records uint64 [n, 2],
        cell records uint64 [m, 8], totals uint64 [D] (what rtf_forest_import
        takes back)."""
        import numpy as np
        raw = np.zeros((self.n_total, 2), np.uint64)
        cells = np.zeros((self.m_total, CELL_KEYS + 1), np.uint64)
        W = np.zeros(self.D, np.uint64)
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        _check(lib().rtf_forest_export(ctypes.byref(self.desc), p(raw), p(cells), p(W),
                                       _stream(stream)), "rtf_forest_export")
        return raw, cells, W

    def export(self, stream=None, with_cells=False):
        """Host copies: key uint64[n], child int32[n, 2], table int32[m] (the guide
        entries), W uint64[D]; with ``with_cells`` also the cell records as
        (keys uint64[m, 7], aux int32[m])."""
        import numpy as np
        n, m = self.n_total, self.m_total
        raw = np.zeros((n, 2), np.uint64)
        cells = np.zeros((m, CELL_KEYS + 1), np.uint64)
        W = np.zeros(self.D, np.uint64)
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)
        _check(lib().rtf_forest_export(ctypes.byref(self.desc), p(raw), p(cells), p(W),
                                       _stream(stream)), "rtf_forest_export")
        key = np.ascontiguousarray(raw[:, 0])
        child = np.ascontiguousarray(raw[:, 1]).view(np.int32).reshape(n, 2)
        refs = np.ascontiguousarray(cells[:, CELL_KEYS]).view(np.int32).reshape(m, 2)
        table = np.ascontiguousarray(refs[:, 0])
        if with_cells:
            return key, child, table, W, (np.ascontiguousarray(cells[:, :CELL_KEYS]),
                                          np.ascontiguousarray(refs[:, 1]))
        return key, child, table, W


def _workspace(nbytes, device):
    torch = _torch()
    # 256-byte aligned: torch's caching allocator returns 512-byte aligned blocks
    ws = torch.empty(int(nbytes), dtype=torch.uint8, device=device)
    assert ws.data_ptr() % 256 == 0
    return ws


def build(w, m: int, ws=None, stream=None, tile: int = 0) -> Forest:
    """Guide table + radix tree forest of one distribution (uint32 weights).
    ``ws`` may be a uint8 device tensor to reuse (e.g. a previous forest's);
    ``tile`` (1024 or 2048; 0 for the default) sets the build tile."""
    torch = _torch()
    _dev(w, torch.int32 if w.dtype == torch.int32 else torch.uint32, "w")
    n = w.numel()
    nb = lib().rtf_workspace_bytes(n, int(m))
    if nb == 0:
        raise RtfError(RTF_ERR_SIZE, "rtf_workspace_bytes")
    if ws is None or ws.numel() < nb:
        ws = _workspace(nb, w.device)
    desc = rtf_forest()
    if tile:
        _check(lib().rtf_build_tiled(_ptr(w), n, int(m), int(tile), _ptr(ws), nb, _stream(stream),
                                     ctypes.byref(desc)), "rtf_build_tiled")
    else:
        _check(lib().rtf_build(_ptr(w), n, int(m), _ptr(ws), nb, _stream(stream),
                               ctypes.byref(desc)), "rtf_build")
    return Forest(ws, desc, w.device)


def build_batched(w, elem_off, cell_off, stream=None, tile: int = 0) -> Forest:
    """Forests of D distributions in one launch sequence (Sec. 5).

    ``elem_off``/``cell_off`` are int64 device tensors of D+1 offsets.  The
    workspace is sized from ``w.numel()`` and ``cell_off[-1]`` (read back).
    ``tile`` (1024 or 2048; 0 for the default) sets the build tile.
    """
    torch = _torch()
    _dev(elem_off, torch.int64, "elem_off")
    _dev(cell_off, torch.int64, "cell_off")
    D = elem_off.numel() - 1
    n_total = w.numel()
    m_total = int(cell_off[-1].item())
    nb = lib().rtf_workspace_bytes_batched(D, n_total, m_total)
    if nb == 0:
        raise RtfError(RTF_ERR_SIZE, "rtf_workspace_bytes_batched")
    ws = _workspace(nb, w.device)
    desc = rtf_forest()
    if tile:
        _check(lib().rtf_build_batched_tiled(_ptr(w), _ptr(elem_off), _ptr(cell_off), D, n_total,
                                             m_total, int(tile), _ptr(ws), nb, _stream(stream),
                                             ctypes.byref(desc)), "rtf_build_batched_tiled")
    else:
        _check(lib().rtf_build_batched(_ptr(w), _ptr(elem_off), _ptr(cell_off), D, n_total,
                                       m_total, _ptr(ws), nb, _stream(stream), ctypes.byref(desc)),
               "rtf_build_batched")
    return Forest(ws, desc, w.device)


def _outputs(S, want_x, device, pairs=1):
    torch = _torch()
    idx = torch.empty(S * pairs, dtype=torch.int32, device=device)
    x = torch.empty(S * pairs, dtype=torch.float64, device=device) if want_x else None
    return idx, x


def _u(u):
    torch = _torch()
    return _dev(u, torch.uint64 if u.dtype == torch.uint64 else torch.int64, "u")


def sample(f: Forest, u, want_x=True, out=None, stream=None):
    """Alg. 2 for distribution 0: (idx int32[S], x float64[S] or None)."""
    _u(u)
    S = u.numel()
    idx, x = out if out is not None else _outputs(S, want_x, u.device)
    _check(lib().rtf_sample(ctypes.byref(f.desc), _ptr(u), S, _ptr(idx), _ptr(x),
                            _stream(stream)), "rtf_sample")
    return idx, x


def sample_batched(f: Forest, sample_off, u, want_x=True, out=None, stream=None):
    torch = _torch()
    _dev(sample_off, torch.int64, "sample_off")
    _u(u)
    S = u.numel()
    idx, x = out if out is not None else _outputs(S, want_x, u.device)
    _check(lib().rtf_sample_batched(ctypes.byref(f.desc), _ptr(sample_off), _ptr(u), S,
                                    _ptr(idx), _ptr(x), _stream(stream)), "rtf_sample_batched")
    return idx, x


def sample_2d(f: Forest, u2, want_xy=True, out=None, stream=None):
    """(row, col) int32[S, 2] and (y, x) float64[S, 2] for S pairs u2[S, 2]."""
    _u(u2)
    S = u2.numel() // 2
    rc, xy = out if out is not None else _outputs(S, want_xy, u2.device, pairs=2)
    _check(lib().rtf_sample_2d(ctypes.byref(f.desc), _ptr(u2), S, _ptr(rc), _ptr(xy),
                               _stream(stream)), "rtf_sample_2d")
    return rc.view(S, 2), (xy.view(S, 2) if xy is not None else None)


def sample_bsearch(f: Forest, u, want_x=True, out=None, stream=None):
    """Baseline: plain binary search over all keys (same mapping)."""
    _u(u)
    S = u.numel()
    idx, x = out if out is not None else _outputs(S, want_x, u.device)
    _check(lib().rtf_sample_bsearch(ctypes.byref(f.desc), _ptr(u), S, _ptr(idx), _ptr(x),
                                    _stream(stream)), "rtf_sample_bsearch")
    return idx, x


def sample_cutpoint_bsearch(f: Forest, u, want_x=True, out=None, stream=None):
    """Baseline: guide table plus bisection inside the cell (same mapping)."""
    _u(u)
    S = u.numel()
    idx, x = out if out is not None else _outputs(S, want_x, u.device)
    _check(lib().rtf_sample_cutpoint_bsearch(ctypes.byref(f.desc), _ptr(u), S, _ptr(idx),
                                             _ptr(x), _stream(stream)),
           "rtf_sample_cutpoint_bsearch")
    return idx, x


def quantize(v, elem_off=None, status=None, out=None, stream=None):
    """float32 weights -> (uint32 q, float64 scale[D]) per distribution."""
    torch = _torch()
    _dev(v, torch.float32, "v")
    D = 1 if elem_off is None else elem_off.numel() - 1
    if elem_off is not None:
        _dev(elem_off, torch.int64, "elem_off")
    if out is None:
        q = torch.empty(v.numel(), dtype=torch.uint32, device=v.device)
        scale = torch.empty(D, dtype=torch.float64, device=v.device)
    else:
        q, scale = out
    _check(lib().rtf_quantize_f32(_ptr(v), _ptr(elem_off), D, v.numel(), _ptr(q), _ptr(scale),
                                  _ptr(status), _stream(stream)), "rtf_quantize_f32")
    return q, scale


def backward(f: Forest, u, idx, grad_x, scale, sample_off=None, ws=None, stream=None):
    """dL/dv (float64[n_total]) of the samples' positions x (index held fixed)."""
    torch = _torch()
    nb = lib().rtf_backward_workspace_bytes(f.D, f.n_total)
    if ws is None:
        ws = _workspace(nb, u.device)
    grad_w = torch.empty(f.n_total, dtype=torch.float64, device=u.device)
    _check(lib().rtf_backward(ctypes.byref(f.desc), _ptr(sample_off), _ptr(u), _ptr(idx),
                              _ptr(grad_x), u.numel(), _ptr(scale), _ptr(grad_w), _ptr(ws), nb,
                              _stream(stream)), "rtf_backward")
    return grad_w


def backward_static(f: Forest, u, idx, grad_x, scale, sample_off=None, out=None, stream=None):
    """rtf_backward_static: backward() with the library's fixed device scratch
    (no workspace; n_total <= 2^20 and D <= 2^16).  `out` is an optional
    preallocated float64[n_total] result, so that the call allocates nothing."""
    torch = _torch()
    grad_w = out if out is not None else torch.empty(f.n_total, dtype=torch.float64,
                                                     device=u.device)
    _check(lib().rtf_backward_static(ctypes.byref(f.desc), _ptr(sample_off), _ptr(u), _ptr(idx),
                                     _ptr(grad_x), u.numel(), _ptr(scale), _ptr(grad_w),
                                     _stream(stream)), "rtf_backward_static")
    return grad_w


class AliasTable:
    """Alias tables built by rtf_alias_build (the non-monotone comparison
    mapping of Sec. 2.6); owns its workspace."""

    def __init__(self, ws, desc, device):
        self.ws, self.desc, self.device = ws, desc, device

    def export(self, stream=None):
        """Host copies (thr uint64[n_total], alias int32[n_total], W uint64[D]);
        raises on an error the build recorded."""
        import numpy as np
        n, D = self.desc.n_total, self.desc.D
        thr = np.zeros(n, np.uint64)
        alias = np.zeros(n, np.int32)
        W = np.zeros(D, np.uint64)
        p = lambda a: a.ctypes.data_as(ctypes.c_void_p)  # noqa: E731
        _check(lib().rtf_alias_export(ctypes.byref(self.desc), p(thr), p(alias), p(W),
                                      _stream(stream)), "rtf_alias_export")
        return thr, alias, W


def alias_build(w, elem_off=None, stream=None) -> AliasTable:
    """Alias tables of D distributions of uint32 weights (rtf_alias_build)."""
    torch = _torch()
    _dev(w, torch.uint32, "w")
    D = 1 if elem_off is None else elem_off.numel() - 1
    if elem_off is not None:
        _dev(elem_off, torch.int64, "elem_off")
    nb = lib().rtf_alias_workspace_bytes(D, w.numel())
    if nb == 0:
        raise RtfError(RTF_ERR_SIZE, "rtf_alias_workspace_bytes")
    ws = _workspace(nb, w.device)
    desc = rtf_alias_table()
    _check(lib().rtf_alias_build(_ptr(w), _ptr(elem_off), D, w.numel(), _ptr(ws), nb,
                                 _stream(stream), ctypes.byref(desc)), "rtf_alias_build")
    return AliasTable(ws, desc, w.device)


def alias_sample(t: AliasTable, u, sample_off=None, out=None, stream=None):
    """Indices of the alias mapping (rtf_alias_sample)."""
    torch = _torch()
    u = _u(u)
    idx = out if out is not None else torch.empty(u.numel(), dtype=torch.int32, device=u.device)
    _check(lib().rtf_alias_sample(ctypes.byref(t.desc), _ptr(sample_off), _ptr(u), u.numel(),
                                  _ptr(idx), _stream(stream)), "rtf_alias_sample")
    return idx


def alias_sample_2d(t: AliasTable, u2, out=None, stream=None):
    """(row, column) pairs of the alias mapping (rtf_alias_sample_2d);
    u2 uint64[S, 2]."""
    torch = _torch()
    u2 = _u(u2)
    S = u2.numel() // 2
    rc = out if out is not None else torch.empty((S, 2), dtype=torch.int32, device=u2.device)
    _check(lib().rtf_alias_sample_2d(ctypes.byref(t.desc), _ptr(u2), S, _ptr(rc),
                                     _stream(stream)), "rtf_alias_sample_2d")
    return rc


def forest_import(nodes_raw, cells_raw, W, elem_off=None, cell_off=None, device="cuda:0",
                  stream=None) -> Forest:
    """rtf_forest_import: a forest from host records (uint64 [n, 2] node
    records and uint64 [m, 8] cell records as Forest.export_raw gives them,
    uint64 [D] totals, int64 [D+1] host offsets or None for one distribution)."""
    import numpy as np
    torch = _torch()
    nodes_raw = np.ascontiguousarray(nodes_raw, np.uint64)
    cells_raw = np.ascontiguousarray(cells_raw, np.uint64)
    W = np.ascontiguousarray(W, np.uint64)
    n, m, D = nodes_raw.shape[0], cells_raw.shape[0], W.size
    L = lib()
    nb = L.rtf_workspace_bytes_batched(D, n, m)
    if nb == 0:
        raise RtfError(RTF_ERR_SIZE, "rtf_workspace_bytes_batched")
    ws = _workspace(nb, torch.device(device))
    p = lambda a: a.ctypes.data_as(ctypes.c_void_p) if a is not None else None  # noqa: E731
    eo = np.ascontiguousarray(elem_off, np.int64) if elem_off is not None else None
    co = np.ascontiguousarray(cell_off, np.int64) if cell_off is not None else None
    desc = rtf_forest()
    _check(L.rtf_forest_import(p(nodes_raw), p(cells_raw), p(W), p(eo), p(co), D, n, m, _ptr(ws), nb,
                               _stream(stream), ctypes.byref(desc)), "rtf_forest_import")
    return Forest(ws, desc, torch.device(device))


def cells_like(elem_off, ratio: float = 1.0):
    """Cell offsets with m_d = max(1, round(ratio * n_d)) per distribution
    (the paper's policy of a guide table proportional to n, Sec. 3)."""
    torch = _torch()
    n_d = (elem_off[1:] - elem_off[:-1]).double()
    m_d = torch.clamp(torch.round(n_d * ratio), min=1).to(torch.int64)
    co = torch.zeros_like(elem_off)
    co[1:] = torch.cumsum(m_d, 0)
    return co


def __getattr__(name):
    if name == "RTFSample":  # defined on first use, so that importing is torch-free
        from .autograd import RTFSample
        return RTFSample
    raise AttributeError(name)
