"""Preallocated quantise -> build -> sample chains for fixed shapes.

A plan owns every buffer the chain needs (weights, workspace, outputs), so
`run()` only enqueues library calls on the current stream: no allocation, no
host synchronisation.  That makes the chain capturable into a HIP graph
(`capture()`), which is how many uneven distributions are built and sampled
with one replay (Sec. 5: many tables and trees at once).
"""
from __future__ import annotations

import ctypes

import torch

from . import (RTF_OK, RtfError, _check, _ptr, _stream, lib, rtf_forest)


class BatchedPlan:
    """Quantise, build and sample D distributions stored back to back.

    elem_off, cell_off, sample_off: int64 device tensors of D+1 offsets.
    n_total = elem_off[-1], m_total = cell_off[-1], S = sample_off[-1]
    (passed from the host so that nothing is read back).
    """

    def __init__(self, elem_off, cell_off, sample_off, n_total, m_total, S, want_x=True,
                 collapsed=False, tile=0):
        dev = elem_off.device
        self.tile = int(tile) or 2048  # elements per build tile (1024 or 2048)
        self.D = elem_off.numel() - 1
        self.elem_off, self.cell_off, self.sample_off = elem_off, cell_off, sample_off
        self.n, self.m, self.S = int(n_total), int(m_total), int(S)
        L = lib()
        self.ws_bytes = L.rtf_workspace_bytes_batched(self.D, self.n, self.m)
        if self.ws_bytes == 0:
            raise RtfError(2, "rtf_workspace_bytes_batched")
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.q = torch.empty(self.n, dtype=torch.uint32, device=dev)
        self.scale = torch.empty(self.D, dtype=torch.float64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.idx = torch.empty(self.S, dtype=torch.int32, device=dev)
        self.x = torch.empty(self.S, dtype=torch.float64, device=dev) if want_x else None
        self.desc = rtf_forest()
        self.collapsed = collapsed
        self.wide_ws = None
        if collapsed:
            self.wide_ws = torch.empty(L.rtf_wide_workspace_bytes(self.n), dtype=torch.uint8,
                                       device=dev)

    def run(self, v, u, stream=None):
        """Enqueue quantise + build (+ collapsed records) + sample; returns
        (idx, x) views."""
        L = lib()
        st = _stream(stream)
        _check(L.rtf_quantize_f32(_ptr(v), _ptr(self.elem_off), self.D, self.n, _ptr(self.q),
                                  _ptr(self.scale), _ptr(self.status), st), "rtf_quantize_f32")
        _check(L.rtf_build_batched_tiled(_ptr(self.q), _ptr(self.elem_off), _ptr(self.cell_off),
                                         self.D, self.n, self.m, self.tile, _ptr(self.ws),
                                         self.ws_bytes, st, ctypes.byref(self.desc)),
               "rtf_build_batched_tiled")
        if self.collapsed:
            _check(L.rtf_forest_widen(ctypes.byref(self.desc), _ptr(self.wide_ws),
                                      self.wide_ws.numel(), st), "rtf_forest_widen")
        _check(L.rtf_sample_batched(ctypes.byref(self.desc), _ptr(self.sample_off), _ptr(u),
                                    self.S, _ptr(self.idx), _ptr(self.x), st),
               "rtf_sample_batched")
        return self.idx, self.x

    def capture(self, v, u):
        """Record run(v, u) into a graph; replay() re-runs it on the same buffers
        (refill v and u in place to sample new data)."""
        torch.cuda.synchronize()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):  # a warm-up outside the capture
            self.run(v, u)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run(v, u)
        return g

    def check(self):
        """Raise on a data error the build or the quantisation recorded."""
        torch.cuda.synchronize()
        code = lib().rtf_check(ctypes.byref(self.desc), None)
        if code != RTF_OK:
            raise RtfError(code, "rtf_check")
        if int(self.status.item()) & (1 << 6):
            raise RtfError(6, "rtf_quantize_f32")


class DiffPlan(BatchedPlan):
    """A BatchedPlan that also owns the adjoint's workspace and outputs, so
    that RTFSample's forward and backward allocate nothing and read nothing
    back: the whole differentiable step can be captured as one HIP graph.

    The forward returns a view of the plan's position buffer, and the
    backward the plan's gradient buffer: both are overwritten by the next
    call through the same plan.
    """

    def __init__(self, elem_off, cell_off, sample_off, n_total, m_total, S, v_dtype=torch.float32,
                 collapsed=False, tile=0):
        super().__init__(elem_off, cell_off, sample_off, n_total, m_total, S, want_x=True,
                         collapsed=collapsed, tile=tile)
        L = lib()
        dev = elem_off.device
        self.bws_bytes = L.rtf_backward_workspace_bytes(self.D, self.n)
        self.bws = torch.empty(self.bws_bytes, dtype=torch.uint8, device=dev)
        self.grad_w = torch.empty(self.n, dtype=torch.float64, device=dev)
        self.grad_v = torch.empty(self.n, dtype=v_dtype, device=dev)

    def backward(self, u, grad_x, stream=None):
        """Enqueue rtf_backward for the last run(); returns grad_v (dL/dv in
        the weights' dtype)."""
        _check(lib().rtf_backward(ctypes.byref(self.desc), _ptr(self.sample_off), _ptr(u),
                                  _ptr(self.idx), _ptr(grad_x), self.S, _ptr(self.scale),
                                  _ptr(self.grad_w), _ptr(self.bws), self.bws_bytes,
                                  _stream(stream)), "rtf_backward")
        self.grad_v.copy_(self.grad_w)
        return self.grad_v
