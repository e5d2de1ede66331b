"""Batched operators and the iterative-refinement CG solver (FP32 or FP64 inner iteration)."""
import ctypes

import numpy as np
import torch

from ._lib import check, lib, release
from .operators import DTYPE, _stream_handle


PRECOND_NONE, PRECOND_JACOBI = 0, 1


class IROptions(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_outer", ctypes.c_int), ("inner_rtol", ctypes.c_double),
                ("inner_maxit", ctypes.c_int), ("graph_iters", ctypes.c_int), ("use_graph", ctypes.c_int),
                ("precond", ctypes.c_int)]


class IRStats(ctypes.Structure):
    _fields_ = [("outer", ctypes.c_int), ("inner_total", ctypes.c_int), ("graph_launches", ctypes.c_int),
                ("converged", ctypes.c_int), ("seconds", ctypes.c_double)]


class Batch:
    """Many operator instances applied in one launch of the element kernel (vectors concatenated)."""

    def __init__(self, ops):
        self.ops = list(ops)  # keeps the operators alive
        arr = (ctypes.c_void_p * len(self.ops))(*[o.handle for o in self.ops])
        h = ctypes.c_void_p()
        check(lib().tmf_batch_create(arr, len(self.ops), ctypes.byref(h)))
        self._h = h
        cnt = ctypes.c_int()
        off = np.zeros(len(self.ops) + 1, np.int64)
        check(lib().tmf_batch_info(h, ctypes.byref(cnt), off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))))
        self.count = cnt.value
        self.offsets = off
        self.length = int(off[-1])
        self.dtype = DTYPE[self.ops[0].prec]
        self.has_coeff = self.ops[0].has_coeff

    @property
    def handle(self):
        return self._h

    def _ptr(self, t, name):
        if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != self.dtype:
            raise TypeError("%s must be a device tensor of %s" % (name, self.dtype))
        if not t.is_contiguous() or t.numel() != self.length:
            raise ValueError("%s must be contiguous with %d values" % (name, self.length))
        return ctypes.c_void_p(t.data_ptr())

    def concat(self, parts):
        return torch.cat([p.reshape(-1) for p in parts]).contiguous()

    def split(self, v):
        return [v[self.offsets[i]:self.offsets[i + 1]] for i in range(self.count)]

    def apply(self, x, coeff=None, out=None, active=None):
        px = self._ptr(x, "x")
        pk = self._ptr(coeff, "coeff") if self.has_coeff else None
        if out is None:
            out = torch.empty_like(x)
        pa = None
        if active is not None:
            if active.dtype != torch.uint8 or not active.is_cuda or active.numel() != self.count:
                raise ValueError("active must be a device uint8 tensor with one flag per instance")
            pa = ctypes.c_void_p(active.data_ptr())
        check(lib().tmf_batch_apply(self._h, pk, px, self._ptr(out, "out"), pa, _stream_handle(x.device)))
        return out

    def diagonal(self, coeff=None, out=None):
        """diag(A_i(coeff_i)) of every instance, concatenated (scalar P2 kinds)."""
        pk = self._ptr(coeff, "coeff") if self.has_coeff else None
        if out is None:
            out = torch.empty(self.length, dtype=self.dtype, device=coeff.device if coeff is not None else "cuda")
        check(lib().tmf_batch_diagonal(self._h, pk, self._ptr(out, "out"), _stream_handle(out.device)))
        return out

    def set_tile(self, cfg):
        check(lib().tmf_batch_set_tile(self._h, int(cfg)))

    def autotune(self, x, coeff=None, y=None, reps=5):
        if y is None:
            y = torch.empty_like(x)
        cfg, ms = ctypes.c_int(), ctypes.c_float()
        check(lib().tmf_batch_autotune(self._h, self._ptr(coeff, "coeff") if self.has_coeff else None,
                                       self._ptr(x, "x"), self._ptr(y, "y"), _stream_handle(x.device), int(reps),
                                       ctypes.byref(cfg), ctypes.byref(ms)))
        return cfg.value, ms.value

    def tune(self, x, coeff=None, y=None, reps=5, cache=None):
        """tmf_batch_tune: autotune with an optional JSON result cache; returns (cfg, ms)."""
        if y is None:
            y = torch.empty_like(x)
        cfg, ms = ctypes.c_int(), ctypes.c_float()
        check(lib().tmf_batch_tune(self._h, self._ptr(coeff, "coeff") if self.has_coeff else None,
                                   self._ptr(x, "x"), self._ptr(y, "y"), _stream_handle(x.device), int(reps),
                                   cache.encode() if cache else None, ctypes.byref(cfg), ctypes.byref(ms)))
        return cfg.value, ms.value

    def __del__(self):
        release(getattr(self, "_h", None), "tmf_batch_destroy")
        self._h = None


class IRSolver:
    """FP64 iterative refinement around an inner CG over a pair of batches: the FP64 batch for the
    outer residual, and the inner batch, FP32 (mixed precision) or FP64 (plain FP64 CG, e.g. the
    FP64 batch itself with inner_rtol below tol)."""

    def __init__(self, b64, b32, tol=1e-10, max_outer=30, inner_rtol=1e-4, inner_maxit=2000, graph_iters=16,
                 use_graph=True, precond=PRECOND_JACOBI):
        self.b64, self.b32 = b64, b32
        opt = IROptions(tol, max_outer, inner_rtol, inner_maxit, graph_iters, 1 if use_graph else 0, int(precond))
        h = ctypes.c_void_p()
        check(lib().tmf_ir_create(b64.handle, b32.handle, ctypes.byref(opt), ctypes.byref(h)))
        self._h = h

    def solve(self, b, x, coeff64=None, coeff32=None, raise_on_notconv=True):
        """Solves in place into x (FP64 device tensor); returns (stats dict, relres array).
        coeff32 is the coefficient in the inner batch's precision."""
        st = IRStats()
        rel = np.zeros(self.b64.count)
        pk64 = self.b64._ptr(coeff64, "coeff64") if self.b64.has_coeff else None
        pk32 = self.b32._ptr(coeff32, "coeff32") if self.b32.has_coeff else None
        status = lib().tmf_ir_solve(self._h, pk64, pk32, self.b64._ptr(b, "b"), self.b64._ptr(x, "x"),
                                    ctypes.byref(st), rel.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    _stream_handle(x.device))
        if status != -5 or raise_on_notconv:
            check(status)
        return ({"outer": st.outer, "inner_total": st.inner_total, "graph_launches": st.graph_launches,
                 "converged": bool(st.converged), "seconds": st.seconds}, rel)

    def __del__(self):
        release(getattr(self, "_h", None), "tmf_ir_destroy")
        self._h = None
