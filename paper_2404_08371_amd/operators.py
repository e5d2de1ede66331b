"""Python handles for meshes and operators (thin wrappers over the C ABI).

Device memory and streams come from PyTorch; every step of an apply runs in
the library's HIP kernels.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check, lib, release

P1_LAPLACE, P1_DIVKGRAD, P2_LAPLACE, P2_DIVKGRAD, P2V_EPSILON, N1_CURLCURL = range(6)
F64, F32 = 0, 1
BC_NONE, BC_DIRICHLET_ZERO = 0, 1
MAP_AFFINE, MAP_SHELL_RADIAL = 0, 1

KIND_NAMES = {P1_LAPLACE: "p1_laplace", P1_DIVKGRAD: "p1_divkgrad", P2_LAPLACE: "p2_laplace",
              P2_DIVKGRAD: "p2_divkgrad", P2V_EPSILON: "p2v_epsilon", N1_CURLCURL: "n1_curlcurl"}
SPACE = {P1_LAPLACE: 1, P1_DIVKGRAD: 1, P2_LAPLACE: 2, P2_DIVKGRAD: 2, P2V_EPSILON: 2, N1_CURLCURL: 2}
# values per slot of the coefficient vector (N1: alpha, then beta)
COEFF_COMPS = {N1_CURLCURL: 2}
DTYPE = {F64: torch.float64, F32: torch.float32}


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


class Mesh:
    """A macro tetrahedral mesh refined uniformly `level` times."""

    def __init__(self, vertices, tets, level, map=MAP_AFFINE):
        v = np.ascontiguousarray(vertices, dtype=np.float64)
        t = np.ascontiguousarray(tets, dtype=np.int64)
        if v.ndim != 2 or v.shape[1] != 3 or t.ndim != 2 or t.shape[1] != 4:
            raise ValueError("vertices must be (nv,3) and tets (nt,4)")
        h = ctypes.c_void_p()
        check(lib().tmf_mesh_create(_ptr(v, ctypes.c_double), v.shape[0], _ptr(t, ctypes.c_int64),
                                    t.shape[0], int(level), int(map), ctypes.byref(h)))
        self._h = h
        self.level, self.map = int(level), int(map)
        self.vertices, self.tets = v, t

    @property
    def handle(self):
        return self._h

    def layout(self, space):
        nl, nu = ctypes.c_int64(), ctypes.c_int64()
        check(lib().tmf_mesh_layout(self._h, int(space), ctypes.byref(nl), ctypes.byref(nu)))
        return nl.value, nu.value

    def dof_info(self, space, keys=True, xyz=True, owner=True, boundary=True):
        """Host arrays describing every slot of the macro-local layout of `space`."""
        nl, _ = self.layout(space)
        out = {}
        k = np.empty((nl, 8), np.int64) if keys else None
        x = np.empty((nl, 3), np.float64) if xyz else None
        o = np.empty(nl, np.uint8) if owner else None
        b = np.empty(nl, np.uint8) if boundary else None
        check(lib().tmf_mesh_dof_info(self._h, int(space),
                                      _ptr(k, ctypes.c_int64) if keys else None,
                                      _ptr(x, ctypes.c_double) if xyz else None,
                                      _ptr(o, ctypes.c_uint8) if owner else None,
                                      _ptr(b, ctypes.c_uint8) if boundary else None))
        for name, arr in (("keys", k), ("xyz", x), ("owner", o), ("boundary", b)):
            if arr is not None:
                out[name] = arr if name in ("keys", "xyz") else arr.astype(bool)
        return out

    def __del__(self):
        release(getattr(self, "_h", None), "tmf_mesh_destroy")
        self._h = None


def _stream_handle(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Operator:
    """y = A(coeff) x on a refined mesh; see include/tetmf.h for the layout."""

    def __init__(self, mesh, kind, prec=F64, bc=BC_DIRICHLET_ZERO, rule=None):
        self.mesh = mesh  # keeps the mesh alive
        self.kind, self.prec, self.bc = int(kind), int(prec), int(bc)
        h = ctypes.c_void_p()
        if rule is not None:
            qb = np.ascontiguousarray(rule[0], dtype=np.float64)
            qw = np.ascontiguousarray(rule[1], dtype=np.float64)
            args = (_ptr(qb, ctypes.c_double), _ptr(qw, ctypes.c_double), int(qw.size))
        else:
            args = (None, None, 0)
        check(lib().tmf_op_create(mesh.handle, self.kind, self.prec, self.bc, *args, ctypes.byref(h)))
        self._h = h
        nl, nu = ctypes.c_int64(), ctypes.c_int64()
        nc, hc = ctypes.c_int(), ctypes.c_int()
        check(lib().tmf_op_info(h, ctypes.byref(nl), ctypes.byref(nu), ctypes.byref(nc), ctypes.byref(hc)))
        self.n_local, self.n_unique, self.ncomp = nl.value, nu.value, nc.value
        self.has_coeff = bool(hc.value)
        self.space = SPACE[self.kind]
        self.dtype = DTYPE[self.prec]
        self.coeff_comps = COEFF_COMPS.get(self.kind, 1)

    @property
    def handle(self):
        return self._h

    def _vec(self, t, name, ncomp):
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise TypeError("%s must be a CUDA/HIP torch tensor" % name)
        if t.dtype != self.dtype:
            raise TypeError("%s has dtype %s, the operator computes in %s" % (name, t.dtype, self.dtype))
        if not t.is_contiguous() or t.numel() != ncomp * self.n_local:
            raise ValueError("%s must be contiguous with %d values" % (name, ncomp * self.n_local))
        return ctypes.c_void_p(t.data_ptr())

    def apply(self, x, coeff=None, out=None):
        """Enqueue y = A(coeff) x on the current stream of x's device; returns y."""
        px = self._vec(x, "x", self.ncomp)
        pk = self._vec(coeff, "coeff", self.coeff_comps) if self.has_coeff else None
        if not self.has_coeff and coeff is not None:
            raise ValueError("this operator takes no coefficient")
        if out is None:
            out = torch.empty_like(x)
        py = self._vec(out, "out", self.ncomp)
        with torch.cuda.device(x.device):
            check(lib().tmf_apply(self._h, pk, px, py, _stream_handle(x.device)))
        return out

    def apply_local(self, x, coeff=None, out=None):
        """Macro-local partial sums (the apply without the interface sum)."""
        px = self._vec(x, "x", self.ncomp)
        pk = self._vec(coeff, "coeff", self.coeff_comps) if self.has_coeff else None
        if out is None:
            out = torch.empty_like(x)
        py = self._vec(out, "out", self.ncomp)
        with torch.cuda.device(x.device):
            check(lib().tmf_apply_local(self._h, pk, px, py, _stream_handle(x.device)))
        return out

    def diagonal(self, coeff=None, out=None):
        """diag(A(coeff)) in the macro-local layout (component-major for the epsilon operator),
        every copy holding the total (P1, exact scalar P2 and epsilon kinds)."""
        pk = self._vec(coeff, "coeff", 1) if self.has_coeff else None
        if not self.has_coeff and coeff is not None:
            raise ValueError("this operator takes no coefficient")
        if out is None:
            out = torch.empty(self.ncomp * self.n_local, dtype=self.dtype,
                              device=coeff.device if coeff is not None else "cuda")
        pd = self._vec(out, "out", self.ncomp)
        with torch.cuda.device(out.device):
            check(lib().tmf_diagonal(self._h, pk, pd, _stream_handle(out.device)))
        return out

    def store_matrices(self, coeff):
        """Evaluate and keep every micro-tet's local matrix A_T(coeff) (P2 div(k grad))."""
        pk = self._vec(coeff, "coeff", 1)
        with torch.cuda.device(coeff.device):
            check(lib().tmf_op_store_matrices(self._h, pk, _stream_handle(coeff.device)))

    def apply_stored(self, x, out=None):
        """y = A x from the stored local matrices."""
        px = self._vec(x, "x", 1)
        if out is None:
            out = torch.empty_like(x)
        with torch.cuda.device(x.device):
            check(lib().tmf_apply_stored(self._h, px, self._vec(out, "out", 1), _stream_handle(x.device)))
        return out

    def tune(self, x, coeff=None, y=None, reps=5, cache=None):
        """Choose the tile shape by timing (tmf_op_tune); with `cache` (a JSON path) a result stored
        for this operator and device is reused and new results are added.  Returns (cfg, ms)."""
        px = self._vec(x, "x", self.ncomp)
        pk = self._vec(coeff, "coeff", self.coeff_comps) if self.has_coeff else None
        if y is None:
            y = torch.empty_like(x)
        cfg, ms = ctypes.c_int(), ctypes.c_float()
        with torch.cuda.device(x.device):
            check(lib().tmf_op_tune(self._h, pk, px, self._vec(y, "y", self.ncomp), _stream_handle(x.device),
                                    int(reps), cache.encode() if cache else None, ctypes.byref(cfg),
                                    ctypes.byref(ms)))
        return cfg.value, ms.value

    def interface_sum_(self, v):
        """In place: every copy of a shared DoF gets the sum over its copies."""
        pv = self._vec(v, "v", self.ncomp)
        with torch.cuda.device(v.device):
            check(lib().tmf_interface_sum(self._h, pv, _stream_handle(v.device)))
        return v

    def adjoint(self, coeff, x, gy, gx=None, gk=None, want_gk=True):
        """Reverse mode of the macro-local apply of the div(k grad) kinds (P1, P2) and the epsilon
        operator: returns (gx, gk); gk is the gradient for the coefficient (k or mu)."""
        nc = self.ncomp
        pk, px, pg = self._vec(coeff, "coeff", 1), self._vec(x, "x", nc), self._vec(gy, "gy", nc)
        if gx is None:
            gx = torch.empty_like(x)
        if gk is None and want_gk:
            gk = torch.empty_like(coeff)
        with torch.cuda.device(x.device):
            check(lib().tmf_apply_adjoint(self._h, pk, px, pg, self._vec(gx, "gx", nc),
                                          self._vec(gk, "gk", 1) if gk is not None else None,
                                          _stream_handle(x.device)))
        return gx, gk

    def __del__(self):
        release(getattr(self, "_h", None), "tmf_op_destroy")
        self._h = None
