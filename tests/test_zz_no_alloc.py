"""The allocation-free apply (seam partial sums in the library's static device
scratch) against the ordinary apply, through the C ABI: two calls in a row on
one GPU, the second on a smaller operator, then the other operator families,
and the size limit (a host-side error, nothing launched).  Bar: FP64 <= 1e-12
relative (max-norm), FP32 <= 1e-5, as for the oracle parity tests."""
import ctypes

import numpy as np
import pytest
import torch

import paper_2404_08371_amd as T
from paper_2404_08371_amd.operators import _stream_handle
import workloads as W

pytestmark = pytest.mark.gpu


def noalloc(op, x, k):
    y = torch.full_like(x, float("nan"))
    st = T.lib().tmf_apply_noalloc(op.handle, ctypes.c_void_p(k.data_ptr()) if k is not None else None,
                                   ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                   _stream_handle(x.device))
    T.check(st)
    return y


def operator(mesh, level, kind, prec, cfg=None):
    mk, mp = {"cube": (W.meshes.kuhn_cube, 0), "ref": (W.meshes.ref_tet, 0),
              "shell": (W.meshes.octahedral_shell, 1)}[mesh]
    v, t = mk()
    m = T.Mesh(v, t, level, mp)
    rule = W.quadrature.rule_degree5() if mp == 1 else None
    op = T.Operator(m, kind, prec, T.BC_DIRICHLET_ZERO, rule=rule)
    if cfg is not None:
        T.check(T.lib().tmf_op_set_tile(op.handle, cfg))
    info = m.dof_info(op.space, owner=False, boundary=False)
    x = np.concatenate([W.uniform_from_keys(3, info["keys"], stream=c) for c in range(op.ncomp)])
    if kind == T.P2V_EPSILON:
        k = W.fields.shell_mu(info["keys"], info["xyz"], 4)
    elif kind == T.P1_DIVKGRAD:
        k = W.fields.perturbed_k(info["keys"], 4)
    elif op.has_coeff:
        k = W.fields.cube_k(info["xyz"])
    else:
        k = None
    xt = torch.tensor(x, dtype=op.dtype, device="cuda")
    kt = torch.tensor(k, dtype=op.dtype, device="cuda") if k is not None else None
    return op, xt, kt


def check(op, x, k):
    ref = op.apply(x, k)
    y = noalloc(op, x, k)
    torch.cuda.synchronize()
    assert not torch.isnan(y).any()
    err = ((y - ref).abs().max() / ref.abs().max()).item()
    assert err <= (1e-12 if op.prec == T.F64 else 1e-5), err
    return err


def test_two_calls_in_a_row_second_smaller():
    print("no-alloc: cube level 6 FP64, then cube level 4", flush=True)
    big = operator("cube", 6, T.P2_DIVKGRAD, T.F64)
    small = operator("cube", 4, T.P2_DIVKGRAD, T.F64)
    e1 = check(*big)
    e2 = check(*small)
    print("errors", e1, e2)


@pytest.mark.parametrize("mesh,level,kind,prec,cfg", [
    ("cube", 5, T.P2_DIVKGRAD, T.F32, None), ("cube", 5, T.P2_LAPLACE, T.F64, 2),
    ("cube", 5, T.P2_DIVKGRAD, T.F64, 5), ("ref", 5, T.P2_DIVKGRAD, T.F64, 1),
    ("shell", 3, T.P2V_EPSILON, T.F64, None), ("ref", 6, T.P1_DIVKGRAD, T.F64, None)])
def test_other_operators(mesh, level, kind, prec, cfg):
    print("no-alloc case", mesh, level, kind, prec, cfg, flush=True)
    check(*operator(mesh, level, kind, prec, cfg))


def test_too_large_is_refused_without_launch():
    op, x, k = operator("cube", 7, T.P2_DIVKGRAD, T.F64)
    y = torch.full_like(x, float("nan"))
    st = T.lib().tmf_apply_noalloc(op.handle, ctypes.c_void_p(k.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                   ctypes.c_void_p(y.data_ptr()), _stream_handle(x.device))
    assert st == -1
    assert b"static scratch" in T.lib().tmf_last_error()
    torch.cuda.synchronize()
    assert torch.isnan(y).all()
