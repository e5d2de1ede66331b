"""GPU operator diagonal against the oracle's diag(D A D).

The diagonal mode of the element kernel adds each micro-tet's local diagonal
(A_T)_vv in LDS and goes through the same seam and interface reduction as the
apply.  FP64: relative error <= 1e-12 (max-norm); FP32: <= 1e-5, as for the
apply.  Outputs start as NaN, so an unwritten slot shows.  The batched
diagonal equals the per-instance ones; kinds without a diagonal are refused.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
import paper_2404_08371_amd as T
from helpers import MESHES, coefficient, oracle_problem, rel_err
import workloads as W

pytestmark = pytest.mark.gpu

LIB_KIND = {O.P2_LAPLACE: T.P2_LAPLACE, O.P2_DIVKGRAD: T.P2_DIVKGRAD}


def lib_op(mesh, level, kind, bc, prec):
    mk, mp = MESHES[mesh]
    v, t = mk()
    m = T.Mesh(v, t, level, mp)
    return m, T.Operator(m, LIB_KIND[kind], prec, bc)


@pytest.mark.parametrize("mesh,level", [("cube", 3), ("cube", 4), ("ref", 5), ("flatshell", 2)])
@pytest.mark.parametrize("kind", [O.P2_LAPLACE, O.P2_DIVKGRAD])
@pytest.mark.parametrize("bc", [O.BC_DIRICHLET_ZERO, O.BC_NONE])
@pytest.mark.parametrize("prec", [T.F64, T.F32])
def test_diagonal_matches_oracle(mesh, level, kind, bc, prec):
    print("diag case", mesh, level, kind, bc, prec, flush=True)
    m, op = lib_op(mesh, level, kind, bc, prec)
    info = m.dof_info(2, owner=False, boundary=False)
    dt = torch.float64 if prec == T.F64 else torch.float32
    k = coefficient(kind, info["keys"], info["xyz"], 7)
    kt = torch.tensor(k, dtype=dt, device="cuda") if k is not None else None
    out = torch.full((op.n_local,), float("nan"), dtype=dt, device="cuda")
    d = op.diagonal(kt, out=out).double().cpu().numpy()
    assert not np.isnan(d).any()
    pr = oracle_problem(mesh, level, kind, bc)
    ref = pr.diagonal(coefficient(kind, pr.keys, pr.xyz, 7))
    e2, ei = rel_err(d, ref)
    assert ei <= (1e-12 if prec == T.F64 else 1e-5), (e2, ei)


@pytest.mark.parametrize("cfg", list(range(7)))
def test_diagonal_every_tile_shape(cfg):
    """Every tile shape the apply may use; with a marching shape the diagonal runs on a box shape."""
    print("diag tile", cfg, flush=True)
    m, op = lib_op("cube", 4, O.P2_DIVKGRAD, O.BC_DIRICHLET_ZERO, T.F64)
    T.check(T.lib().tmf_op_set_tile(op.handle, cfg))
    info = m.dof_info(2, owner=False, boundary=False)
    kt = torch.tensor(coefficient(O.P2_DIVKGRAD, info["keys"], info["xyz"], 7), device="cuda")
    d = op.diagonal(kt, out=torch.full((op.n_local,), float("nan"), dtype=torch.float64, device="cuda"))
    pr = oracle_problem("cube", 4, O.P2_DIVKGRAD, O.BC_DIRICHLET_ZERO)
    ref = pr.diagonal(coefficient(O.P2_DIVKGRAD, pr.keys, pr.xyz, 7))
    assert rel_err(d.cpu().numpy(), ref)[1] <= 1e-12


def test_batch_diagonal_equals_single():
    print("batch diag", flush=True)
    levels = [3, 0, 4, 2, 1]
    a, phi = W.fields.batch_k_params(len(levels), 10)
    v, t = W.meshes.ref_tet()
    meshes = [T.Mesh(v, t, lv) for lv in levels]
    ops = [T.Operator(mm, T.P2_DIVKGRAD, T.F64) for mm in meshes]
    ks = [torch.tensor(W.fields.batch_k(mm.dof_info(2, owner=False)["xyz"], a[i], phi[i]), device="cuda")
          for i, mm in enumerate(meshes)]
    b = T.Batch(ops)
    D = b.diagonal(b.concat(ks), out=torch.full((b.length,), float("nan"), dtype=torch.float64, device="cuda"))
    for i, (op, k) in enumerate(zip(ops, ks)):
        di = op.diagonal(k)
        part = D[b.offsets[i]:b.offsets[i + 1]]
        assert not torch.isnan(part).any()
        assert (part - di).abs().max().item() <= 1e-13 * di.abs().max().item(), i


def test_diagonal_refused_for_other_kinds():
    v, t = W.meshes.kuhn_cube()
    m = T.Mesh(v, t, 2)
    op = T.Operator(m, T.N1_CURLCURL, T.F64)
    d = torch.empty(op.n_local, dtype=torch.float64, device="cuda")
    k = torch.ones(2 * op.n_local, dtype=torch.float64, device="cuda")
    st = T.lib().tmf_diagonal(op.handle, ctypes.c_void_p(k.data_ptr()), ctypes.c_void_p(d.data_ptr()), None)
    assert st == -4  # TMF_EUNSUPPORTED


P1_AND_EPS = [("ref", 5, O.P1_LAPLACE), ("cube", 4, O.P1_LAPLACE), ("ref", 6, O.P1_DIVKGRAD), ("cube", 3, O.P1_DIVKGRAD),
              ("flatshell", 2, O.P1_DIVKGRAD), ("cube", 2, O.P2V_EPSILON), ("flatshell", 3, O.P2V_EPSILON),
              ("shell", 1, O.P2V_EPSILON), ("shell", 3, O.P2V_EPSILON)]


@pytest.mark.parametrize("mesh,level,kind", P1_AND_EPS)
@pytest.mark.parametrize("bc", [O.BC_DIRICHLET_ZERO, O.BC_NONE])
@pytest.mark.parametrize("prec", [T.F64, T.F32])
def test_p1_and_epsilon_diagonal_match_oracle(mesh, level, kind, bc, prec):
    """diag(D A D) of the P1 kinds (vertex-centric) and of the epsilon operator (per component;
    affine and radially blended maps) against the oracle."""
    from test_gpu_parity import lib_problem
    print("diag case", mesh, level, kind, bc, prec, flush=True)
    m, op = lib_problem(mesh, level, kind, bc, prec)
    info = m.dof_info(op.space, owner=False, boundary=False)
    dt = torch.float64 if prec == T.F64 else torch.float32
    k = coefficient(kind, info["keys"], info["xyz"], 7)
    kt = torch.tensor(k, dtype=dt, device="cuda") if k is not None else None
    out = torch.full((op.ncomp * op.n_local,), float("nan"), dtype=dt, device="cuda")
    d = op.diagonal(kt, out=out).double().cpu().numpy()
    assert not np.isnan(d).any()
    pr = oracle_problem(mesh, level, kind, bc)
    ref = pr.diagonal(coefficient(kind, pr.keys, pr.xyz, 7))
    e2, ei = rel_err(d, ref)
    assert ei <= (1e-12 if prec == T.F64 else 1e-5), (e2, ei)


def test_epsilon_diagonal_second_tile_shape():
    from test_gpu_parity import lib_problem
    m, op = lib_problem("shell", 2, O.P2V_EPSILON, O.BC_DIRICHLET_ZERO, T.F64)
    info = m.dof_info(2, owner=False, boundary=False)
    kt = torch.tensor(coefficient(O.P2V_EPSILON, info["keys"], info["xyz"], 7), device="cuda")
    d0 = op.diagonal(kt)
    T.check(T.lib().tmf_op_set_tile(op.handle, 1))
    d1 = op.diagonal(kt)
    assert (d0 - d1).abs().max().item() <= 1e-13 * d0.abs().max().item()
