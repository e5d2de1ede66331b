"""GPU quadrature variant of P2 div(k grad) (the under-integration option:
weights from a degree-2 rule) against the oracle's quadrature element, FP64
<= 1e-12 and FP32 <= 1e-5 relative max-norm; with a degree-5 rule the variant
equals the exactly integrated GPU operator (the integrand has degree 4).
Operations defined for the exact operator only refuse the variant."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
import paper_2404_08371_amd as T
from helpers import rel_err
import workloads as W

pytestmark = pytest.mark.gpu


def setup(level, bc, prec, rule):
    v, t = W.meshes.kuhn_cube()
    m = T.Mesh(v, t, level)
    op = T.Operator(m, T.P2_DIVKGRAD, prec, bc, rule=rule)
    info = m.dof_info(2, owner=False, boundary=False)
    dt = torch.float64 if prec == T.F64 else torch.float32
    k = torch.tensor(W.fields.cube_k(info["xyz"]), dtype=dt, device="cuda")
    x = torch.tensor(W.uniform_from_keys(6, info["keys"]), dtype=dt, device="cuda")
    return m, op, k, x


@pytest.mark.parametrize("level", [3, 4])
@pytest.mark.parametrize("bc", [O.BC_DIRICHLET_ZERO, O.BC_NONE])
@pytest.mark.parametrize("prec", [T.F64, T.F32])
def test_degree2_variant_matches_oracle(level, bc, prec):
    print("quad case", level, bc, prec, flush=True)
    rule = W.quadrature.rule_degree2()
    m, op, k, x = setup(level, bc, prec, rule)
    y = op.apply(x, k, out=torch.full_like(x, float("nan"))).double().cpu().numpy()
    assert not np.isnan(y).any()
    v, t = W.meshes.kuhn_cube()
    pr = O.Problem(v, t, level, O.P2_DIVKGRAD, bc, qbary=rule[0], qw=rule[1])
    ref = pr.apply(W.uniform_from_keys(6, pr.keys), W.fields.cube_k(pr.xyz))
    e2, ei = rel_err(y, ref)
    assert ei <= (1e-12 if prec == T.F64 else 1e-5), (e2, ei)


def test_degree5_variant_equals_exact_operator():
    m, op5, k, x = setup(4, O.BC_DIRICHLET_ZERO, T.F64, W.quadrature.rule_degree5())
    ope = T.Operator(m, T.P2_DIVKGRAD, T.F64, O.BC_DIRICHLET_ZERO)
    a, b = op5.apply(x, k), ope.apply(x, k)
    assert (a - b).abs().max().item() <= 1e-12 * b.abs().max().item()


def test_variant_refuses_exact_only_operations():
    m, op, k, x = setup(2, O.BC_DIRICHLET_ZERO, T.F64, W.quadrature.rule_degree2())
    d = torch.empty_like(x)
    L = T.lib()
    assert L.tmf_diagonal(op.handle, ctypes.c_void_p(k.data_ptr()), ctypes.c_void_p(d.data_ptr()), None) == -4
    assert L.tmf_op_store_matrices(op.handle, ctypes.c_void_p(k.data_ptr()), None) == -4
