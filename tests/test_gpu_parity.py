"""GPU parity: the HIP operators against the FP64 oracle, element by element.

Tolerances: FP64 relative error (2-norm and max-norm, relative to the
oracle's norms) <= 1e-12, the bound the target states for FP64.  FP32 applies
evaluate the same formulas with 24-bit mantissas; with O(100) accumulated
terms per output the expected relative error is ~1e-6, and the bound used is
1e-5 relative to the max-norm of y.
"""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import paper_2404_08371_amd as T
from helpers import MESHES, inputs, oracle_problem, rel_err
import workloads as W

pytestmark = pytest.mark.gpu

LIB_KIND = {O.P1_LAPLACE: T.P1_LAPLACE, O.P1_DIVKGRAD: T.P1_DIVKGRAD, O.P2_LAPLACE: T.P2_LAPLACE,
            O.P2_DIVKGRAD: T.P2_DIVKGRAD, O.P2V_EPSILON: T.P2V_EPSILON}


def lib_problem(mesh, level, kind, bc, prec, tile=None):
    mk, mp = MESHES[mesh]
    v, t = mk()
    m = T.Mesh(v, t, level, mp)
    rule = W.quadrature.rule_degree5() if mp == 1 else None
    op = T.Operator(m, LIB_KIND[kind], prec, bc, rule=rule)
    return m, op


def run_case(mesh, level, kind, bc, prec, seed=1):
    print("case", mesh, level, T.KIND_NAMES[LIB_KIND[kind]], "bc", bc, "prec", prec, flush=True)
    sys.stdout.flush()
    m, op = lib_problem(mesh, level, kind, bc, prec)
    info = m.dof_info(op.space, owner=False, boundary=False)
    x, k = inputs(kind, info["keys"], info["xyz"], seed)
    pr = oracle_problem(mesh, level, kind, bc)
    xo, ko = inputs(kind, pr.keys, pr.xyz, seed)
    assert np.array_equal(x, xo)
    dt = torch.float64 if prec == T.F64 else torch.float32
    xt = torch.tensor(x, dtype=dt, device="cuda")
    kt = torch.tensor(k, dtype=dt, device="cuda") if k is not None else None
    y = op.apply(xt, kt)
    torch.cuda.synchronize()
    ref = pr.apply(xo, ko)
    return rel_err(y.double().cpu().numpy(), ref)


CASES = []
for kind in (O.P1_LAPLACE, O.P1_DIVKGRAD):
    CASES += [("ref", l, kind) for l in (0, 1, 2, 3, 4, 5)] + [("cube", l, kind) for l in (0, 2, 3)]
    CASES += [("flatshell", 1, kind)]
for kind in (O.P2_LAPLACE, O.P2_DIVKGRAD):
    CASES += [("ref", l, kind) for l in (0, 1, 2, 3, 4)] + [("cube", l, kind) for l in (0, 1, 3)]
    CASES += [("flatshell", 1, kind)]
# epsilon: levels 3 and 4 hold several 4 x 4 x 4 tile boxes per macro, so the
# seam reduction adds partial sums of neighbouring tiles
CASES += [("cube", l, O.P2V_EPSILON) for l in (0, 1, 2, 3, 4)] + [("flatshell", l, O.P2V_EPSILON) for l in (1, 3)]
CASES += [("shell", l, O.P2V_EPSILON) for l in (0, 1, 2, 3)]


@pytest.mark.parametrize("bc", [O.BC_DIRICHLET_ZERO, O.BC_NONE])
@pytest.mark.parametrize("mesh,level,kind", CASES)
def test_fp64_parity(mesh, level, kind, bc):
    e2, ei = run_case(mesh, level, kind, bc, T.F64)
    assert e2 <= 1e-12 and ei <= 1e-12, (e2, ei)


@pytest.mark.parametrize("mesh,level,kind", [c for c in CASES if c[1] <= 3 and MESHES[c[0]][1] == 0])
def test_fp32_parity(mesh, level, kind):
    e2, ei = run_case(mesh, level, kind, O.BC_DIRICHLET_ZERO, T.F32)
    print("fp32 rel err", e2, ei)
    assert ei <= 1e-5, (e2, ei)


# tile shapes of the scalar P2 kinds: 4 boxes, then 3 marching column segments
# (2, 4 and 8 sub-boxes of 4 x 4 x 4 cubes)
ALL_TILES = list(range(7))
MARCH_TILES = [4, 5, 6]


@pytest.mark.parametrize("cfg", ALL_TILES)
@pytest.mark.parametrize("kind,prec", [(O.P2_DIVKGRAD, T.F64), (O.P2_LAPLACE, T.F64), (O.P2_DIVKGRAD, T.F32)])
def test_every_tile_shape(cfg, kind, prec):
    """Each autotuner candidate computes the same operator (level 4: 16 cubes per edge, ragged boxes)."""
    import ctypes
    print("tile case", cfg, kind, prec, flush=True)
    m, op = lib_problem("cube", 4, kind, O.BC_DIRICHLET_ZERO, prec)
    T.check(T.lib().tmf_op_set_tile(op.handle, cfg))
    info = m.dof_info(2, owner=False, boundary=False)
    x, k = inputs(kind, info["keys"], info["xyz"], 3)
    pr = oracle_problem("cube", 4, kind, O.BC_DIRICHLET_ZERO)
    dt = torch.float64 if prec == T.F64 else torch.float32
    y = op.apply(torch.tensor(x, dtype=dt, device="cuda"),
                 torch.tensor(k, dtype=dt, device="cuda") if k is not None else None)
    e2, ei = rel_err(y.double().cpu().numpy(), pr.apply(x, k))
    assert ei <= (1e-12 if prec == T.F64 else 1e-5), (e2, ei)


@pytest.mark.parametrize("mesh,level,kind", [("cube", 3, O.P2_DIVKGRAD), ("cube", 4, O.P2_LAPLACE),
                                             ("flatshell", 2, O.P2V_EPSILON), ("shell", 1, O.P2V_EPSILON)])
@pytest.mark.parametrize("bc", [O.BC_DIRICHLET_ZERO, O.BC_NONE])
def test_local_apply_then_interface_sum_is_the_apply(mesh, level, kind, bc):
    """The macro-local apply (seam reduction only) followed by the interface sum
    gives the full apply bit for bit: the same values summed in the same order.
    Outputs start as NaN, so a slot that no kernel writes (or that is read
    before it is written) shows."""
    print("local case", mesh, level, kind, bc, flush=True)
    m, op = lib_problem(mesh, level, kind, bc, T.F64)
    info = m.dof_info(op.space, owner=False, boundary=False)
    x, k = inputs(kind, info["keys"], info["xyz"], 4)
    xt = torch.tensor(x, device="cuda")
    kt = torch.tensor(k, device="cuda") if k is not None else None
    y = op.apply(xt, kt, out=torch.full_like(xt, float("nan")))
    yl = op.interface_sum_(op.apply_local(xt, kt, out=torch.full_like(xt, float("nan"))))
    assert not torch.isnan(y).any() and not torch.isnan(yl).any()
    assert torch.equal(y, yl)
    pr = oracle_problem(mesh, level, kind, bc)
    ref = pr.apply(*inputs(kind, pr.keys, pr.xyz, 4))
    for v in (y, yl):
        e2, ei = rel_err(v.cpu().numpy(), ref)
        assert e2 <= 1e-12 and ei <= 1e-12, (e2, ei)


@pytest.mark.parametrize("cfg", MARCH_TILES)
@pytest.mark.parametrize("mesh,level", [("ref", 0), ("ref", 1), ("ref", 3), ("ref", 5), ("cube", 2), ("cube", 5),
                                        ("flatshell", 3)])
@pytest.mark.parametrize("bc", [O.BC_DIRICHLET_ZERO, O.BC_NONE])
@pytest.mark.parametrize("kind,prec", [(O.P2_DIVKGRAD, T.F64), (O.P2_LAPLACE, T.F64), (O.P2_DIVKGRAD, T.F32)])
def test_marching_tiles(cfg, mesh, level, bc, kind, prec):
    """The marching kernel on single macros and multi-macro meshes at levels where a segment holds
    one sub-box (levels 0-2), where segments are cut short by the macro's diagonal face, and where
    several segments stack in z (level 5: 32 cubes per edge), with both boundary conditions.  Outputs
    start as NaN, so a slot that no kernel writes shows."""
    print("march case", cfg, mesh, level, bc, kind, prec, flush=True)
    m, op = lib_problem(mesh, level, kind, bc, prec)
    T.check(T.lib().tmf_op_set_tile(op.handle, cfg))
    info = m.dof_info(2, owner=False, boundary=False)
    x, k = inputs(kind, info["keys"], info["xyz"], 8)
    dt = torch.float64 if prec == T.F64 else torch.float32
    xt = torch.tensor(x, dtype=dt, device="cuda")
    y = op.apply(xt, torch.tensor(k, dtype=dt, device="cuda") if k is not None else None,
                 out=torch.full_like(xt, float("nan")))
    assert not torch.isnan(y).any()
    pr = oracle_problem(mesh, level, kind, bc)
    e2, ei = rel_err(y.double().cpu().numpy(), pr.apply(*inputs(kind, pr.keys, pr.xyz, 8)))
    assert ei <= (1e-12 if prec == T.F64 else 1e-5), (e2, ei)


@pytest.mark.parametrize("cfg", ALL_TILES)
def test_repeated_applies_agree(cfg):
    """Every entry of y is written by exactly one thread (outputs start as NaN),
    and repeated applies agree bit for bit: every sum (in-box accumulation,
    seam and interface reductions) is formed in a fixed order."""
    print("repeat case", cfg, flush=True)
    m, op = lib_problem("cube", 5, O.P2_DIVKGRAD, O.BC_DIRICHLET_ZERO, T.F64)
    T.check(T.lib().tmf_op_set_tile(op.handle, cfg))
    info = m.dof_info(2, owner=False, boundary=False)
    x, k = inputs(O.P2_DIVKGRAD, info["keys"], info["xyz"], 5)
    xt, kt = torch.tensor(x, device="cuda"), torch.tensor(k, device="cuda")
    y0 = op.apply(xt, kt, out=torch.full_like(xt, float("nan")))
    assert not torch.isnan(y0).any()
    for _ in range(5):
        y = op.apply(xt, kt, out=torch.full_like(xt, float("nan")))
        assert torch.equal(y, y0)


@pytest.mark.parametrize("mesh,level,kind,prec", [("shell", 2, O.P2V_EPSILON, T.F64), ("shell", 2, O.P2V_EPSILON, T.F32),
                                                  ("cube", 4, O.P2_LAPLACE, T.F32), ("flatshell", 3, O.P2V_EPSILON, T.F64)])
def test_repeated_applies_are_bitwise_equal(mesh, level, kind, prec):
    """Bit-for-bit repeats for the vector operator (4 wavefronts per box) and FP32."""
    print("repeat case", mesh, level, kind, prec, flush=True)
    m, op = lib_problem(mesh, level, kind, O.BC_DIRICHLET_ZERO, prec)
    info = m.dof_info(2, owner=False, boundary=False)
    x, k = inputs(kind, info["keys"], info["xyz"], 6)
    dt = torch.float64 if prec == T.F64 else torch.float32
    xt = torch.tensor(x, dtype=dt, device="cuda")
    kt = torch.tensor(k, dtype=dt, device="cuda") if k is not None else None
    y0 = op.apply(xt, kt)
    for _ in range(4):
        assert torch.equal(op.apply(xt, kt), y0)
