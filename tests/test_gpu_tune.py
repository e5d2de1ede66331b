"""The autotuner's result cache (tmf_op_tune / tmf_batch_tune) and the
epsilon operator's second tile shape."""
import json

import numpy as np
import pytest
import torch

import oracle as O
import paper_2404_08371_amd as T
from helpers import inputs, oracle_problem, rel_err
import workloads as W

pytestmark = pytest.mark.gpu


def cube_op(level=4, prec=T.F64):
    v, t = W.meshes.kuhn_cube()
    m = T.Mesh(v, t, level)
    op = T.Operator(m, T.P2_DIVKGRAD, prec)
    info = m.dof_info(2, owner=False, boundary=False)
    dt = op.dtype
    x = torch.tensor(W.uniform_from_keys(3, info["keys"]), dtype=dt, device="cuda")
    k = torch.tensor(W.fields.cube_k(info["xyz"]), dtype=dt, device="cuda")
    return op, x, k


def test_op_tune_cache_roundtrip(tmp_path):
    print("tune cache op", flush=True)
    path = str(tmp_path / "tiles.json")
    op, x, k = cube_op()
    cfg, ms = op.tune(x, k, reps=2, cache=path)
    data = json.load(open(path))
    assert len(data) == 1
    (key, ent), = data.items()
    assert "level=4" in key and "macros=6" in key and "gfx950" in key
    assert ent["cfg"] == cfg and 0 <= ent["box"] < 4
    # a fresh operator of the same problem takes the cached shapes without timing
    op2, x2, k2 = cube_op()
    cfg2, ms2 = op2.tune(x2, k2, reps=2, cache=path)
    assert cfg2 == cfg and abs(ms2 - ent["ms"]) <= 1e-6 * max(1.0, ent["ms"])
    y = op2.apply(x2, k2)
    assert torch.equal(y, op.apply(x, k))
    # another level adds an entry
    op3, x3, k3 = cube_op(level=3, prec=T.F32)
    op3.tune(x3, k3, reps=2, cache=path)
    assert len(json.load(open(path))) == 2


def test_tune_cache_rejects_foreign_file(tmp_path):
    path = tmp_path / "bad.json"
    path.write_text("[1, 2, 3]")
    op, x, k = cube_op(level=2)
    with pytest.raises(T.TetmfError):
        op.tune(x, k, reps=1, cache=str(path))


def test_batch_tune_cache(tmp_path):
    print("tune cache batch", flush=True)
    path = str(tmp_path / "tiles.json")
    v, t = W.meshes.ref_tet()
    ops = [T.Operator(T.Mesh(v, t, lv), T.P2_DIVKGRAD, T.F32) for lv in (3, 4, 2)]
    b = T.Batch(ops)
    X = torch.rand(b.length, dtype=torch.float32, device="cuda")
    K = 1 + torch.rand(b.length, dtype=torch.float32, device="cuda")
    cfg, ms = b.tune(X, K, reps=2, cache=path)
    (key, ent), = json.load(open(path)).items()
    assert "levels=3:1,4:1,2:1" in key and ent["cfg"] == cfg
    b2 = T.Batch([T.Operator(T.Mesh(v, t, lv), T.P2_DIVKGRAD, T.F32) for lv in (3, 4, 2)])
    cfg2, _ = b2.tune(X, K, reps=2, cache=path)
    assert cfg2 == cfg


@pytest.mark.parametrize("mesh,level,prec", [("shell", 2, T.F64), ("flatshell", 3, T.F64), ("cube", 3, T.F64),
                                             ("shell", 2, T.F32)])
def test_epsilon_second_tile_shape(mesh, level, prec):
    """The 8 x 4 x 2 box of the epsilon kernels against the oracle (affine and blended maps)."""
    from test_gpu_parity import lib_problem
    print("eps tile 1", mesh, level, prec, flush=True)
    m, op = lib_problem(mesh, level, O.P2V_EPSILON, O.BC_DIRICHLET_ZERO, prec)
    T.check(T.lib().tmf_op_set_tile(op.handle, 1))
    info = m.dof_info(2, owner=False, boundary=False)
    x, k = inputs(O.P2V_EPSILON, info["keys"], info["xyz"], 9)
    dt = torch.float64 if prec == T.F64 else torch.float32
    y = op.apply(torch.tensor(x, dtype=dt, device="cuda"), torch.tensor(k, dtype=dt, device="cuda"))
    pr = oracle_problem(mesh, level, O.P2V_EPSILON, O.BC_DIRICHLET_ZERO)
    e2, ei = rel_err(y.double().cpu().numpy(), pr.apply(*inputs(O.P2V_EPSILON, pr.keys, pr.xyz, 9)))
    assert ei <= (1e-12 if prec == T.F64 else 1e-5), (e2, ei)


def test_epsilon_second_tile_shape_gradients():
    """dL/dx and dL/dmu with the 8 x 4 x 2 box on the blended shell at level 3 (several boxes per macro)."""
    from test_gpu_adjoint import eps_problem
    print("eps tile 1 gradients", flush=True)
    m, op, info, mu, x, b = eps_problem("shell", 3)
    gy = torch.tensor(b, device="cuda")
    mt, xt = torch.tensor(mu, device="cuda"), torch.tensor(x, device="cuda")
    gx0, gm0 = op.adjoint(mt, xt, gy)
    T.check(T.lib().tmf_op_set_tile(op.handle, 1))
    gx1, gm1 = op.adjoint(mt, xt, gy)
    for a0, a1 in ((gx0, gx1), (gm0, gm1)):
        assert (a0 - a1).abs().max().item() <= 1e-12 * a0.abs().max().item()
