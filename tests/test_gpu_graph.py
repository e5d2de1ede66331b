"""Applies captured into a HIP graph and replayed: every replay gives the eager
apply's result bit for bit, with eager work and synchronisations between the
replays.  The apply launches kernels only (no allocation, no memset) once an
operator's buffers exist, so it can be recorded by a caller's graph capture."""
import sys

import numpy as np
import pytest
import torch

import oracle as O
import paper_2404_08371_amd as T
from helpers import inputs
from test_gpu_parity import lib_problem

pytestmark = pytest.mark.gpu

CASES = [("ref", 4, O.P1_LAPLACE, T.F64), ("cube", 3, O.P2_DIVKGRAD, T.F64), ("cube", 3, O.P2_DIVKGRAD, T.F32),
         ("shell", 2, O.P2V_EPSILON, T.F64)]


@pytest.mark.parametrize("mesh,level,kind,prec", CASES)
def test_graph_replays_equal_eager(mesh, level, kind, prec):
    print("case", mesh, level, kind, prec, flush=True)
    sys.stdout.flush()
    m, op = lib_problem(mesh, level, kind, O.BC_DIRICHLET_ZERO, prec)
    info = m.dof_info(op.space, owner=False, boundary=False)
    x, k = inputs(kind, info["keys"], info["xyz"], 5)
    dt = torch.float64 if prec == T.F64 else torch.float32
    xt = torch.tensor(x, dtype=dt, device="cuda")
    kt = torch.tensor(k, dtype=dt, device="cuda") if k is not None else None
    ref = op.apply(xt, kt)
    y = torch.empty_like(ref)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        op.apply(xt, kt, out=y)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        op.apply(xt, kt, out=y)
        op.apply(xt, kt, out=y)
    other = torch.empty_like(ref)
    for rep in range(3):
        y.fill_(np.nan)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, ref), "replay %d differs from the eager apply" % rep
        op.apply(xt * 2, kt, out=other)  # eager work between the replays
        torch.cuda.synchronize()
        assert torch.equal(other, op.apply(xt * 2, kt))
