"""GPU N1 operator (alpha curl curl + beta, first-kind Nedelec, alpha and beta
nodal P1; equation N1 of section "Curl-Curl and Mass") against the oracle.

Edge DoFs sit at the P2-lattice midpoints and are oriented by the canonical
keys of their endpoints on both sides.  FP64: relative max-norm error
<= 1e-12; FP32: <= 1e-5 (as for the other operators).  Meshes with several
macros check the orientation across interfaces; the gradient of a P1
function must be in the kernel of the curl-curl part on the GPU as well.
Outputs start as NaN, so an unwritten slot shows.
"""
import numpy as np
import pytest
import torch

import oracle as O
import paper_2404_08371_amd as T
from helpers import MESHES, oracle_problem, rel_err
import workloads as W

pytestmark = pytest.mark.gpu


n1_coeff = W.fields.n1_coeff


def lib_n1(mesh, level, bc, prec):
    mk, mp = MESHES[mesh]
    v, t = mk()
    m = T.Mesh(v, t, level, mp)
    return m, T.Operator(m, T.N1_CURLCURL, prec, bc)


def run(mesh, level, bc, prec, cfg=None, seed=3):
    print("n1 case", mesh, level, bc, prec, cfg, flush=True)
    m, op = lib_n1(mesh, level, bc, prec)
    if cfg is not None:
        T.check(T.lib().tmf_op_set_tile(op.handle, cfg))
    info = m.dof_info(2, owner=False, boundary=False)
    dt = torch.float64 if prec == T.F64 else torch.float32
    x = W.uniform_from_keys(seed, info["keys"])
    c = n1_coeff(info["xyz"])
    y = op.apply(torch.tensor(x, dtype=dt, device="cuda"), torch.tensor(c, dtype=dt, device="cuda"),
                 out=torch.full((op.n_local,), float("nan"), dtype=dt, device="cuda"))
    y = y.double().cpu().numpy()
    assert not np.isnan(y).any()
    pr = oracle_problem(mesh, level, O.N1_CURLCURL, bc)
    ref = pr.apply(W.uniform_from_keys(seed, pr.keys), n1_coeff(pr.xyz))
    return rel_err(y, ref)


@pytest.mark.parametrize("mesh,level", [("ref", 4), ("cube", 2), ("cube", 4), ("flatshell", 2)])
@pytest.mark.parametrize("bc", [O.BC_DIRICHLET_ZERO, O.BC_NONE])
@pytest.mark.parametrize("prec", [T.F64, T.F32])
def test_n1_matches_oracle(mesh, level, bc, prec):
    e2, ei = run(mesh, level, bc, prec)
    assert ei <= (1e-12 if prec == T.F64 else 1e-5), (e2, ei)


@pytest.mark.parametrize("cfg", [0, 1, 2, 3])
def test_n1_every_tile_shape(cfg):
    e2, ei = run("cube", 4, O.BC_DIRICHLET_ZERO, T.F64, cfg)
    assert ei <= 1e-12, (e2, ei)


def test_n1_gradients_in_kernel_on_gpu():
    """x = interpolated gradient of a P1 function (built on the oracle's identical slot layout): the
    curl-curl part (beta = 0) maps it to 0 on the 6-macro cube."""
    from oracle.lattice import EDGES
    v, t = W.meshes.kuhn_cube()
    pr = O.Problem(v, t, 3, O.N1_CURLCURL, O.BC_NONE)
    psi = np.random.default_rng(5).standard_normal(pr.n_unique)[pr.uid]
    x = np.zeros(pr.n_local)
    for m, tn, P, nodes in pr.element_batches():
        for e, (a, b) in enumerate(EDGES):
            va, vb = nodes[:, a], nodes[:, b]
            up = pr.uid[va] < pr.uid[vb]
            x[nodes[:, 4 + e]] = np.where(up, psi[vb] - psi[va], psi[va] - psi[vb])
    m, op = lib_n1("cube", 3, O.BC_NONE, T.F64)
    c = n1_coeff(m.dof_info(2)["xyz"])
    c[op.n_local:] = 0.0
    y = op.apply(torch.tensor(x, device="cuda"), torch.tensor(c, device="cuda")).cpu().numpy()
    cm = c.copy()
    cm[:op.n_local], cm[op.n_local:] = 0.0, 1.0
    scale = np.abs(op.apply(torch.tensor(x, device="cuda"), torch.tensor(cm, device="cuda")).cpu().numpy()).max()
    assert np.abs(y).max() <= 1e-12 * max(scale, 1.0)
