"""Pins of the oracle's N1 operator (equation N1 of section "Curl-Curl and
Mass": alpha curl curl + beta, first-kind lowest-order Nedelec elements, alpha
and beta nodal P1).

The DoF of an edge is the tangential integral along the edge oriented by the
canonical keys of its endpoints.  Checks that do not use the element matrices:
* curl grad = 0: the interpolant of the gradient of any P1 function,
  x_e = psi(q) - psi(p), is in the kernel of the curl-curl part;
* the space reproduces u = a + b x r exactly, so with alpha = 1, beta = 0 the
  energy x.A x is int |curl u|^2 = |2 b|^2 vol, and with alpha = 0, beta = 1
  and u = a it is |a|^2 vol (on the 6-macro cube, so the orientation across
  macro interfaces enters);
* the matrix-free apply equals the sparse assembly; A is symmetric and
  positive semi-definite, with zero rows on the vertex slots.
"""
import numpy as np
import pytest

import oracle as O
from oracle.lattice import EDGES
import workloads as W


def _problem(mesh, level, bc=O.BC_NONE):
    v, t = {"ref": W.meshes.ref_tet, "cube": W.meshes.kuhn_cube}[mesh]()
    return O.Problem(v, t, level, O.N1_CURLCURL, bc)


def _edges(pr):
    """(midpoint slot, tail vertex slot, head vertex slot) of every element edge, global orientation."""
    mids, tails, heads = [], [], []
    for m, tn, P, nodes in pr.element_batches():
        for e, (a, b) in enumerate(EDGES):
            va, vb = nodes[:, a], nodes[:, b]
            up = pr.uid[va] < pr.uid[vb]
            mids.append(nodes[:, 4 + e])
            tails.append(np.where(up, va, vb))
            heads.append(np.where(up, vb, va))
    return np.concatenate(mids), np.concatenate(tails), np.concatenate(heads)


def _coeff(pr, alpha, beta):
    return np.concatenate([np.full(pr.n_local, float(alpha)), np.full(pr.n_local, float(beta))])


def _interp(pr, field):
    """Nedelec interpolant of a field linear in r: u(midpoint) . (head - tail), on every copy."""
    mid, tail, head = _edges(pr)
    x = np.zeros(pr.n_local)
    x[mid] = np.einsum("ed,ed->e", field(0.5 * (pr.xyz[tail] + pr.xyz[head])), pr.xyz[head] - pr.xyz[tail])
    return x


def _energy(pr, x, coeff):
    return pr.to_unique(x) @ pr.to_unique(pr.apply(x, coeff))


@pytest.mark.parametrize("mesh,level", [("ref", 2), ("cube", 1)])
def test_gradients_are_in_the_curl_curl_kernel(mesh, level):
    pr = _problem(mesh, level)
    rng = np.random.default_rng(0)
    psi = rng.standard_normal(pr.n_unique)[pr.uid]
    mid, tail, head = _edges(pr)
    x = np.zeros(pr.n_local)
    x[mid] = psi[head] - psi[tail]
    alpha = np.concatenate([1 + 0.5 * np.sin(pr.xyz @ np.array([1.0, 2.0, 3.0])), np.zeros(pr.n_local)])
    y = pr.apply(x, alpha)
    # scale: the same x through the mass part (beta = 1) is O(|x| h^3); the curl-curl image must vanish
    scale = np.abs(pr.apply(x, _coeff(pr, 0, 1))).max()
    assert np.abs(y).max() <= 1e-12 * max(scale, 1.0)


@pytest.mark.parametrize("mesh,level,vol", [("cube", 1, 1.0), ("ref", 2, 1.0 / 6.0)])
def test_energies_of_reproduced_fields(mesh, level, vol):
    pr = _problem(mesh, level)
    a, b = np.array([0.3, -1.1, 0.7]), np.array([0.9, 0.4, -0.6])
    x = _interp(pr, lambda r: a + np.cross(b, r))
    assert abs(_energy(pr, x, _coeff(pr, 1, 0)) - 4 * (b @ b) * vol) <= 1e-12 * (b @ b)
    xa = _interp(pr, lambda r: np.broadcast_to(a, r.shape))
    assert abs(_energy(pr, xa, _coeff(pr, 0, 1)) - (a @ a) * vol) <= 1e-12 * (a @ a)


@pytest.mark.parametrize("bc", [O.BC_NONE, O.BC_DIRICHLET_ZERO])
def test_apply_equals_assembly_symmetric_psd(bc):
    pr = _problem("cube", 1, bc)
    rng = np.random.default_rng(1)
    coeff = np.concatenate([1 + 0.5 * rng.uniform(-1, 1, pr.n_unique)[pr.uid],
                            1 + 0.5 * rng.uniform(-1, 1, pr.n_unique)[pr.uid]])
    A = pr.assemble(coeff)
    x = pr.to_local(rng.standard_normal(pr.n_unique))
    assert np.abs(pr.to_unique(pr.apply(x, coeff)) - A @ pr.to_unique(x)).max() <= 1e-13 * np.abs(A).max()
    Ad = A.toarray()
    assert np.abs(Ad - Ad.T).max() <= 1e-14 * np.abs(Ad).max()
    assert np.linalg.eigvalsh(Ad).min() >= -1e-12 * np.abs(Ad).max()
    vert = np.zeros(pr.n_unique, bool)
    vert[pr.uid[(pr.keys[:, 0] >= 0) & np.all(pr.pts[np.arange(pr.n_local) % pr.L] % 2 == 0, axis=1)]] = True
    assert np.abs(Ad[vert]).max() == 0.0
