"""Pins of the oracle's quadrature variant of P2 div(k grad) (the paper's
under-integration option of section "Variable-Coefficient Diffusion": the
degree-4 integrand k grad(phi_i).grad(phi_j) with a degree-2 rule).

* A rule exact to degree 5 reproduces the exact element matrices; the
  degree-2 rule does so for constant k (the integrand is then quadratic) and
  differs for variable k.
* Convergence on a manufactured solution (u = sin(pi x) sin(pi y) sin(pi z) on
  the unit cube, k = 1 + xyz/2, f = -div(k grad u), load vector with the
  degree-5 rule, direct solve, nodal max-norm error at levels 1..3): the
  degree-2 rule keeps the rate of exact integration, while a rule exact only
  for linear polynomials (the 4 vertices) loses it, as the paper reports.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from oracle import elements as el
import workloads as W

VERTEX_RULE = (np.eye(4), np.full(4, 1.0 / 24.0))


def _P(seed=0):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((50, 4, 3))


def test_degree5_rule_reproduces_exact_element():
    P = _P()
    k = np.random.default_rng(1).uniform(0.5, 1.5, (50, 10))
    A = el.p2_divkgrad(P, k)
    Aq = el.p2_divkgrad_quad(P, k, *W.quadrature.rule_degree5())
    assert np.abs(A - Aq).max() <= 1e-12 * np.abs(A).max()


def test_degree2_rule_exact_for_constant_k_only():
    P = _P(2)
    kc = np.full((50, 10), 1.7)
    A = el.p2_divkgrad(P, kc)
    assert np.abs(A - el.p2_divkgrad_quad(P, kc, *W.quadrature.rule_degree2())).max() <= 1e-12 * np.abs(A).max()
    kv = np.random.default_rng(3).uniform(0.5, 1.5, (50, 10))
    d = np.abs(el.p2_divkgrad(P, kv) - el.p2_divkgrad_quad(P, kv, *W.quadrature.rule_degree2())).max()
    assert d > 1e-6 * np.abs(el.p2_divkgrad(P, kv)).max()


def _f(x):
    pi = np.pi
    s, c = np.sin(pi * x), np.cos(pi * x)
    u = s[..., 0] * s[..., 1] * s[..., 2]
    gu = pi * np.stack([c[..., 0] * s[..., 1] * s[..., 2], s[..., 0] * c[..., 1] * s[..., 2],
                        s[..., 0] * s[..., 1] * c[..., 2]], -1)
    gk = 0.5 * np.stack([x[..., 1] * x[..., 2], x[..., 0] * x[..., 2], x[..., 0] * x[..., 1]], -1)
    return -((gk * gu).sum(-1) - 3 * pi ** 2 * (1 + 0.5 * x[..., 0] * x[..., 1] * x[..., 2]) * u)


def _nodal_error(level, rule):
    v, t = W.meshes.kuhn_cube()
    kw = {} if rule is None else dict(qbary=rule[0], qw=rule[1])
    pr = O.Problem(v, t, level, O.P2_DIVKGRAD, O.BC_DIRICHLET_ZERO, **kw)
    X = pr.xyz
    k = 1 + 0.5 * X[:, 0] * X[:, 1] * X[:, 2]
    qb, qw = W.quadrature.rule_degree5()
    vals, _ = el.p2_eval(qb)
    b = np.zeros(pr.n_local)
    for m, tn, P, nodes in pr.element_batches():
        vol, _ = el.geometry(P)
        be = 6 * vol[:, None] * np.einsum("q,eq,qi->ei", qw, _f(np.einsum("qa,ead->eqd", qb, P)), vals)
        b += np.bincount(nodes.ravel(), weights=be.ravel(), minlength=b.size)
    bu = pr.to_unique(pr._mask(pr.interface_sum(b)))
    A = pr.assemble(k)
    inner = pr.to_unique(pr.interior.astype(float)) > 0
    uu = np.zeros(pr.n_unique)
    uu[inner] = spla.spsolve(A[inner][:, inner].tocsc(), bu[inner])
    ue = pr.to_unique(np.sin(np.pi * X[:, 0]) * np.sin(np.pi * X[:, 1]) * np.sin(np.pi * X[:, 2]))
    return np.abs(uu - ue).max()


def _rate(rule):
    e = [_nodal_error(lv, rule) for lv in (1, 2, 3)]
    return np.log2(e[1] / e[2])


def test_degree2_rule_keeps_the_convergence_rate():
    r_exact, r_u = _rate(None), _rate(W.quadrature.rule_degree2())
    r_lin = _rate(VERTEX_RULE)
    print("rates: exact %.2f, degree 2 %.2f, vertex rule %.2f" % (r_exact, r_u, r_lin))
    assert r_exact >= 3.5 and abs(r_u - r_exact) <= 0.1
    assert r_lin <= 2.0
