"""The algebraic forms the element kernels evaluate, checked on the CPU
against the definitions they replace (no kernel code runs here; the GPU
parity tests compare the kernels themselves with the oracle).

* P2 div(k grad): the exact weights W_ce = (1/|T|) int k lambda_c lambda_e
  for nodal P2 k, evaluated as 840 W_ce = 4 k_ce + b_c + b_e (c != e),
  840 W_cc = 4 (b_c + 2 k_c), b_c = k_c + 4 E_c + h, h = sum E - 3 V / 2
  (V: sum of vertex values, E_c: sum of the edge values at vertex c),
  against exact monomial integration (int lambda^g = 6 |T| g! / (|g| + 3)!).
* Gradients of P2 fields as P1 fields: ref-grad u(q) = sum_a lambda_a(q) sp[a]
  with the gradient coefficients s[a][a] = 3 u_a, s[a][b] = 4 u_ab - u_b,
  sp[a][r] = s[a][r+1] - s[a][0]; and the output rule
  sum_q S_q . ref-grad phi_i(q) = Y(sigma), sigma[a][b] = T_a . ref-grad lambda_b,
  T_a = sum_q lambda_a(q) S_q (vertex b: 4 sigma[b][b] - sum_a sigma[a][b];
  edge bc: 4 (sigma[c][b] + sigma[b][c])), against the oracle's P2 basis.
* The radially blended shell map: DPhi = a0 I + xi v^T with v . xi = 0, so
  DPhi^-1 = (I - xi v^T / a0) / a0 and det DPhi = a0^3, against the oracle's
  map derivative inverted by LAPACK.
* The coefficient gradient of the P2 div(k grad) form, gk_b = W(e_b) : M, in
  the closed form of the derivative of the collected weights, against the
  exact weights of each unit coefficient vector.
"""
from fractions import Fraction
from math import factorial

import numpy as np
import pytest

import oracle.elements as E

EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]


def _mono_int(g):
    """(1/|T|) int_T prod lambda_a^g_a, exactly."""
    return Fraction(6 * np.prod([factorial(x) for x in g]), factorial(sum(g) + 3))


def _weights_exact(k):
    """(1/|T|) int (sum_b k_b phi_b) lambda_c lambda_e, P2 basis in monomials."""
    k = [Fraction(x) for x in k]
    W = [[Fraction(0)] * 4 for _ in range(4)]
    for c in range(4):
        for e in range(4):
            def term(g, coef):
                gg = list(g)
                gg[c] += 1
                gg[e] += 1
                return coef * _mono_int(gg)
            acc = Fraction(0)
            for b in range(4):  # phi_b = 2 lambda_b^2 - lambda_b
                g2 = [0] * 4
                g2[b] = 2
                g1 = [0] * 4
                g1[b] = 1
                acc += k[b] * (term(g2, 2) - term(g1, 1))
            for j, (a, b) in enumerate(EDGES):  # phi_ab = 4 lambda_a lambda_b
                g = [0] * 4
                g[a] += 1
                g[b] += 1
                acc += k[4 + j] * term(g, 4)
            W[c][e] = acc
    return W


def _weights_collected(k):
    E_ = [k[4] + k[5] + k[6], k[4] + k[7] + k[8], k[5] + k[7] + k[9], k[6] + k[8] + k[9]]
    V = k[0] + k[1] + k[2] + k[3]
    h = sum(E_) - Fraction(3, 2) * V
    b = [k[c] + 4 * E_[c] + h for c in range(4)]
    W = [[None] * 4 for _ in range(4)]
    for c in range(4):
        W[c][c] = 4 * (b[c] + 2 * k[c]) / 840
    for j, (c, d) in enumerate(EDGES):
        W[c][d] = W[d][c] = (4 * k[4 + j] + b[c] + b[d]) / 840
    return W


@pytest.mark.parametrize("seed", range(4))
def test_collected_p2_weights_equal_exact_integrals(seed):
    rng = np.random.default_rng(seed)
    k = [Fraction(int(v), 7) for v in rng.integers(-20, 21, 10)]
    assert _weights_collected(k) == _weights_exact(k)


def _grad_coeffs(u):
    s = np.zeros((4, 4))
    for a in range(4):
        s[a, a] = 3 * u[a]
    for j, (a, b) in enumerate(EDGES):
        s[a, b] = 4 * u[4 + j] - u[b]
        s[b, a] = 4 * u[4 + j] - u[a]
    return s[:, 1:] - s[:, :1]


def _random_bary(rng, n):
    lam = rng.random((n, 4))
    return lam / lam.sum(1, keepdims=True)


def test_p2_gradient_is_p1_in_lambda():
    rng = np.random.default_rng(1)
    lam = _random_bary(rng, 9)
    _, dv = E.p2_eval(lam)
    dref = dv[:, :, 1:] - dv[:, :, :1]  # reference gradients (nq, 10, 3)
    for _ in range(3):
        u = rng.standard_normal(10)
        sp = _grad_coeffs(u)
        assert np.allclose(lam @ sp, np.einsum("i,qir->qr", u, dref), rtol=0, atol=1e-13)


def test_p2_output_rule_from_lambda_weighted_sums():
    rng = np.random.default_rng(2)
    lam = _random_bary(rng, 7)
    S = rng.standard_normal((7, 3))
    _, dv = E.p2_eval(lam)
    dref = dv[:, :, 1:] - dv[:, :, :1]
    direct = np.einsum("qr,qir->i", S, dref)
    T = lam.T @ S  # T_a = sum_q lambda_a(q) S_q
    gl = np.vstack([-np.ones(3), np.eye(3)])  # reference gradients of lambda_0..3
    sig = T @ gl.T  # sigma[a][b] = T_a . grad lambda_b
    y = np.zeros(10)
    for b in range(4):
        y[b] = 4 * sig[b, b] - sig[:, b].sum()
    for j, (b, c) in enumerate(EDGES):
        y[4 + j] = 4 * (sig[c, b] + sig[b, c])
    assert np.allclose(y, direct, rtol=0, atol=1e-12)


def test_shell_map_derivative_closed_form_inverse():
    rng = np.random.default_rng(3)
    for _ in range(50):
        s = rng.choice([-1.0, 1.0], 3)
        xi = s * rng.uniform(0.05, 1.0, 3)  # a point of the octant of s
        D = E.shell_jacobian(xi, s)
        n = np.linalg.norm(xi)
        rho = s @ xi
        a0 = rho / n
        v = s / n - rho * xi / n ** 3
        # v . xi = rho/n - rho/n: zero up to the rounding of terms of size a0
        assert abs(v @ xi) <= 1e-14 * a0
        Dinv = (np.eye(3) - np.outer(xi, v) / a0) / a0
        assert np.allclose(Dinv, np.linalg.inv(D), rtol=0, atol=1e-13 * np.abs(Dinv).max())
        assert np.isclose(np.linalg.det(D), a0 ** 3, rtol=1e-13)


def _gradk_collected(M):
    """d(gy . y)/dk for gy . y = sum_ce W(k)_ce M_ce, from the collected weights:
    840 gk_c = Z_c + 8 M_cc - 3/2 sum Z, 840 gk_ce = 4 P_ce + 4 (Z_c + Z_e) + 2 sum Z,
    P_ce = M_ce + M_ec, Z_c = sum_{e != c} P_ce + 4 M_cc."""
    P = M + M.T
    Z = np.array([sum(P[c, e] for e in range(4) if e != c) + 4 * M[c, c] for c in range(4)])
    g = np.zeros(10)
    for c in range(4):
        g[c] = Z[c] + 8 * M[c, c] - 1.5 * Z.sum()
    for j, (c, e) in enumerate(EDGES):
        g[4 + j] = 4 * P[c, e] + 4 * (Z[c] + Z[e]) + 2 * Z.sum()
    return g / 840


def test_coefficient_gradient_of_collected_weights():
    rng = np.random.default_rng(4)
    for _ in range(3):
        M = rng.standard_normal((4, 4))
        want = np.zeros(10)
        for b in range(10):
            kb = [Fraction(int(i == b)) for i in range(10)]
            Wb = np.array([[float(x) for x in row] for row in _weights_exact(kb)])
            want[b] = (Wb * M).sum()
        assert np.allclose(_gradk_collected(M), want, rtol=0, atol=1e-14 * np.abs(want).max())
