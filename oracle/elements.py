"""Oracle: element matrices of the operators, in FP64, from their definitions.

Test infrastructure only: the product library never imports this package.

Equation (4.1) of section "Matrix-Free Finite Elements" writes the operator
as a sum of local operators A_T; this module computes A_T (row = test
function j, column = trial function i) for

* P1  : integrand grad(phi_i).grad(phi_j)                 (equation P1)
* P1k : k grad(phi_i).grad(phi_j), k nodal P1             (k in K = P1, as the
                                                          curl-curl study uses)
* P2  : grad(phi_i).grad(phi_j), P2 Lagrange              (P2, constant coefficient)
* P2k : k grad(phi_i).grad(phi_j), k nodal P2             (equation P2V)
* EPS : 2 mu eps(u):eps(v), eps = sym grad, vector P2, mu nodal P2
        (the symmetric-gradient operator; not in the paper, textbook definition)
* N1  : alpha curl(phi_i).curl(phi_j) + beta phi_i.phi_j, first-kind
        lowest-order Nedelec elements, alpha and beta nodal P1 (equation N1 of
        section "Curl-Curl and Mass")

All signs are those of positive semi-definite stiffness matrices, as the
paper's local-matrix equations define them.

Basis functions are polynomials in the barycentric coordinates lambda_0..3:
P1 phi_a = lambda_a; P2 vertex phi_a = lambda_a (2 lambda_a - 1), P2 edge
phi_ab = 4 lambda_a lambda_b with edges ordered 01,02,03,12,13,23.  With
grad(phi) = sum_a (d phi / d lambda_a) grad(lambda_a), every affine-element
integral reduces to integrals of barycentric monomials, which are exact:

    int_T lambda^alpha = 6 |T| alpha! / (|alpha| + 3)!

so the affine element matrices below are exact rationals times geometry
(the exact degree-4 integration the P2V study calls for).  The blended
(curved) shell element has no such closed form; it is integrated with a
given quadrature rule, which is part of that operator's definition.
"""
from fractions import Fraction
from math import factorial

import numpy as np

from .lattice import EDGES

# ---------------------------------------------------------------- polynomials
# polynomial = dict {exponent tuple (a0,a1,a2,a3): Fraction}


def _mono(e, c=1):
    return {tuple(e): Fraction(c)}


def _lam(a):
    e = [0, 0, 0, 0]
    e[a] = 1
    return _mono(e)


def _add(p, q, s=1):
    r = dict(p)
    for k, v in q.items():
        r[k] = r.get(k, 0) + s * v
    return {k: v for k, v in r.items() if v != 0}


def _scale(p, s):
    return {k: v * s for k, v in p.items()}


def _mul(p, q):
    r = {}
    for k1, v1 in p.items():
        for k2, v2 in q.items():
            k = tuple(a + b for a, b in zip(k1, k2))
            r[k] = r.get(k, 0) + v1 * v2
    return {k: v for k, v in r.items() if v != 0}


def _diff(p, a):
    r = {}
    for k, v in p.items():
        if k[a] > 0:
            e = list(k)
            e[a] -= 1
            r[tuple(e)] = r.get(tuple(e), 0) + v * k[a]
    return r


def bary_integral(p):
    """(1/|T|) int_T p for a polynomial p in barycentric coordinates (exact)."""
    s = Fraction(0)
    for e, v in p.items():
        num = 6
        for a in e:
            num *= factorial(a)
        s += v * Fraction(num, factorial(sum(e) + 3))
    return s


def p1_basis():
    return [_lam(a) for a in range(4)]


def p2_basis():
    basis = []
    for a in range(4):
        basis.append(_add(_scale(_mul(_lam(a), _lam(a)), 2), _lam(a), -1))
    for a, b in EDGES:
        basis.append(_scale(_mul(_lam(a), _lam(b)), 4))
    return basis


def _tensors():
    P2 = p2_basis()
    dP2 = [[_diff(f, a) for a in range(4)] for f in P2]
    # C0[i,j,a,b] = (1/|T|) int d_a phi_i d_b phi_j
    C0 = np.zeros((10, 10, 4, 4))
    # CM[m,i,j,a,b] = (1/|T|) int phi_m d_a phi_i d_b phi_j
    CM = np.zeros((10, 10, 10, 4, 4))
    for i in range(10):
        for j in range(10):
            for a in range(4):
                for b in range(4):
                    prod = _mul(dP2[i][a], dP2[j][b])
                    C0[i, j, a, b] = float(bary_integral(prod))
                    for m in range(10):
                        CM[m, i, j, a, b] = float(bary_integral(_mul(P2[m], prod)))
    # mass-type integrals used by pins
    int_phi = np.array([float(bary_integral(f)) for f in P2])
    return C0, CM, int_phi


P2_C0, P2_CM, P2_INT_PHI = _tensors()


# ------------------------------------------------------------------- geometry

def geometry(P):
    """Affine-element geometry of vertex positions P (...,4,3).

    Returns (vol, grads): |T| (...) and the barycentric gradients (...,4,3);
    grad(lambda_1..3) are the rows of J^-1 with J = [P1-P0, P2-P0, P3-P0] as
    columns, grad(lambda_0) = -(their sum).
    """
    P = np.asarray(P, dtype=np.float64)
    J = np.stack([P[..., 1, :] - P[..., 0, :], P[..., 2, :] - P[..., 0, :],
                  P[..., 3, :] - P[..., 0, :]], -1)
    det = np.linalg.det(J)
    Jinv = np.linalg.inv(J)
    g = np.concatenate([-Jinv.sum(-2, keepdims=True), Jinv], -2)
    return np.abs(det) / 6.0, g


# ------------------------------------------------------------ element matrices

def p1_laplace(P):
    vol, g = geometry(P)
    return vol[..., None, None] * np.einsum("...ad,...bd->...ab", g, g)


def p1_divkgrad(P, k):
    """k nodal P1 (...,4): int k grad(l_i).grad(l_j) = (|T| mean(k)) grad(l_i).grad(l_j)."""
    return np.asarray(k).mean(-1)[..., None, None] * p1_laplace(P)


def p2_laplace(P):
    vol, g = geometry(P)
    G = np.einsum("...ad,...bd->...ab", g, g)
    # A[j,i] = |T| sum_ab G_ab C0[i,j,a,b]
    return vol[..., None, None] * np.einsum("...ab,ijab->...ji", G, P2_C0)


def p2_divkgrad(P, k):
    vol, g = geometry(P)
    G = np.einsum("...ad,...bd->...ab", g, g)
    # per element: sum_ab G_ab CM[m,i,j,a,b] -> (...,m,i,j), then contract with k_m
    T = np.einsum("...ab,mijab->...mji", G, P2_CM)
    return vol[..., None, None] * np.einsum("...m,...mji->...ji", np.asarray(k), T)


def p2_divkgrad_quad(P, k, qbary, qw):
    """P2 div(k grad) integrated with a quadrature rule on the reference tet
    (weights summing to 1/6): A_ji = 6 |T| sum_q w_q k(q) grad(phi_i).grad(phi_j) at q,
    k nodal P2.  Exact for rules of degree >= 4; the paper's under-integrated
    variant uses a degree-2 rule (section "Variable-Coefficient Diffusion")."""
    vol, g = geometry(P)
    vals, dv = p2_eval(qbary)                       # (nq,10), (nq,10,4)
    kq = np.einsum("...m,qm->...q", np.asarray(k), vals)
    grads = np.einsum("qia,...ad->...qid", dv, g)    # (...,nq,10,3)
    A = np.einsum("q,...q,...qjd,...qid->...ji", np.asarray(qw), kq, grads, grads)
    return 6.0 * vol[..., None, None] * A


def _strain_pairs(g):
    """S[a,c,b,d] = 2 sym(e_c (x) g_a) : sym(e_d (x) g_b) for gradient vectors g (...,4,3)."""
    eye = np.eye(3)
    # E[a,c] = sym(e_c (x) g_a): (...,4,3,3,3) indexed [a, c, r, s]
    outer = np.einsum("cr,...as->...acrs", eye, g)
    E = 0.5 * (outer + np.swapaxes(outer, -1, -2))
    return 2.0 * np.einsum("...acrs,...bdrs->...acbd", E, E)


def eps_affine(P, mu):
    """Vector P2 epsilon operator on an affine element; DoF index = component*10 + node."""
    vol, g = geometry(P)
    # Mmu[i,j,a,b] = int mu d_a phi_i d_b phi_j
    Mmu = vol[..., None, None, None, None] * np.einsum("...m,mijab->...ijab", np.asarray(mu), P2_CM)
    S = _strain_pairs(g)
    A = np.einsum("...ijab,...acbd->...djci", Mmu, S)  # rows (d,j), cols (c,i)
    sh = A.shape[:-4]
    return A.reshape(sh + (30, 30))


def _lambda3():
    """I3[m,p,q] = (1/|T|) int lambda_m lambda_p lambda_q (exact)."""
    I3 = np.zeros((4, 4, 4))
    for m in range(4):
        for p in range(4):
            for q in range(4):
                I3[m, p, q] = float(bary_integral(_mul(_mul(_lam(m), _lam(p)), _lam(q))))
    return I3


N1_I3 = _lambda3()


def n1_curlcurl_mass(P, alpha, beta):
    """Nedelec (first kind, lowest order) element matrix of
    int alpha curl(phi_i).curl(phi_j) + beta phi_i.phi_j, edges i = (a, b) in
    the order 01,02,03,12,13,23, each oriented from a to b:
        phi_ab = lambda_a grad(lambda_b) - lambda_b grad(lambda_a),
        curl phi_ab = 2 grad(lambda_a) x grad(lambda_b),
    alpha, beta nodal P1 (...,4).  alpha enters the constant curl product
    through its mean; beta phi_i.phi_j is a cubic in the barycentrics."""
    vol, g = geometry(P)
    alpha, beta = np.asarray(alpha, float), np.asarray(beta, float)
    G = np.einsum("...ad,...bd->...ab", g, g)
    curls = np.stack([2.0 * np.cross(g[..., a, :], g[..., b, :]) for a, b in EDGES], -2)  # (...,6,3)
    K = alpha.mean(-1)[..., None, None] * np.einsum("...id,...jd->...ij", curls, curls)
    # B3[p,q] = (1/|T|) int beta lambda_p lambda_q
    B3 = np.einsum("...m,mpq->...pq", beta, N1_I3)
    M = np.empty(K.shape)
    for i, (a, b) in enumerate(EDGES):
        for j, (c, d) in enumerate(EDGES):
            M[..., i, j] = (B3[..., a, c] * G[..., b, d] - B3[..., a, d] * G[..., b, c]
                            - B3[..., b, c] * G[..., a, d] + B3[..., b, d] * G[..., a, c])
    return vol[..., None, None] * (K + M)


# ------------------------------------------------- reference-element evaluation

def p2_eval(bary):
    """P2 basis values (nq,10) and barycentric partials (nq,10,4) at points bary (nq,4)."""
    bary = np.asarray(bary, dtype=np.float64)
    basis = p2_basis()
    vals = np.zeros((bary.shape[0], 10))
    dv = np.zeros((bary.shape[0], 10, 4))

    def ev(p):
        out = np.zeros(bary.shape[0])
        for e, c in p.items():
            out += float(c) * np.prod(bary ** np.array(e), axis=1)
        return out

    for i, f in enumerate(basis):
        vals[:, i] = ev(f)
        for a in range(4):
            dv[:, i, a] = ev(_diff(f, a))
    return vals, dv


def shell_jacobian(xi, s):
    """Derivative of the radial map Phi(xi) = xi (s.xi)/|xi| at xi (...,3); s = octant signs."""
    xi = np.asarray(xi, dtype=np.float64)
    nrm = np.linalg.norm(xi, axis=-1)[..., None, None]
    rho = (xi @ s)[..., None, None]
    eye = np.eye(3)
    return (rho / nrm) * eye + xi[..., :, None] * (s[None, :] / nrm - rho * xi[..., None, :] / nrm ** 3)


def blended_jacobians(Pxi, s, qbary, dmap=None):
    """Jacobians of the composed element map at the points of a rule.

    Section "Tabulation of Factors of the Weak Form" (remark on curvilinear
    elements): a curved element is the image Phi(F_T(x)) of the reference
    tet, F_T the affine map of the flat micro-tet with vertices Pxi (...,4,3)
    and Phi the blending map.  By the chain rule its Jacobian at the
    reference point x_q is J_q = DPhi(xi_q) J_T with xi_q = F_T(x_q) (the
    point's position in the flat mesh) and J_T = [P1-P0, P2-P0, P3-P0].
    Returns J (...,nq,3,3).  `dmap(xi)` overrides DPhi (default: the radial
    shell map with octant signs s).
    """
    if dmap is None:
        dmap = lambda xi: shell_jacobian(xi, s)
    Pxi = np.asarray(Pxi, dtype=np.float64)
    JT = np.stack([Pxi[..., 1, :] - Pxi[..., 0, :], Pxi[..., 2, :] - Pxi[..., 0, :],
                   Pxi[..., 3, :] - Pxi[..., 0, :]], -1)
    out = []
    for q in range(len(qbary)):
        xi = np.einsum("a,...ad->...d", qbary[q], Pxi)
        out.append(dmap(xi) @ JT)
    return np.stack(out, -3)


def eps_blended(Pxi, mu, s, qbary, qw, dmap=None):
    """Vector P2 epsilon operator on a curved element of the radially blended shell.

    Pxi (...,4,3): element vertices in the flat (parametric) mesh; the physical
    element is Phi(F_T(ref)).  At each quadrature point x_q of the reference
    tet the Jacobian is J = DPhi(F_T(x_q)) J_T (blended_jacobians), the weight
    w_q |det J|, physical gradients grad(phi) = J^-T ref-grad(phi), and
    mu_q = sum_m mu_m phi_m(x_q).
    `dmap(xi)` overrides the map derivative (default: the radial shell map).
    """
    Pxi = np.asarray(Pxi, dtype=np.float64)
    Jall = blended_jacobians(Pxi, s, qbary, dmap)
    vals, dv = p2_eval(qbary)
    # reference gradients: d/dx_r = d/dlambda_r - d/dlambda_0 (r = 1..3)
    dref = dv[:, :, 1:] - dv[:, :, :1]  # (nq,10,3)
    sh = Pxi.shape[:-2]
    A = np.zeros(sh + (30, 30))
    eye = np.eye(3)
    for q in range(len(qw)):
        J = Jall[..., q, :, :]
        det = np.abs(np.linalg.det(J))
        Jinv = np.linalg.inv(J)
        grad = np.einsum("ir,...rd->...id", dref[q], Jinv)  # grad phi_i = J^-T ref-grad
        muq = np.einsum("...m,m->...", np.asarray(mu), vals[q])
        outer = np.einsum("cr,...is->...icrs", eye, grad)
        E = 0.5 * (outer + np.swapaxes(outer, -1, -2))  # eps(phi_i e_c)
        Aq = 2.0 * np.einsum("...icrs,...jdrs->...djci", E, E)
        A += (qw[q] * det * muq)[..., None, None] * Aq.reshape(sh + (30, 30))
    return A
