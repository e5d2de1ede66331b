"""Pins of the oracle's element matrices against independent computations.

The oracle integrates barycentric monomials exactly; these tests recompute
element matrices with sympy (symbolic integration of explicit Cartesian basis
functions on the reference tetrahedron) or with a conical-product Gauss
rule, and check closed forms and invariants the definitions fix.
"""
import numpy as np
import pytest
import sympy as sp
from scipy.special import roots_jacobi

from oracle import elements as el
from workloads import quadrature as Q

REF = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=float)
X, Y, Z = sp.symbols("x y z")
LAM = [1 - X - Y - Z, X, Y, Z]
EDGES = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
P2_SYM = [LAM[a] * (2 * LAM[a] - 1) for a in range(4)] + [4 * LAM[a] * LAM[b] for a, b in EDGES]


def _tet_integral(expr):
    return sp.integrate(expr, (X, 0, 1 - Y - Z), (Y, 0, 1 - Z), (Z, 0, 1))


def _random_tet(seed):
    rng = np.random.default_rng(seed)
    P = rng.standard_normal((4, 3))
    return P


def _conical_rule(order=6):
    """Gauss rule on the reference tet by the collapsed map (u,v,w) -> (u, v(1-u), w(1-u)(1-v))."""
    tu, wu = roots_jacobi(order, 2, 0)
    tv, wv = roots_jacobi(order, 1, 0)
    tw, ww = roots_jacobi(order, 0, 0)
    u, v, w = (tu + 1) / 2, (tv + 1) / 2, (tw + 1) / 2
    pts, wts = [], []
    for a in range(order):
        for b in range(order):
            for c in range(order):
                x = u[a]
                y = v[b] * (1 - u[a])
                z = w[c] * (1 - u[a]) * (1 - v[b])
                pts.append((x, y, z))
                wts.append(wu[a] / 8 * wv[b] / 4 * ww[c] / 2)
    return np.array(pts), np.array(wts)


_GRAD = [[sp.lambdify((X, Y, Z), sp.diff(f, s)) for s in (X, Y, Z)] for f in P2_SYM]
_VAL = [sp.lambdify((X, Y, Z), f) for f in P2_SYM]


def _ref_basis(pts):
    vals = np.array([[_VAL[i](*p) for i in range(10)] for p in pts])
    grads = np.array([[[_GRAD[i][d](*p) for d in range(3)] for i in range(10)] for p in pts])
    return vals, grads


def test_p1_reference_element_closed_form():
    K = el.p1_laplace(REF)
    expect = np.array([[3, -1, -1, -1], [-1, 1, 0, 0], [-1, 0, 1, 0], [-1, 0, 0, 1]]) / 6
    assert np.allclose(K, expect, atol=1e-15)


def test_p1_element_scales_linearly_with_h():
    P = _random_tet(1)
    assert np.allclose(el.p1_laplace(0.25 * P), 0.25 * el.p1_laplace(P), rtol=1e-13)
    k = np.array([1.0, 2.0, 3.0, 4.0])
    assert np.allclose(el.p1_divkgrad(P, k), 2.5 * el.p1_laplace(P), rtol=1e-14)


def test_p2_laplace_reference_matches_sympy():
    A = np.zeros((10, 10))
    for i in range(10):
        for j in range(10):
            g = sum(sp.diff(P2_SYM[i], s) * sp.diff(P2_SYM[j], s) for s in (X, Y, Z))
            A[j, i] = float(_tet_integral(sp.expand(g)))
    assert np.allclose(el.p2_laplace(REF), A, atol=1e-15)


def test_p2_basis_integrals_textbook():
    # int phi_vertex = -|T|/20, int phi_edge = |T|/5
    assert np.allclose(el.P2_INT_PHI, [-1 / 20] * 4 + [1 / 5] * 6, atol=1e-16)
    for i in (0, 5):
        assert np.isclose(float(_tet_integral(sp.expand(P2_SYM[i]))) * 6, el.P2_INT_PHI[i])


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_p2_divkgrad_matches_conical_gauss(seed):
    P = _random_tet(seed)
    k = 1 + np.random.default_rng(seed + 10).uniform(-0.5, 0.5, 10)
    pts, wts = _conical_rule(6)
    vals, rg = _ref_basis(pts)
    J = np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]], 1)
    Jinv = np.linalg.inv(J)
    det = abs(np.linalg.det(J))
    grads = np.einsum("qir,rd->qid", rg, Jinv)
    kq = vals @ k
    A = np.einsum("q,q,qid,qjd->ji", wts * det, kq, grads, grads)
    got = el.p2_divkgrad(P, k)
    assert np.allclose(got, A, rtol=1e-12, atol=1e-13 * np.abs(A).max())
    # symmetric local matrix: 55 unique entries of 100
    assert np.allclose(got, got.T, rtol=1e-14, atol=1e-15)
    assert np.allclose(el.p2_divkgrad(P, np.ones(10)), el.p2_laplace(P), rtol=1e-13)


def _rigid_modes(Pnodes):
    """Six rigid motions (constants, rotations) sampled at nodes (10,3): (6, 30) component-major."""
    modes = []
    for c in range(3):
        u = np.zeros((3, 10))
        u[c] = 1
        modes.append(u.ravel())
    for w in np.eye(3):
        u = np.cross(w, Pnodes).T
        modes.append(u.ravel())
    return np.array(modes)


def _p2_nodes(P):
    return np.concatenate([P, [(P[a] + P[b]) / 2 for a, b in EDGES]])


@pytest.mark.parametrize("seed", [0, 3])
def test_epsilon_affine_kernel_is_rigid_motions(seed):
    P = _random_tet(seed)
    mu = np.exp(np.random.default_rng(seed).standard_normal(10) * 0.3)
    A = el.eps_affine(P, mu)
    assert np.allclose(A, A.T, atol=1e-13 * np.abs(A).max())
    R = _rigid_modes(_p2_nodes(P))
    assert np.abs(A @ R.T).max() < 1e-12 * np.abs(A).max()
    ev = np.linalg.eigvalsh(A)
    assert (ev > -1e-12 * ev.max()).all()
    assert np.sum(ev > 1e-10 * ev.max()) == 30 - 6  # kernel is exactly the rigid motions


def test_epsilon_component_trace_is_four_times_scalar_operator():
    # sum_c A[(j,c),(i,c)] = int mu (3 + 1) grad phi_i . grad phi_j
    P = _random_tet(5)
    mu = 1 + np.random.default_rng(7).uniform(0, 1, 10)
    A = el.eps_affine(P, mu).reshape(3, 10, 3, 10)
    tr = sum(A[c, :, c, :] for c in range(3))
    assert np.allclose(tr, 4 * el.p2_divkgrad(P, mu), rtol=1e-13, atol=1e-14)


def test_epsilon_matches_conical_gauss_definition():
    P = _random_tet(11)
    mu = 1 + np.random.default_rng(12).uniform(0, 1, 10)
    pts, wts = _conical_rule(6)
    vals, rg = _ref_basis(pts)
    J = np.stack([P[1] - P[0], P[2] - P[0], P[3] - P[0]], 1)
    grads = np.einsum("qir,rd->qid", rg, np.linalg.inv(J))
    det = abs(np.linalg.det(J))
    A = np.zeros((3, 10, 3, 10))
    for q in range(len(wts)):
        for i in range(10):
            for c in range(3):
                Gu = np.zeros((3, 3))
                Gu[c] = grads[q, i]  # grad of phi_i e_c: row c
                Eu = 0.5 * (Gu + Gu.T)
                for j in range(10):
                    for d in range(3):
                        Gv = np.zeros((3, 3))
                        Gv[d] = grads[q, j]
                        Ev = 0.5 * (Gv + Gv.T)
                        A[d, j, c, i] += wts[q] * det * (vals[q] @ mu) * 2 * np.sum(Eu * Ev)
    assert np.allclose(el.eps_affine(P, mu), A.reshape(30, 30), rtol=1e-12, atol=1e-13)


def test_blended_element_with_identity_map_equals_affine():
    P = _random_tet(4)
    mu = 1 + np.random.default_rng(1).uniform(0, 1, 10)
    qb, qw = Q.rule_degree5()  # exact for the degree-4 affine integrand
    B = el.eps_blended(P, mu, np.ones(3), qb, qw, dmap=lambda xi: np.broadcast_to(np.eye(3), xi.shape[:-1] + (3, 3)))
    assert np.allclose(B, el.eps_affine(P, mu), rtol=1e-12, atol=1e-13 * np.abs(B).max())


def test_shell_jacobian_matches_finite_differences():
    rng = np.random.default_rng(2)
    s = np.array([1.0, -1.0, 1.0])
    for _ in range(5):
        xi = np.abs(rng.uniform(0.1, 1, 3)) * s
        phi = lambda z: z * (z @ s) / np.linalg.norm(z)
        h = 1e-6
        fd = np.stack([(phi(xi + h * e) - phi(xi - h * e)) / (2 * h) for e in np.eye(3)], 1)
        assert np.allclose(el.shell_jacobian(xi, s), fd, atol=1e-9)


def test_blended_element_kills_constants_and_is_symmetric():
    from workloads import meshes
    v, t = meshes.octahedral_shell()
    P = v[t[4]]
    s = np.sign(P.mean(0))
    mu = 1 + np.random.default_rng(3).uniform(0, 1, 10)
    qb, qw = Q.rule_degree5()
    B = el.eps_blended(P, mu, s, qb, qw)
    assert np.allclose(B, B.T, atol=1e-13 * np.abs(B).max())
    for c in range(3):
        u = np.zeros((3, 10))
        u[c] = 1
        assert np.abs(B @ u.ravel()).max() < 1e-12 * np.abs(B).max()


def _shell_map(z):
    """Radial map of the shell written out: z |z|_1 / |z|_2."""
    return z * np.abs(z).sum() / np.linalg.norm(z)


def _blended_by_finite_differences(P, mu, qb, qw, h=1e-5):
    """The curved element rebuilt without the oracle's Jacobian code: J at each
    quadrature point by central differences of the composed map
    x -> Phi(P0 + J_T x), reference basis from sympy, strains written out."""
    JT = (P[1:] - P[0]).T
    G = lambda xh: _shell_map(P[0] + JT @ xh)
    pts = qb[:, 1:]
    vals, grads = _ref_basis(pts)
    A = np.zeros((3, 10, 3, 10))
    for q in range(len(qw)):
        J = np.stack([(G(pts[q] + h * e) - G(pts[q] - h * e)) / (2 * h) for e in np.eye(3)], 1)
        det = abs(np.linalg.det(J))
        gphys = grads[q] @ np.linalg.inv(J)     # row i: J^-T applied to the reference gradient
        muq = vals[q] @ mu
        for c in range(3):
            for i in range(10):
                Gu = np.zeros((3, 3))
                Gu[c] = gphys[i]
                Eu = 0.5 * (Gu + Gu.T)
                for d in range(3):
                    for j in range(10):
                        Gv = np.zeros((3, 3))
                        Gv[d] = gphys[j]
                        Ev = 0.5 * (Gv + Gv.T)
                        A[d, j, c, i] += qw[q] * det * muq * 2 * np.sum(Eu * Ev)
    return A.reshape(30, 30)


@pytest.mark.parametrize("macro,level,tidx,which", [(0, 0, 0, 0), (7, 0, 0, 0), (13, 1, 2, 0), (22, 2, 5, 0),
                                                    (4, 2, 3, 5), (17, 2, 0, 9)])
def test_blended_element_matches_composed_map_finite_differences(macro, level, tidx, which):
    """Section "Tabulation of Factors of the Weak Form" (curvilinear remark): the
    curved element's Jacobian at a quadrature point is that of the composed map
    Phi(F_T(x)) there.  Rebuilt from finite differences of the composed map
    (error ~1e-10), the element matrix agrees with the oracle's to 1e-7.  A
    Jacobian composed in the wrong order, or DPhi taken anywhere but at the
    quadrature point, is off by O(1) on a macro and O(h) on a micro-tet."""
    from oracle import lattice as lat
    from workloads import meshes
    v, t = meshes.octahedral_shell()
    n = 2 ** level
    pts = lat.micro_tets(n, lat.TYPE_NAMES[tidx])[which]
    P = v[t[macro][0]] + (pts / n) @ (v[t[macro][1:]] - v[t[macro][0]])
    s = np.sign(v[t[macro]].mean(0))
    mu = 1 + np.random.default_rng(macro).uniform(0, 1, 10)
    qb, qw = Q.rule_degree5()
    B = el.eps_blended(P, mu, s, qb, qw)
    ref = _blended_by_finite_differences(P, mu, qb, qw)
    assert np.abs(B - ref).max() <= 1e-7 * np.abs(ref).max()


def test_blended_shell_volume_converges():
    """Sum over the micro-tets of the shell and the points of the rule of
    w_q |det J_q| (the Jacobians the blended element uses) approaches the
    volume 4/3 pi (1 - 0.55^3) of the shell the map covers exactly.  The
    integrand |det DPhi| |det J_T| is smooth, so a degree-5 rule converges
    at order about 6 in h; DPhi frozen at one point per element would give
    order 2."""
    import oracle as O
    from workloads import meshes
    v, t = meshes.octahedral_shell()
    qb, qw = Q.rule_degree5()
    exact = 4.0 / 3.0 * np.pi * (1 - 0.55 ** 3)
    errs = []
    for level in range(4):
        pr = O.Problem(v, t, level, O.P2V_EPSILON, O.BC_NONE, map_=O.MAP_SHELL_RADIAL, qbary=qb, qw=qw)
        vol = 0.0
        for m, tn, P, nodes in pr.element_batches():
            s = np.sign(v[t[m]].mean(0))
            J = el.blended_jacobians(P, s, qb)
            vol += float(np.einsum("q,eq->", qw, np.abs(np.linalg.det(J))))
        errs.append(abs(vol - exact))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(3)]
    print("volume errors", errs, "observed orders", rates)
    assert errs[-1] <= 1e-7 * exact
    assert min(rates[1:]) >= 5.0
