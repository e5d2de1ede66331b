"""Pins of the oracle's global operators: invariants, closed forms, brute force.

Equation (4.1): A = sum_T P_T A_T R_T.  These tests check the assembled
behaviour against facts of the continuous problem (constants and linear
fields in the kernel, the 7-point stencil of the Kuhn/Freudenthal cube, exact
quadratic consistency of P2), against a sparse-matrix assembly, and the
gradients against finite differences (exact for a quadratic loss).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla
import sympy as sp

import oracle as O
from oracle import elements as el
import workloads as W

KINDS = [O.P1_LAPLACE, O.P1_DIVKGRAD, O.P2_LAPLACE, O.P2_DIVKGRAD, O.P2V_EPSILON]


def _coeff(pr):
    return 1 + 0.5 * np.sin(pr.xyz @ np.array([1.0, 2.0, 3.0]))


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("mesh", ["ref", "cube", "shell"])
def test_constants_in_kernel(kind, mesh):
    v, t = {"ref": W.meshes.ref_tet, "cube": W.meshes.kuhn_cube,
            "shell": W.meshes.octahedral_shell}[mesh]()
    kw = {}
    if mesh == "shell" and kind == O.P2V_EPSILON:
        kw = dict(map_=O.MAP_SHELL_RADIAL, qbary=W.quadrature.rule_degree5()[0],
                  qw=W.quadrature.rule_degree5()[1])
    pr = O.Problem(v, t, 1, kind, O.BC_NONE, **kw)
    k = _coeff(pr)
    for c in range(pr.ncomp):
        u = np.zeros(pr.ncomp * pr.n_local)
        u[c * pr.n_local:(c + 1) * pr.n_local] = 1.0
        y = pr.apply(u, k)
        assert np.abs(y).max() < 1e-13


@pytest.mark.parametrize("kind", [O.P1_LAPLACE, O.P2_LAPLACE])
def test_linear_fields_in_kernel_on_interior_rows(kind):
    v, t = W.meshes.kuhn_cube()
    pr = O.Problem(v, t, 2, kind, O.BC_NONE)
    u = pr.xyz @ np.array([0.3, -1.2, 2.0]) + 0.7
    y = pr.apply(u, _coeff(pr))
    interior = ~O.Problem(v, t, 2, kind, O.BC_DIRICHLET_ZERO).boundary
    assert np.abs(y[interior]).max() < 1e-12


@pytest.mark.parametrize("level", [2, 3])
def test_p1_on_kuhn_cube_is_the_7_point_stencil(level):
    v, t = W.meshes.kuhn_cube()
    pr = O.Problem(v, t, level, O.P1_LAPLACE, O.BC_NONE)
    n = 2 ** level
    h = 1.0 / n
    rng = np.random.default_rng(level)
    grid = rng.standard_normal((n + 1, n + 1, n + 1))
    ijk = np.rint(pr.xyz * n).astype(int)
    u = grid[ijk[:, 0], ijk[:, 1], ijk[:, 2]]
    y = pr.apply(u)
    inside = ((ijk > 0) & (ijk < n)).all(1)
    i, j, k = ijk[inside].T
    fd = h * (6 * grid[i, j, k] - grid[i + 1, j, k] - grid[i - 1, j, k] - grid[i, j + 1, k]
              - grid[i, j - 1, k] - grid[i, j, k + 1] - grid[i, j, k - 1])
    assert np.allclose(y[inside], fd, rtol=1e-12, atol=1e-13)


def _p2_row_integrals(pr, f_nodal_linear):
    """int f phi_i for a linear f given at micro-vertices, per local P2 DoF, via sympy rationals."""
    X, Y, Z = sp.symbols("x y z")
    lam = [1 - X - Y - Z, X, Y, Z]
    edges = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    basis = [lam[a] * (2 * lam[a] - 1) for a in range(4)] + [4 * lam[a] * lam[b] for a, b in edges]
    # R[a,i] = (1/|T|) int lambda_a phi_i (reference volume 1/6)
    R = np.array([[6 * float(sp.integrate(sp.expand(lam[a] * basis[i]), (X, 0, 1 - Y - Z),
                                          (Y, 0, 1 - Z), (Z, 0, 1))) for i in range(10)]
                  for a in range(4)])
    out = np.zeros(pr.n_local)
    for m, tn, P, nodes in pr.element_batches():
        vol, _ = el.geometry(P)
        fv = f_nodal_linear(P)  # (E,4)
        out += np.bincount(nodes.ravel(), weights=(vol[:, None] * (fv @ R)).ravel(), minlength=pr.n_local)
    return pr.interface_sum(out)


def test_p2_laplace_exact_on_quadratics():
    v, t = W.meshes.kuhn_cube()
    pr = O.Problem(v, t, 2, O.P2_LAPLACE, O.BC_NONE)
    x, y, z = pr.xyz.T
    u = 0.5 * x * x - 1.5 * y * y + 2.0 * z * z + 0.3 * x * y - 0.7 * y * z + x - 2
    lap = 0.5 * 2 - 1.5 * 2 + 2.0 * 2  # Laplacian of u
    rhs = _p2_row_integrals(pr, lambda P: np.full(P.shape[:2], -lap))
    out = pr.apply(u)
    interior = ~O.Problem(v, t, 2, O.P2_LAPLACE).boundary
    assert np.allclose(out[interior], rhs[interior], rtol=1e-12, atol=1e-13)


def test_p2_divkgrad_exact_for_linear_k_and_quadratic_u():
    v, t = W.meshes.kuhn_cube()
    pr = O.Problem(v, t, 2, O.P2_DIVKGRAD, O.BC_NONE)
    kc = np.array([0.4, -0.3, 0.2])
    k = 2.0 + pr.xyz @ kc
    x, y, z = pr.xyz.T
    u = x * x + 2 * y * y - z * z + x * z
    # -div(k grad u) = -(grad k . grad u) - k lap u ; grad u = (2x+z, 4y, -2z+x), lap u = 4
    def f(P):
        px, py, pz = P[..., 0], P[..., 1], P[..., 2]
        gu = np.stack([2 * px + pz, 4 * py, -2 * pz + px], -1)
        kk = 2.0 + P @ kc
        return -(gu @ kc) - kk * 4.0
    rhs = _p2_row_integrals(pr, f)
    out = pr.apply(u, k)
    interior = ~O.Problem(v, t, 2, O.P2_DIVKGRAD).boundary
    assert np.allclose(out[interior], rhs[interior], rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("level", [0, 1, 2])
def test_matrix_free_equals_sparse_assembly(kind, level):
    v, t = W.meshes.kuhn_cube()
    pr = O.Problem(v, t, level, kind, O.BC_DIRICHLET_ZERO)
    rng = np.random.default_rng(level)
    k = _coeff(pr)
    xu = rng.standard_normal(pr.ncomp * pr.n_unique)
    A = pr.assemble(k)
    y = pr.apply(pr.to_local(xu), k)
    ref = pr.to_local(A @ xu)
    assert np.allclose(y, ref, rtol=1e-13, atol=1e-14 * np.abs(ref).max())


@pytest.mark.parametrize("kind", KINDS)
def test_dirichlet_rows_and_columns_symmetry_definiteness(kind):
    v, t = W.meshes.kuhn_cube()
    pr = O.Problem(v, t, 1, kind, O.BC_DIRICHLET_ZERO)
    k = _coeff(pr)
    A = pr.assemble(k).toarray()
    bnd = np.zeros(pr.n_unique, bool)
    bnd[pr.uid] = pr.boundary
    bnd = np.tile(bnd, pr.ncomp)
    assert np.abs(A[bnd]).max() == 0 and np.abs(A[:, bnd]).max() == 0
    assert np.allclose(A, A.T, atol=1e-14 * np.abs(A).max())
    ev = np.linalg.eigvalsh(A[np.ix_(~bnd, ~bnd)])
    assert ev.min() > 0


def test_layout_counts():
    v, t = W.meshes.kuhn_cube()
    pr = O.Problem(v, t, 3, O.P2_LAPLACE)
    assert pr.n_unique == 17 ** 3 and pr.n_local == 6 * 969
    assert pr.boundary[pr.owner].sum() == 17 ** 3 - 15 ** 3
    v, t = W.meshes.octahedral_shell()
    pr = O.Problem(v, t, 1, O.P2_LAPLACE)
    # vertices + edges + faces + cells of the flat mesh refined: count via Euler-type formula
    nu = pr.n_unique
    N = pr.N
    expect = 12 + 42 * (N - 1) + 56 * (N - 1) * (N - 2) // 2 + 24 * (N - 1) * (N - 2) * (N - 3) // 6
    assert nu == expect


def test_outputs_are_consistent_across_copies():
    v, t = W.meshes.octahedral_shell()
    pr = O.Problem(v, t, 1, O.P2_DIVKGRAD, O.BC_NONE)
    x = W.uniform_from_keys(1, pr.keys)
    y = pr.apply(x, _coeff(pr))
    tot = np.zeros(pr.n_unique)
    tot[pr.uid] = y
    assert np.array_equal(tot[pr.uid], y)


@pytest.mark.parametrize("kind", [O.P1_DIVKGRAD, O.P2_DIVKGRAD])
def test_coefficient_gradient_brute_force(kind):
    v, t = W.meshes.kuhn_cube()
    pr = O.Problem(v, t, 1, kind, O.BC_DIRICHLET_ZERO)
    rng = np.random.default_rng(0)
    x = pr.to_local(rng.standard_normal(pr.n_unique))
    gy = pr.to_local(rng.standard_normal(pr.n_unique))
    k = _coeff(pr)
    g = pr.coeff_gradient(k, x, gy)
    gu = pr.to_unique(g)
    for m in range(pr.n_unique):
        e = np.zeros(pr.n_unique)
        e[m] = 1
        d = pr.to_unique(gy) @ pr.to_unique(pr.apply(x, pr.to_local(e)))
        assert abs(gu[m] - d) < 1e-13 * max(1, abs(d))


@pytest.mark.parametrize("kind", [O.P1_DIVKGRAD, O.P2_DIVKGRAD])
def test_loss_gradients_central_differences(kind):
    v, t = W.meshes.ref_tet()
    pr = O.Problem(v, t, 2, kind, O.BC_DIRICHLET_ZERO)
    k = W.fields.perturbed_k(pr.keys, 5)
    x = W.uniform_from_keys(6, pr.keys)
    b = W.uniform_from_keys(7, pr.keys)
    L, gx, gk = pr.loss_gradients(k, x, b)
    rng = np.random.default_rng(8)
    h = 1e-6
    for _ in range(8):
        for which in ("x", "k"):
            d = pr.to_local(rng.uniform(-1, 1, pr.n_unique))
            d /= np.linalg.norm(pr.to_unique(d))
            if which == "x":
                Lp = pr.loss_gradients(k, x + h * d, b)[0]
                Lm = pr.loss_gradients(k, x - h * d, b)[0]
                g = gx
            else:
                Lp = pr.loss_gradients(k + h * d, x, b)[0]
                Lm = pr.loss_gradients(k - h * d, x, b)[0]
                g = gk
            fd = (Lp - Lm) / (2 * h)
            an = pr.to_unique(g) @ pr.to_unique(d)
            assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3 * L)


def _eps_problem(mesh):
    if mesh == "cube":
        v, t = W.meshes.kuhn_cube()
        return O.Problem(v, t, 1, O.P2V_EPSILON, O.BC_DIRICHLET_ZERO)
    v, t = W.meshes.octahedral_shell()
    qb, qw = W.quadrature.rule_degree5()
    return O.Problem(v, t, 0, O.P2V_EPSILON, O.BC_DIRICHLET_ZERO, map_=O.MAP_SHELL_RADIAL, qbary=qb, qw=qw)


@pytest.mark.parametrize("mesh", ["cube", "shell"])
def test_epsilon_mu_gradient_brute_force(mesh):
    """A(mu) is linear in mu: gy . (A(mu + e_m) - A(mu)) x equals the gradient at m exactly (affine and blended)."""
    pr = _eps_problem(mesh)
    rng = np.random.default_rng(1)
    x = pr.to_local(rng.standard_normal(3 * pr.n_unique))
    gy = pr.to_local(rng.standard_normal(3 * pr.n_unique))
    mu = 1 + 0.5 * np.sin(pr.xyz @ np.array([1.0, 2.0, 3.0]))
    g = pr.coeff_gradient(mu, x, gy)
    gu = np.zeros(pr.n_unique)
    gu[pr.uid] = g
    assert np.array_equal(g, gu[pr.uid])  # consistent over copies
    base = pr.to_unique(gy) @ pr.to_unique(pr.apply(x, mu))
    for m in rng.choice(pr.n_unique, 12, replace=False):
        e = np.zeros(pr.n_unique)
        e[m] = 1
        d = pr.to_unique(gy) @ pr.to_unique(pr.apply(x, mu + e[pr.uid])) - base
        assert abs(gu[m] - d) < 1e-11 * max(1, abs(base)), m


def test_epsilon_loss_gradient_central_differences():
    pr = _eps_problem("shell")
    mu = W.fields.shell_mu(pr.keys, pr.xyz, 3)
    x = pr.to_local(np.random.default_rng(2).uniform(-1, 1, 3 * pr.n_unique))
    b = pr.to_local(np.random.default_rng(3).uniform(-1, 1, 3 * pr.n_unique))
    L, gx, gk = pr.loss_gradients(mu, x, b)
    rng = np.random.default_rng(4)
    h = 1e-6
    for _ in range(6):
        du = rng.uniform(-1, 1, pr.n_unique)
        du /= np.linalg.norm(du)
        Lp = pr.loss_gradients(mu + h * du[pr.uid], x, b)[0]
        Lm = pr.loss_gradients(mu - h * du[pr.uid], x, b)[0]
        gu = np.zeros(pr.n_unique)
        gu[pr.uid] = gk
        an = gu @ du
        assert abs((Lp - Lm) / (2 * h) - an) <= 1e-6 * max(abs(an), 1e-3 * L)


def test_cg_matches_sparse_direct_solve():
    v, t = W.meshes.ref_tet()
    pr = O.Problem(v, t, 3, O.P2_DIVKGRAD, O.BC_DIRICHLET_ZERO)
    k = _coeff(pr)
    b = pr._mask(W.uniform_from_keys(11, pr.keys))
    x, it = pr.cg(b, k, tol=1e-13)
    A = pr.assemble(k)
    inner = pr.to_unique(pr.interior.astype(float)) > 0
    xd = np.zeros(pr.n_unique)
    xd[inner] = spla.spsolve(A[inner][:, inner].tocsc(), pr.to_unique(b)[inner])
    assert np.allclose(pr.to_unique(x), xd, rtol=1e-10, atol=1e-10 * np.abs(xd).max())


def test_local_sum_shares_add_up_to_the_apply():
    """The element loop split into shares (as the CPU baseline splits it over worker
    processes) adds up to the apply, up to summation order."""
    v, t = W.meshes.kuhn_cube()
    pr = O.Problem(v, t, 2, O.P2_DIVKGRAD, O.BC_DIRICHLET_ZERO)
    x = W.uniform_from_keys(2, pr.keys)
    k = W.fields.cube_k(pr.xyz)
    ref = pr.apply(x, k)
    y = pr.finish(sum(pr.local_sum(x, k, share=(i, 5)) for i in range(5)))
    assert np.abs(y - ref).max() <= 1e-14 * np.abs(ref).max()
