"""Pins of the oracle's operator diagonal (the generator's diagonal-assembly
operation, section "Code Generation for FEM on Hybrid Tetrahedral Grids").

diag(D A D)_i = e_i . A e_i: checked by brute force through the (separately
pinned) matrix-free apply, against the sparse assembly on meshes with shared
faces, and through the coefficient: k = c everywhere gives c times the
Laplacian's diagonal.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

MESHES = {"ref": W.meshes.ref_tet, "cube": W.meshes.kuhn_cube, "shell": W.meshes.octahedral_shell}


def _coeff(pr):
    return 1 + 0.5 * np.sin(pr.xyz @ np.array([1.0, 2.0, 3.0]))


@pytest.mark.parametrize("kind", [O.P1_LAPLACE, O.P1_DIVKGRAD, O.P2_LAPLACE, O.P2_DIVKGRAD])
@pytest.mark.parametrize("bc", [O.BC_NONE, O.BC_DIRICHLET_ZERO])
def test_diagonal_brute_force(kind, bc):
    v, t = MESHES["cube"]()
    pr = O.Problem(v, t, 1, kind, bc)
    k = _coeff(pr) if (kind in (O.P1_DIVKGRAD, O.P2_DIVKGRAD, O.P2V_EPSILON)) else None
    d = pr.to_unique(pr.diagonal(k))
    brute = np.zeros(pr.n_unique)
    for u in range(pr.n_unique):
        e = np.zeros(pr.n_unique)
        e[u] = 1.0
        brute[u] = pr.to_unique(pr.apply(pr.to_local(e), k))[u]
    assert np.abs(d - brute).max() <= 1e-14 * np.abs(brute).max()


@pytest.mark.parametrize("kind", [O.P2_LAPLACE, O.P2_DIVKGRAD, O.P2V_EPSILON])
@pytest.mark.parametrize("mesh,level", [("cube", 2), ("shell", 1), ("ref", 3)])
def test_diagonal_equals_sparse_assembly(kind, mesh, level):
    v, t = MESHES[mesh]()
    pr = O.Problem(v, t, level, kind, O.BC_DIRICHLET_ZERO)
    k = _coeff(pr) if (kind in (O.P1_DIVKGRAD, O.P2_DIVKGRAD, O.P2V_EPSILON)) else None
    d = pr.diagonal(k)
    ref = pr.to_local(pr.assemble(k).diagonal())
    assert np.abs(d - ref).max() <= 1e-13 * np.abs(ref).max()
    # consistent: every copy of a shared DoF holds the same value
    assert np.array_equal(d, pr.to_local(pr.to_unique(d)))


@pytest.mark.parametrize("space_kinds", [(O.P1_LAPLACE, O.P1_DIVKGRAD), (O.P2_LAPLACE, O.P2_DIVKGRAD)])
def test_constant_coefficient_scales_the_laplacian_diagonal(space_kinds):
    lap, divk = space_kinds
    v, t = MESHES["cube"]()
    pl = O.Problem(v, t, 2, lap, O.BC_DIRICHLET_ZERO)
    pk = O.Problem(v, t, 2, divk, O.BC_DIRICHLET_ZERO)
    c = 2.75
    dl = pl.diagonal()
    dk = pk.diagonal(np.full(pk.n_local, c))
    assert np.abs(dk - c * dl).max() <= 1e-13 * np.abs(dk).max()


@pytest.mark.parametrize("kind", [O.P2_LAPLACE, O.P2_DIVKGRAD])
def test_diagonal_positive_inside_zero_on_dirichlet_rows(kind):
    v, t = MESHES["cube"]()
    pr = O.Problem(v, t, 2, kind, O.BC_DIRICHLET_ZERO)
    k = _coeff(pr) if (kind in (O.P1_DIVKGRAD, O.P2_DIVKGRAD, O.P2V_EPSILON)) else None
    d = pr.diagonal(k)
    assert np.all(d[pr.boundary] == 0.0)
    assert np.all(d[~pr.boundary] > 0.0)
