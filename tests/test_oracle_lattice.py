"""Pins of the oracle's refinement lattice against Bey's rule and counting facts.

Section "Hybrid Tetrahedral Grids": uniform refinement produces six
translation-invariant micro-tet types; section "Sawtooth Loop Strategy" gives
the per-type loop bounds B(white-up, n) = n, B(4 middle types, n) = n - 1,
B(white-down, n) = n - 2.
"""
import itertools
from math import comb

import numpy as np
import pytest

from oracle import lattice as L


@pytest.mark.parametrize("level", range(0, 5))
def test_type_table_equals_recursive_bey(level):
    n = 2 ** level
    bey = sorted(tuple(sorted(t)) for t in L.bey_refine(level))
    tab = sorted(tuple(sorted(map(tuple, t.tolist()))) for nm in L.TYPE_NAMES
                 for t in L.micro_tets(n, nm))
    assert bey == tab
    assert len(tab) == 8 ** level


@pytest.mark.parametrize("level", range(0, 6))
def test_type_counts_match_loop_bounds(level):
    n = 2 ** level
    # exclusive upper bounds B(o, m): sum over z < B(o,n), y < B(o,n-z), x < B(o,n-z-y)
    B = {"WU": lambda m: m, "WD": lambda m: m - 2}
    for nm in L.TYPE_NAMES:
        b = B.get(nm, lambda m: m - 1)
        cnt = sum(1 for z in range(max(b(n), 0)) for y in range(max(b(n - z), 0))
                  for x in range(max(b(n - z - y), 0)))
        assert len(L.micro_tets(n, nm)) == cnt
    assert len(L.micro_tets(n, "WU")) == comb(n + 2, 3)
    assert len(L.micro_tets(n, "O1")) == comb(n + 1, 3)
    assert len(L.micro_tets(n, "WD")) == comb(n, 3)


@pytest.mark.parametrize("level", range(0, 5))
def test_micro_tets_tile_the_macro(level):
    n = 2 ** level
    tets = np.concatenate([L.micro_tets(n, nm) for nm in L.TYPE_NAMES])
    J = np.stack([tets[:, 1] - tets[:, 0], tets[:, 2] - tets[:, 0], tets[:, 3] - tets[:, 0]], -1)
    det = np.rint(np.linalg.det(J)).astype(int)
    assert (np.abs(det) == 1).all()  # every type has unit determinant in index units
    assert np.abs(det).sum() == n ** 3  # |macro| = n^3 / 6 = sum of n^3 micro volumes 1/6
    # every micro-face is shared by exactly 2 micro-tets unless it lies on the macro boundary
    faces = {}
    for t in tets:
        for f in range(4):
            key = tuple(sorted(map(tuple, np.delete(t, f, 0).tolist())))
            faces[key] = faces.get(key, 0) + 1
    for key, c in faces.items():
        p = np.array(key)
        on_bnd = any((p[:, d] == 0).all() for d in range(3)) or (p.sum(1) == n).all()
        assert c == (1 if on_bnd else 2)


def test_translation_invariance_of_types():
    # every micro-tet of a type is the type's reference vertex set translated
    for nm in L.TYPE_NAMES:
        t = L.micro_tets(8, nm)
        rel = t - t[:, :1]
        assert (rel == rel[0]).all()


def test_interior_vertex_has_14_neighbours_and_24_elements():
    n = 8
    tets = np.concatenate([L.micro_tets(n, nm) for nm in L.TYPE_NAMES])
    p = np.array([2, 2, 2])
    inc = [t for t in tets if (t == p).all(1).any()]
    assert len(inc) == 24
    nb = {tuple(q - p) for t in inc for q in t if not (q == p).all()}
    expect = {(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, -1, 0), (1, 0, -1), (0, 1, -1), (1, -1, 1)}
    expect |= {tuple(-np.array(e)) for e in expect}
    assert nb == expect


@pytest.mark.parametrize("N", [0, 1, 2, 5, 16])
def test_packed_index_is_a_bijection(N):
    pts = L.lattice_points(N)
    assert len(pts) == L.lattice_size(N) == comb(N + 3, 3)
    assert (L.packed_index(pts, N) == np.arange(len(pts))).all()
    # i is fastest: consecutive storage along a row
    assert (np.diff(pts[:, 2]) >= 0).all()


def test_canonical_keys_match_on_shared_faces():
    # two tets sharing the face (1,2,3) with different local vertex orders
    N = 4
    pts = L.lattice_points(N)
    ka = L.point_keys([0, 1, 2, 3], pts, N)
    kb = L.point_keys([3, 1, 2, 4], pts, N)
    face_a = {tuple(k) for k in ka if 0 not in k[0::2]}
    face_b = {tuple(k) for k in kb if 4 not in k[0::2]}
    assert face_a == face_b and len(face_a) == comb(N + 2, 2)
