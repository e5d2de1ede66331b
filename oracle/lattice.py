"""Oracle: refinement lattice of a macro-tetrahedron, DoF layout and keys.

Test infrastructure only: the product library never imports this package.

Section "Hybrid Tetrahedral Grids" of the paper: each macro-tetrahedron is
refined uniformly (Bey's rule) `level` times; every micro-tetrahedron is a
translate of one of six reference micro-tetrahedra, and DoFs are addressed
implicitly.  The exact vertex sets of the six types and the storage order are
deferred by the paper to other work; the readings used here are

* index space of macro (v0,v1,v2,v3) at level l, n = 2^l: lattice point
  (i,j,k), i,j,k >= 0, i+j+k <= n, at v0 + (i(v1-v0) + j(v2-v0) + k(v3-v0))/n,
  with integer barycentric coordinates (n-i-j-k, i, j, k);
* the six types are the translates by a cube base b of the vertex sets in
  TYPES, present iff b >= 0 and sum(b) <= n - LIMIT[type]; the loop-bound
  function of the sawtooth strategy (section "Sawtooth Loop Strategy") read
  with exclusive bounds gives the same per-type counts;
* packed storage per macro: points ordered with i fastest, then j, then k;
  P1 DoFs live on the lattice of size N = n, P2 DoFs on the lattice of size
  N = 2n (micro-vertex p -> 2p, micro-edge (p,q) -> p+q);
* canonical key of a point: the pairs (global vertex id, barycentric integer)
  with nonzero integer, sorted by vertex id, padded with (-1, 0).

`bey_refine` refines by Bey's rule directly, independently of the type
table, so tests can compare the two.
"""
import numpy as np

TYPE_NAMES = ("WU", "O1", "O2", "O3", "O4", "WD")
TYPES = {
    "WU": ((0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)),
    "O1": ((1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1)),
    "O2": ((1, 0, 0), (0, 1, 0), (1, 1, 0), (1, 0, 1)),
    "O3": ((0, 1, 0), (0, 0, 1), (1, 0, 1), (0, 1, 1)),
    "O4": ((0, 1, 0), (1, 1, 0), (1, 0, 1), (0, 1, 1)),
    "WD": ((1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1)),
}
LIMIT = {"WU": 1, "O1": 2, "O2": 2, "O3": 2, "O4": 2, "WD": 3}

# local edge order of a tetrahedron's P2 edge DoFs
EDGES = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def bey_children(t):
    """Bey's eight children of tet t = (x0,x1,x2,x3) (integer points, even coordinates)."""
    x0, x1, x2, x3 = (np.asarray(p) for p in t)
    m = lambda a, b: tuple(((a + b) // 2).tolist())
    x0, x1, x2, x3 = (tuple(p.tolist()) for p in (x0, x1, x2, x3))
    a = lambda p: np.asarray(p)
    x01, x02, x03 = m(a(x0), a(x1)), m(a(x0), a(x2)), m(a(x0), a(x3))
    x12, x13, x23 = m(a(x1), a(x2)), m(a(x1), a(x3)), m(a(x2), a(x3))
    return [
        (x0, x01, x02, x03), (x01, x1, x12, x13), (x02, x12, x2, x23), (x03, x13, x23, x3),
        (x01, x02, x03, x13), (x01, x02, x12, x13), (x02, x03, x13, x23), (x02, x12, x13, x23),
    ]


def bey_refine(level):
    """Micro-tets of the index-space macro after `level` recursive Bey refinements.

    Returns a list of 4-tuples of integer lattice points on the level-`level`
    lattice (n = 2^level).
    """
    n = 2 ** level
    tets = [((0, 0, 0), (n, 0, 0), (0, n, 0), (0, 0, n))]
    for _ in range(level):
        tets = [c for t in tets for c in bey_children(t)]
    return tets


def micro_tets(n, type_name):
    """Micro-tets of one type from the type table: (E,4,3) integer vertex points.

    The valid cube bases of a type are exactly the lattice points of the packed
    lattice of size n - LIMIT[type].
    """
    m = n - LIMIT[type_name]
    if m < 0:
        return np.zeros((0, 4, 3), dtype=np.int64)
    b = lattice_points(m)
    off = np.array(TYPES[type_name], dtype=np.int64)
    return b[:, None, :] + off[None, :, :]


def lattice_size(N):
    return (N + 1) * (N + 2) * (N + 3) // 6


def lattice_points(N):
    """All points (i,j,k), i+j+k <= N, in packed storage order (i fastest, then j, then k)."""
    out = []
    for k in range(N + 1):
        M = N - k
        rows = M + 1 - np.arange(M + 1)
        j = np.repeat(np.arange(M + 1), rows)
        start = np.repeat(np.cumsum(rows) - rows, rows)
        i = np.arange(j.size) - start
        out.append(np.stack([i, j, np.full(j.size, k)], -1))
    return np.concatenate(out).astype(np.int64)


def packed_index(p, N):
    """Storage index of points p (...,3) in the packed lattice of size N (counting formula)."""
    p = np.asarray(p, dtype=np.int64)
    i, j, k = p[..., 0], p[..., 1], p[..., 2]
    c3 = lambda m: (m + 1) * (m + 2) * (m + 3) // 6
    M = N - k
    return (c3(N) - c3(N - k)) + (j * (M + 1) - j * (j - 1) // 2) + i


def barycentric(p, N):
    p = np.asarray(p, dtype=np.int64)
    return np.stack([N - p[..., 0] - p[..., 1] - p[..., 2], p[..., 0], p[..., 1], p[..., 2]], -1)


def point_keys(gids, p, N):
    """Canonical keys (L,8) of lattice points p (L,3) of the macro with global vertex ids gids."""
    a = barycentric(p, N)
    g = np.broadcast_to(np.asarray(gids, dtype=np.int64), a.shape)
    g = np.where(a > 0, g, np.iinfo(np.int64).max)
    order = np.argsort(g, axis=-1, kind="stable")
    gs = np.take_along_axis(g, order, -1)
    as_ = np.take_along_axis(a, order, -1)
    gs = np.where(gs == np.iinfo(np.int64).max, -1, gs)
    as_ = np.where(gs == -1, 0, as_)
    out = np.empty(gs.shape[:-1] + (8,), dtype=np.int64)
    out[..., 0::2] = gs
    out[..., 1::2] = as_
    return out
