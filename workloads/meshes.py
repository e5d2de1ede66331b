"""Macro (coarse) tetrahedral meshes of the paper's workloads.

Each mesh is (vertices float64 [nv,3], tets int64 [nt,4]).  The vertex order
of a tet fixes its refinement lattice (vertex 0 is the lattice origin).
"""
import itertools
import numpy as np

MAP_AFFINE = 0
MAP_SHELL_RADIAL = 1


def ref_tet():
    """The reference tetrahedron (0,0,0),(1,0,0),(0,1,0),(0,0,1)."""
    v = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], dtype=np.float64)
    return v, np.array([[0, 1, 2, 3]], dtype=np.int64)


def kuhn_cube():
    """Unit cube split into 6 tets along the (0,0,0)-(1,1,1) diagonal.

    Tet for permutation s of the axes: 0, e_s0, e_s0+e_s1, (1,1,1); the
    permutations are taken in lexicographic order.  Cube corner (x,y,z) has
    vertex id x + 2y + 4z.
    """
    v = np.array([[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)],
                 dtype=np.float64)
    vid = lambda p: int(p[0] + 2 * p[1] + 4 * p[2])
    tets = []
    for s in itertools.permutations(range(3)):
        p0 = np.zeros(3, dtype=int)
        p1 = p0.copy(); p1[s[0]] = 1
        p2 = p1.copy(); p2[s[1]] = 1
        p3 = np.ones(3, dtype=int)
        tets.append([vid(p0), vid(p1), vid(p2), vid(p3)])
    return v, np.array(tets, dtype=np.int64)


def octahedral_shell(r_in=0.55, r_out=1.0):
    """Thick spherical shell as 24 macro-tets (8 octant prisms x 3 tets).

    Direction ids: +x=0, -x=1, +y=2, -y=3, +z=4, -z=5.  Inner vertex id d sits
    at r_in*e_d, outer vertex id 6+d at r_out*e_d.  The octant prism with
    inner triangle (a,b,c), a<b<c, and outer triangle (a',b',c') is split into
    (a,b,c,a'), (b,c,a',b'), (c,a',b',c').  Every quad side face between
    directions p<q gets the diagonal inner-q -- outer-p in both prisms that
    share it, so the split is conforming.  The flat mesh is mapped onto the
    shell by the radial map x = xi*|xi|_1/|xi|_2 (MAP_SHELL_RADIAL).
    """
    dirs = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]],
                    dtype=np.float64)
    v = np.concatenate([r_in * dirs, r_out * dirs])
    tets = []
    for a in (0, 1):
        for b in (2, 3):
            for c in (4, 5):
                ao, bo, co = a + 6, b + 6, c + 6
                tets += [[a, b, c, ao], [b, c, ao, bo], [c, ao, bo, co]]
    return v, np.array(tets, dtype=np.int64)


def shell_map(xi):
    """Radial blending map of the shell: xi * |xi|_1 / |xi|_2 (rows of xi)."""
    xi = np.asarray(xi, dtype=np.float64)
    return xi * (np.abs(xi).sum(-1) / np.linalg.norm(xi, axis=-1))[..., None]
