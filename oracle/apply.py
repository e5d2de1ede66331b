"""Oracle: matrix-free operator application y = A x in FP64 (plain numpy).

Test infrastructure only: the product library never imports this package.

Implements equation (4.1) of section "Matrix-Free Finite Elements" literally:
y = sum_T P_T A_T R_T x, looping over macro-tetrahedra and, inside each, over
the micro-tetrahedra of every type (elements.py gives A_T, lattice.py gives
the micro-tets and the DoF layout).  Elements are processed in vectorised
batches; the scatter P_T is a histogram add.  A DoF on a face, edge or vertex
shared by several macro-tetrahedra is stored once per macro ("macro-local"
layout): after the local sums, the copies of each DoF (equal canonical keys)
are added and every copy receives the total, so inputs and outputs are
consistent vectors.

Boundary condition DIRICHLET_ZERO is y = D A D x with D the 0/1 mask of DoFs
not on the domain boundary (a DoF is on the domain boundary when one of its
copies lies on a macro face that belongs to a single macro-tetrahedron).

Also: the same operator assembled as a sparse matrix (for brute-force
checks), its diagonal (assembly of the matrix diagonal is the second
operation the paper's generator provides, section "Code Generation for FEM
on Hybrid Tetrahedral Grids"), the gradient of L = 0.5 |A(k) x - b|^2 with
respect to x and k, and plain conjugate gradients.
"""
import numpy as np
import scipy.sparse as sp

from . import elements as el
from .lattice import (EDGES, TYPE_NAMES, barycentric, lattice_points, lattice_size,
                      micro_tets, packed_index, point_keys)

P1_LAPLACE, P1_DIVKGRAD, P2_LAPLACE, P2_DIVKGRAD, P2V_EPSILON, N1_CURLCURL = range(6)
BC_NONE, BC_DIRICHLET_ZERO = 0, 1
MAP_AFFINE, MAP_SHELL_RADIAL = 0, 1

# N1 (curl-curl + mass) uses the P2 lattice: an edge DoF sits at the edge's
# midpoint slot (vertex slots carry no DoF: their rows and columns are zero),
# and the coefficients alpha, beta sit at the vertex slots of a
# two-component coefficient vector [alpha | beta].  The DoF is the tangential
# integral along the edge oriented from the endpoint with the smaller
# canonical key to the larger.
SPACE = {P1_LAPLACE: 1, P1_DIVKGRAD: 1, P2_LAPLACE: 2, P2_DIVKGRAD: 2, P2V_EPSILON: 2, N1_CURLCURL: 2}
HAS_COEFF = {P1_LAPLACE: False, P1_DIVKGRAD: True, P2_LAPLACE: False, P2_DIVKGRAD: True,
             P2V_EPSILON: True, N1_CURLCURL: True}
COEFF_COMP = {N1_CURLCURL: 2}

CHUNK = 65536


class Problem:
    """One operator on one refined macro mesh (oracle side)."""

    def __init__(self, vertices, tets, level, kind, bc=BC_DIRICHLET_ZERO, map_=MAP_AFFINE,
                 qbary=None, qw=None):
        self.V = np.asarray(vertices, dtype=np.float64)
        self.tets = np.asarray(tets, dtype=np.int64)
        self.level = int(level)
        self.n = 2 ** self.level
        self.kind, self.bc, self.map = kind, bc, map_
        self.space = SPACE[kind]
        self.N = self.n * self.space
        self.L = lattice_size(self.N)
        self.nt = len(self.tets)
        self.n_local = self.nt * self.L
        self.ncomp = 3 if kind == P2V_EPSILON else 1
        self.qbary = None if qbary is None else np.asarray(qbary, dtype=np.float64)
        self.qw = None if qw is None else np.asarray(qw, dtype=np.float64)
        self.pts = lattice_points(self.N)
        self._layout()

    # ------------------------------------------------------------- layout
    def _layout(self):
        bary = barycentric(self.pts, self.N)  # (L,4)
        keys = np.concatenate([point_keys(self.tets[m], self.pts, self.N) for m in range(self.nt)])
        _, first, uid = np.unique(keys, axis=0, return_index=True, return_inverse=True)
        self.keys = keys
        self.uid = uid.reshape(-1)
        self.n_unique = int(self.uid.max()) + 1
        self.owner = np.zeros(self.n_local, dtype=bool)
        self.owner[first] = True
        # faces: face f of macro m is opposite vertex f
        faces = {}
        for m in range(self.nt):
            for f in range(4):
                key = tuple(sorted(np.delete(self.tets[m], f).tolist()))
                faces[key] = faces.get(key, 0) + 1
        bnd_copy = np.zeros(self.n_local, dtype=bool)
        xi = np.empty((self.n_local, 3))
        for m in range(self.nt):
            t = self.tets[m]
            for f in range(4):
                key = tuple(sorted(np.delete(t, f).tolist()))
                if faces[key] == 1:
                    bnd_copy[m * self.L:(m + 1) * self.L] |= bary[:, f] == 0
            xi[m * self.L:(m + 1) * self.L] = (bary @ self.V[t]) / self.N
        bnd_u = np.zeros(self.n_unique, dtype=bool)
        np.logical_or.at(bnd_u, self.uid, bnd_copy)
        self.boundary = bnd_u[self.uid]
        self.xi = xi
        if self.map == MAP_SHELL_RADIAL:
            self.xyz = xi * (np.abs(xi).sum(-1) / np.linalg.norm(xi, axis=-1))[:, None]
        else:
            self.xyz = xi.copy()
        self.interior = ~self.boundary if self.bc == BC_DIRICHLET_ZERO else np.ones(self.n_local, bool)

    # ---------------------------------------------------------- elements
    def element_batches(self):
        """Yield (macro, type, P (E,4,3) flat-mesh vertex positions, nodes (E,nn) local indices)."""
        for m in range(self.nt):
            t = self.tets[m]
            V0 = self.V[t[0]]
            Jm = (self.V[t[1:]] - V0)  # rows: v1-v0, v2-v0, v3-v0
            for tn in TYPE_NAMES:
                pts_all = micro_tets(self.n, tn)
                for s in range(0, len(pts_all), CHUNK):
                    pts = pts_all[s:s + CHUNK]
                    P = V0 + (pts / self.n) @ Jm
                    if self.space == 1:
                        nodes = packed_index(pts, self.N)
                    else:
                        vn = 2 * pts
                        en = np.stack([pts[:, a] + pts[:, b] for a, b in EDGES], 1)
                        nodes = packed_index(np.concatenate([vn, en], 1), self.N)
                    yield m, tn, P, nodes + m * self.L

    def _coeff_e(self, coeff, nodes):
        """Element coefficient values (N1: alpha and beta at the 4 vertex slots)."""
        if not HAS_COEFF[self.kind]:
            return None
        if self.kind == N1_CURLCURL:
            v = nodes[:, :4]
            return coeff[v], coeff[self.n_local + v]
        return coeff[nodes]

    def element_matrices(self, P, c_e, macro, nodes=None):
        k = self.kind
        if self.map == MAP_SHELL_RADIAL and k != P2V_EPSILON:
            raise ValueError("the blended map is defined for the epsilon operator")
        if k == N1_CURLCURL:
            # local orientation a -> b (a < b) turned to the global one: the
            # edge DoF's sign is + when the canonical keys increase from a to b
            A6 = el.n1_curlcurl_mass(P, *c_e)
            u = self.uid[nodes[:, :4]]
            sgn = np.stack([np.where(u[:, a] < u[:, b], 1.0, -1.0) for a, b in EDGES], 1)
            A = np.zeros((len(P), 10, 10))
            A[:, 4:, 4:] = sgn[:, :, None] * A6 * sgn[:, None, :]
            return A
        if k == P1_LAPLACE:
            return el.p1_laplace(P)
        if k == P1_DIVKGRAD:
            return el.p1_divkgrad(P, c_e)
        if k == P2_LAPLACE:
            return el.p2_laplace(P)
        if k == P2_DIVKGRAD:
            # with a rule on an affine mesh: the quadrature (under-integration) variant
            if self.qbary is not None and self.map == MAP_AFFINE:
                return el.p2_divkgrad_quad(P, c_e, self.qbary, self.qw)
            return el.p2_divkgrad(P, c_e)
        if self.map == MAP_AFFINE:
            return el.eps_affine(P, c_e)
        if self.qbary is None:
            raise ValueError("the blended map needs a quadrature rule")
        s = np.sign(self.V[self.tets[macro]].mean(0))
        return el.eps_blended(P, c_e, s, self.qbary, self.qw)

    def _dof_index(self, nodes):
        if self.ncomp == 1:
            return nodes
        return np.concatenate([nodes + c * self.n_local for c in range(3)], 1)

    def _check(self, x, coeff):
        x = np.asarray(x, dtype=np.float64)
        if x.shape != (self.ncomp * self.n_local,):
            raise ValueError("x has shape %s, expected (%d,)" % (x.shape, self.ncomp * self.n_local))
        if HAS_COEFF[self.kind]:
            coeff = np.asarray(coeff, dtype=np.float64)
            if coeff.shape != (COEFF_COMP.get(self.kind, 1) * self.n_local,):
                raise ValueError("coefficient has the wrong shape")
        return x, coeff

    def _mask(self, v):
        if self.ncomp == 1:
            return v * self.interior
        return v * np.tile(self.interior, 3)

    def interface_sum(self, v):
        """Sum the copies of each DoF and give every copy the total."""
        out = np.empty_like(v)
        for c in range(self.ncomp):
            seg = v[c * self.n_local:(c + 1) * self.n_local]
            tot = np.bincount(self.uid, weights=seg, minlength=self.n_unique)
            out[c * self.n_local:(c + 1) * self.n_local] = tot[self.uid]
        return out

    # ------------------------------------------------------------- apply
    def apply(self, x, coeff=None, rows=None):
        """y = A x.  With `rows` (local indices), only y at those rows (and their copies) is exact."""
        return self.finish(self.local_sum(x, coeff, rows=rows))

    def local_sum(self, x, coeff=None, rows=None, share=(0, 1)):
        """The element loop of the apply: sum over micro-tets T of P_T A_T R_T (D x), before the
        interface sum and the output mask.  `share` = (i, n) restricts it to the element batches
        whose index is i modulo n (the n shares add up to the whole loop)."""
        x, coeff = self._check(x, coeff)
        xm = self._mask(x)
        y = np.zeros_like(x)
        need = None
        if rows is not None:
            need = np.isin(self.uid, np.unique(self.uid[np.asarray(rows)]))
        for j, (m, tn, P, nodes) in enumerate(self.element_batches()):
            if j % share[1] != share[0]:
                continue
            if need is not None:
                sel = need[nodes].any(1)
                if not sel.any():
                    continue
                P, nodes = P[sel], nodes[sel]
            A = self.element_matrices(P, self._coeff_e(coeff, nodes), m, nodes)
            idx = self._dof_index(nodes)
            ye = np.einsum("eji,ei->ej", A, xm[idx])
            y += np.bincount(idx.ravel(), weights=ye.ravel(), minlength=y.size)
        return y

    def finish(self, y):
        """Interface sum over the copies of each DoF, then the output mask D."""
        return self._mask(self.interface_sum(y))

    # ---------------------------------------------------------- diagonal
    def diagonal(self, coeff=None):
        """diag(D A D) on every copy: each element's (A_T)_vv added into node v,
        the copies of a DoF summed, boundary rows 0."""
        if HAS_COEFF[self.kind]:
            coeff = np.asarray(coeff, dtype=np.float64)
        d = np.zeros(self.ncomp * self.n_local)
        for m, tn, P, nodes in self.element_batches():
            A = self.element_matrices(P, self._coeff_e(coeff, nodes), m, nodes)
            idx = self._dof_index(nodes)
            de = np.einsum("ejj->ej", A)
            d += np.bincount(idx.ravel(), weights=de.ravel(), minlength=d.size)
        return self._mask(self.interface_sum(d))

    # ------------------------------------------------------------ sparse
    def assemble(self, coeff=None):
        """Sparse matrix of D A D on unique DoFs (component-major for vector operators)."""
        rows, cols, vals = [], [], []
        if HAS_COEFF[self.kind]:
            coeff = np.asarray(coeff, dtype=np.float64)
        for m, tn, P, nodes in self.element_batches():
            A = self.element_matrices(P, self._coeff_e(coeff, nodes), m, nodes)
            u = self.uid[nodes]
            if self.ncomp == 3:
                u = np.concatenate([u + c * self.n_unique for c in range(3)], 1)
            nd = u.shape[1]
            rows.append(np.repeat(u, nd, axis=1).ravel())
            cols.append(np.tile(u, (1, nd)).ravel())
            vals.append(A.reshape(len(u), -1).ravel())
        nu = self.ncomp * self.n_unique
        M = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(nu, nu))
        d = np.zeros(self.n_unique)
        d[self.uid] = self.interior
        D = sp.diags(np.tile(d, self.ncomp))
        return (D @ M @ D).tocsr()

    def to_unique(self, v):
        out = np.zeros(self.ncomp * self.n_unique)
        for c in range(self.ncomp):
            out[c * self.n_unique + self.uid] = v[c * self.n_local:(c + 1) * self.n_local]
        return out

    def to_local(self, u):
        return np.concatenate([u[c * self.n_unique:(c + 1) * self.n_unique][self.uid]
                               for c in range(self.ncomp)])

    # ----------------------------------------------------------- adjoint
    def coeff_gradient(self, coeff, x, gy):
        """g_k = d (gy . A(k) x) / dk for each unique coefficient DoF, on every copy.

        A(k) is linear in k, so g_k[m] = sum over elements T containing node m of
        (D gy)_T . (dA_T/dk_m) (D x)_T (for the epsilon operator k is mu and
        dA_T/dmu_b = A_T(e_b), vector components included).
        """
        if self.kind not in (P1_DIVKGRAD, P2_DIVKGRAD, P2V_EPSILON):
            raise ValueError("coefficient gradient is defined for the div(k grad) and epsilon operators")
        coeff = np.asarray(coeff, dtype=np.float64)
        xm, rm = self._mask(np.asarray(x, float)), self._mask(np.asarray(gy, float))
        g = np.zeros(self.n_local)
        for m, tn, P, nodes in self.element_batches():
            if self.kind == P2V_EPSILON:
                # A_T(mu) is linear in the 10 nodal values of mu: dA_T/dmu_b = A_T(e_b)
                idx = self._dof_index(nodes)
                xe, re = xm[idx], rm[idx]
                ge = np.empty(nodes.shape)
                for b in range(nodes.shape[1]):
                    eb = np.zeros(nodes.shape)
                    eb[:, b] = 1.0
                    Ab = self.element_matrices(P, eb, m)
                    ge[:, b] = np.einsum("ej,eji,ei->e", re, Ab, xe)
                g += np.bincount(nodes.ravel(), weights=ge.ravel(), minlength=g.size)
                continue
            xe, re = xm[nodes], rm[nodes]
            if self.kind == P1_DIVKGRAD:
                K = el.p1_laplace(P)
                s = np.einsum("ej,eji,ei->e", re, K, xe) / 4.0
                ge = np.repeat(s[:, None], 4, axis=1)
            else:
                vol, gr = el.geometry(P)
                G = np.einsum("ead,ebd->eab", gr, gr)
                T = np.einsum("eab,mijab->emji", G, el.P2_CM)
                ge = vol[:, None] * np.einsum("ej,emji,ei->em", re, T, xe)
            g += np.bincount(nodes.ravel(), weights=ge.ravel(), minlength=g.size)
        # the coefficient is a scalar field: sum its copies
        tot = np.bincount(self.uid, weights=g, minlength=self.n_unique)
        return tot[self.uid]

    def loss_gradients(self, coeff, x, b):
        """L = 0.5 |A(k) x - b|^2 over unique DoFs: returns (L, dL/dx, dL/dk) on every copy."""
        r = self.apply(x, coeff) - np.asarray(b, float)
        r_u = self.to_unique(r)
        L = 0.5 * float(r_u @ r_u)
        gx = self.apply(r, coeff)
        gk = self.coeff_gradient(coeff, x, r)
        return L, gx, gk

    # ---------------------------------------------------------------- CG
    def cg(self, b, coeff=None, tol=1e-14, maxiter=20000):
        """Plain conjugate gradients on the consistent vectors (dots over unique DoFs)."""
        b = np.asarray(b, dtype=np.float64)
        own = np.tile(self.owner, self.ncomp)
        dot = lambda u, v: float(np.dot(u[own], v[own]))
        x = np.zeros_like(b)
        r = self._mask(b.copy())
        p = r.copy()
        rr = dot(r, r)
        nb = np.sqrt(dot(b, b))
        it = 0
        while np.sqrt(rr) > tol * nb and it < maxiter:
            Ap = self.apply(p, coeff)
            a = rr / dot(p, Ap)
            x += a * p
            r -= a * Ap
            rr_new = dot(r, r)
            p = r + (rr_new / rr) * p
            rr = rr_new
            it += 1
        return x, it
