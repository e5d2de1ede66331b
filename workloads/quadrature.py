"""Fully symmetric quadrature rules on the tetrahedron, solved from moments.

A rule is (bary [nq,4], w [nq]) on the reference tetrahedron
(0,0,0),(1,0,0),(0,1,0),(0,0,1) with weights summing to its volume 1/6; the
reference point of row q is bary[q,1:].  Point sets are unions of orbits of
the permutation group S4 acting on barycentric coordinates:

  S4      (1/4, 1/4, 1/4, 1/4)                       1 point
  S31(a)  permutations of (a, a, a, 1-3a)             4 points
  S22(a)  permutations of (a, a, 1/2-a, 1/2-a)        6 points

Orbit parameters and weights solve the moment equations
sum_q w_q x^a y^b z^c = a! b! c! / (a+b+c+3)!  for all a+b+c <= degree
by nonlinear least squares from a fixed start, and the solution is accepted
only when every moment matches to 1e-14.  The rules are problem data: the
blended shell operator is defined with a rule, and the same arrays are handed
to every implementation.
"""
import itertools
import math

import numpy as np
from scipy.optimize import least_squares


def _orbit(kind, a):
    if kind == "S4":
        base = [(0.25, 0.25, 0.25, 0.25)]
    elif kind == "S31":
        base = [(a, a, a, 1 - 3 * a)]
    elif kind == "S22":
        base = [(a, a, 0.5 - a, 0.5 - a)]
    else:
        raise ValueError(kind)
    # one unrounded representative per distinct permutation
    out = []
    seen = set()
    for p in itertools.permutations(base[0]):
        key = tuple(round(c, 12) for c in p)
        if key not in seen:
            seen.add(key)
            out.append(p)
    return np.array(out, dtype=np.float64)


def exact_moment(a, b, c):
    """Integral of x^a y^b z^c over the reference tetrahedron."""
    return math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)


def monomials(degree):
    return [(a, b, c) for a in range(degree + 1) for b in range(degree + 1 - a)
            for c in range(degree + 1 - a - b)]


def moment_residuals(bary, w, degree):
    x = bary[:, 1:]
    res = []
    for a, b, c in monomials(degree):
        res.append(np.sum(w * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c) - exact_moment(a, b, c))
    return np.array(res)


def _assemble(kinds, params):
    npar = sum(1 for k in kinds if k != "S4")
    ab = params[:npar]
    ws = params[npar:]
    pts, wts = [], []
    it = iter(ab)
    for kind, wk in zip(kinds, ws):
        a = next(it) if kind != "S4" else None
        o = _orbit(kind, a)
        pts.append(o)
        wts.append(np.full(len(o), wk))
    return np.concatenate(pts), np.concatenate(wts)


def _solve(kinds, start, degree):
    def f(p):
        b, w = _assemble(kinds, p)
        return moment_residuals(b, w, degree)

    sol = least_squares(f, np.array(start, dtype=np.float64), xtol=1e-15, ftol=1e-15, gtol=1e-15,
                        max_nfev=2000)
    bary, w = _assemble(kinds, sol.x)
    r = moment_residuals(bary, w, degree)
    if np.max(np.abs(r)) > 1e-14:
        raise RuntimeError("quadrature rule did not converge: residual %g" % np.max(np.abs(r)))
    return bary, w


def rule_degree2():
    """4-point rule exact to degree 2: S31 with a = (5 - sqrt 5)/20, weights 1/24."""
    a = (5.0 - math.sqrt(5.0)) / 20.0
    bary = _orbit("S31", a)
    return bary, np.full(4, 1.0 / 24.0)


_CACHE = {}


def rule_degree5():
    """14-point rule exact to degree 5: two S31 orbits and one S22 orbit, all weights positive."""
    if "d5" not in _CACHE:
        # start: S31 near a vertex-ward and a face-ward position, S22 near the edges
        _CACHE["d5"] = _solve(["S31", "S31", "S22"], [0.1, 0.3, 0.05, 0.012, 0.018, 0.007], 5)
    b, w = _CACHE["d5"]
    return b.copy(), w.copy()


def rule_degree4_negative():
    """11-point rule exact to degree 4 (S4 + S31 + S22); its centroid weight is negative."""
    if "d4" not in _CACHE:
        _CACHE["d4"] = _solve(["S31", "S22", "S4"], [0.07, 0.1, 0.008, 0.025, -0.013], 4)
    b, w = _CACHE["d4"]
    return b.copy(), w.copy()
