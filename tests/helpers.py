"""Shared helpers of the test suite: build matching library / oracle problems.

Inputs on both sides come from the key-hashed generators in `workloads`, fed
with each side's own canonical keys and node positions, so the library's
layout code and the oracle's layout code are exercised independently.
"""
import numpy as np

import oracle as O
import workloads as W

MESHES = {"ref": (W.meshes.ref_tet, 0), "cube": (W.meshes.kuhn_cube, 0),
          "shell": (W.meshes.octahedral_shell, 1), "flatshell": (W.meshes.octahedral_shell, 0)}


def coefficient(kind, keys, xyz, seed):
    """Nodal coefficient of each workload family (None for constant-coefficient kinds)."""
    if kind in (O.P1_LAPLACE, O.P2_LAPLACE):
        return None
    if kind == O.P2V_EPSILON:
        return W.fields.shell_mu(keys, xyz, seed)
    if kind == O.P1_DIVKGRAD:
        return W.fields.perturbed_k(keys, seed)
    return W.fields.cube_k(xyz)


def inputs(kind, keys, xyz, seed):
    ncomp = 3 if kind == O.P2V_EPSILON else 1
    x = np.concatenate([W.uniform_from_keys(seed, keys, stream=c) for c in range(ncomp)])
    return x, coefficient(kind, keys, xyz, seed + 100)


def oracle_problem(mesh, level, kind, bc):
    mk, mp = MESHES[mesh]
    v, t = mk()
    kw = {}
    if mp == 1:
        qb, qw = W.quadrature.rule_degree5()
        kw = dict(map_=O.MAP_SHELL_RADIAL, qbary=qb, qw=qw)
    return O.Problem(v, t, level, kind, bc, **kw)


def rel_err(y, ref):
    y, ref = np.asarray(y, float), np.asarray(ref, float)
    d = y - ref
    n2 = np.linalg.norm(ref)
    ni = np.abs(ref).max()
    return (np.linalg.norm(d) / n2 if n2 > 0 else np.linalg.norm(d),
            np.abs(d).max() / ni if ni > 0 else np.abs(d).max())
