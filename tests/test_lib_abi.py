"""CPU checks of the C ABI: every declared symbol is exported, and the host-side
layout code (pure C++, no GPU needed) agrees with the oracle's independent
layout; argument errors are reported without touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
import paper_2404_08371_amd as T
from paper_2404_08371_amd import _lib
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "tetmf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(tmf_\w+)\s*\(", src, flags=re.M)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(_lib.path())
    names = declared_functions()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    bound = {s[0] for s in _lib.SIGNATURES}
    assert set(names) == bound, set(names) ^ bound


@pytest.mark.parametrize("mesh", ["ref", "cube", "shell"])
@pytest.mark.parametrize("level", [0, 1, 3])
@pytest.mark.parametrize("space", [1, 2])
def test_layout_matches_oracle(mesh, level, space):
    mk, mp = {"ref": (W.meshes.ref_tet, 0), "cube": (W.meshes.kuhn_cube, 0),
              "shell": (W.meshes.octahedral_shell, 1)}[mesh]
    v, t = mk()
    m = T.Mesh(v, t, level, mp)
    info = m.dof_info(space)
    kw = {}
    if mp == 1:
        kw = dict(map_=O.MAP_SHELL_RADIAL, qbary=W.quadrature.rule_degree5()[0], qw=W.quadrature.rule_degree5()[1])
    kind = O.P1_LAPLACE if space == 1 else O.P2V_EPSILON if mp == 1 else O.P2_LAPLACE
    pr = O.Problem(v, t, level, kind, O.BC_DIRICHLET_ZERO, **kw)
    assert m.layout(space) == (pr.n_local, pr.n_unique)
    assert np.array_equal(info["keys"], pr.keys)
    assert np.array_equal(info["owner"], pr.owner)
    assert np.array_equal(info["boundary"], pr.boundary)
    assert np.allclose(info["xyz"], pr.xyz, rtol=0, atol=1e-14)


def _status(fn, *args):
    return fn(*args)


def test_mesh_argument_errors():
    L = T.lib()
    v, t = W.meshes.ref_tet()
    h = ctypes.c_void_p()
    vp = v.ctypes.data_as(ctypes.POINTER(ctypes.c_double))

    def create(tets, level=1, map_=0, nv=4):
        tt = np.ascontiguousarray(tets, np.int64)
        return L.tmf_mesh_create(vp, nv, tt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(tt), level,
                                 map_, ctypes.byref(h))

    assert create(t) == 0
    L.tmf_mesh_destroy(h)
    assert create([[0, 1, 2, 4]]) == -1  # id out of range
    assert create([[0, 1, 1, 2]]) == -1  # repeated id
    assert create(t, level=10) == -1
    assert create(t, level=-1) == -1
    assert create(t, map_=7) == -1
    assert create(t, nv=3) == -1
    vf = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [1, 1, 0]], float)  # flat tet
    assert L.tmf_mesh_create(vf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 4,
                             t.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 1, 1, 0, ctypes.byref(h)) == -1
    assert b"zero volume" in L.tmf_last_error()
    # a face shared by three tets
    v3 = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [0, 0, -1], [1, 1, 1]], float)
    t3 = np.array([[0, 1, 2, 3], [0, 1, 2, 4], [0, 1, 2, 5]], np.int64)
    assert L.tmf_mesh_create(v3.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 6,
                             t3.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 3, 1, 0, ctypes.byref(h)) == -1
    # shell map: a tet crossing an octant boundary
    vx = np.array([[1, 0, 0], [-1, 0.5, 0], [0, 1, 0], [0, 0, 1]], float)
    assert L.tmf_mesh_create(vx.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 4,
                             t.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 1, 1, 1, ctypes.byref(h)) == -1
    with pytest.raises(T.TetmfError):
        T.Mesh(v, [[0, 1, 2, 2]], 1)


def test_operator_argument_errors_before_any_device_call():
    L = T.lib()
    v, t = W.meshes.ref_tet()
    m = T.Mesh(v, t, 9)
    h = ctypes.c_void_p()
    assert L.tmf_op_create(m.handle, 9, 0, 1, None, None, 0, ctypes.byref(h)) == -1  # bad kind
    assert L.tmf_op_create(m.handle, 0, 5, 1, None, None, 0, ctypes.byref(h)) == -1  # bad precision
    assert L.tmf_op_create(m.handle, 0, 0, 4, None, None, 0, ctypes.byref(h)) == -1  # bad bc
    assert L.tmf_op_create(m.handle, 3, 0, 1, None, None, 0, ctypes.byref(h)) == -1  # P2 above level 8
    qb, qw = W.quadrature.rule_degree5()
    m1 = T.Mesh(v, t, 1)
    qbp = qb.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    qwp = qw.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L.tmf_op_create(m1.handle, 2, 0, 1, qbp, qwp, 14, ctypes.byref(h)) == -1  # rule on affine mesh
    vs, ts = W.meshes.octahedral_shell()
    ms = T.Mesh(vs, ts, 1, T.MAP_SHELL_RADIAL)
    assert L.tmf_op_create(ms.handle, 2, 0, 1, None, None, 0, ctypes.byref(h)) == -4  # scalar kind, curved
    assert L.tmf_op_create(ms.handle, 4, 0, 1, None, None, 0, ctypes.byref(h)) == -1  # curved needs a rule
    bad = qw.copy()
    bad[0] += 0.01
    assert L.tmf_op_create(ms.handle, 4, 0, 1, qbp, bad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 14,
                           ctypes.byref(h)) == -1  # weights must sum to 1/6
    assert L.tmf_apply(None, None, None, None, None) == -1
    assert T.lib().tmf_status_string(-5) == b"not converged"
