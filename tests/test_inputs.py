"""Pins of the shared input generators (meshes, quadrature rules, key hashes)."""
import itertools

import numpy as np
import pytest

import workloads as W
from workloads import quadrature as Q


@pytest.mark.parametrize("rule,degree", [(Q.rule_degree2, 2), (Q.rule_degree5, 5),
                                         (Q.rule_degree4_negative, 4)])
def test_rules_integrate_monomials_exactly(rule, degree):
    bary, w = rule()
    assert np.allclose(bary.sum(1), 1.0, atol=1e-15)
    assert np.max(np.abs(Q.moment_residuals(bary, w, degree))) < 1e-15
    # and not one degree more (the rules are not accidentally higher order)
    assert np.max(np.abs(Q.moment_residuals(bary, w, degree + 1))) > 1e-8


def test_rules_are_fully_symmetric():
    for rule in (Q.rule_degree2, Q.rule_degree5, Q.rule_degree4_negative):
        bary, w = rule()
        pts = {tuple(np.round(b, 12)): round(x, 14) for b, x in zip(bary, w)}
        for b, x in zip(bary, w):
            for p in itertools.permutations(b):
                assert pts[tuple(np.round(p, 12))] == round(x, 14)


def test_degree5_rule_weights_positive():
    _, w = Q.rule_degree5()
    assert len(w) == 14 and (w > 0).all()


def test_key_hash_reproducible_and_uniform():
    keys = np.arange(80000, dtype=np.int64).reshape(-1, 8)
    a = W.uniform_from_keys(3, keys)
    assert np.array_equal(a, W.uniform_from_keys(3, keys))
    assert not np.array_equal(a, W.uniform_from_keys(4, keys))
    assert a.min() >= -1 and a.max() < 1 and abs(a.mean()) < 0.03
    g = W.normal_from_keys(5, keys)
    assert abs(g.mean()) < 0.05 and abs(g.std() - 1) < 0.05


def test_splitmix64_reference_values():
    # first outputs of SplitMix64 seeded with 0 (state advanced by the golden gamma)
    out = []
    s = np.uint64(0)
    for _ in range(3):
        out.append(int(W.splitmix64(np.array([s]))[0]))
        s = np.uint64((int(s) + 0x9E3779B97F4A7C15) % 2 ** 64)
    assert out[0] == 0xE220A8397B1DCDAF
    assert out[1] == 0x6E789E6AA1B965F4
    assert out[2] == 0x06C45D188009454F


def _faces(tets):
    faces = {}
    for t in tets:
        for f in range(4):
            key = tuple(sorted(np.delete(t, f)))
            faces[key] = faces.get(key, 0) + 1
    return faces


def _vol(v, t):
    return np.linalg.det(np.stack([v[t[1]] - v[t[0]], v[t[2]] - v[t[0]], v[t[3]] - v[t[0]]], 1)) / 6


def test_kuhn_cube_mesh():
    v, t = W.meshes.kuhn_cube()
    assert len(t) == 6
    vols = [abs(_vol(v, x)) for x in t]
    assert np.allclose(vols, 1 / 6) and np.isclose(sum(vols), 1.0)
    f = _faces(t)
    assert max(f.values()) == 2 and sum(1 for c in f.values() if c == 1) == 12


def test_octahedral_shell_mesh():
    v, t = W.meshes.octahedral_shell()
    assert v.shape == (12, 3) and t.shape == (24, 4)
    f = _faces(t)
    assert max(f.values()) == 2
    assert len(f) == 56 and sum(1 for c in f.values() if c == 2) == 40
    edges = {tuple(sorted(e)) for x in t for e in itertools.combinations(x, 2)}
    assert len(edges) == 42
    assert 12 - 42 + 56 - 24 == 2  # Euler characteristic of a (hollow) ball's triangulation
    assert all(abs(_vol(v, x)) > 1e-6 for x in t)
    # boundary faces lie on the inner or the outer octahedron surface
    for key, c in f.items():
        if c == 1:
            r = {round(np.linalg.norm(v[i]), 6) for i in key}
            assert len(r) == 1
    # flat volume = octahedron(1) - octahedron(0.55)
    assert np.isclose(sum(abs(_vol(v, x)) for x in t), 4 / 3 * (1 - 0.55 ** 3))


def test_shell_map_radii():
    rng = np.random.default_rng(0)
    xi = rng.standard_normal((100, 3))
    xi /= np.abs(xi).sum(1)[:, None]
    for r in (0.55, 1.0):
        x = W.meshes.shell_map(r * xi)
        assert np.allclose(np.linalg.norm(x, axis=1), r)
