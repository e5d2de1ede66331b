"""Coefficient fields and right-hand sides of the benchmark workloads.

Formulas are evaluated at physical node positions supplied by the caller;
random values are hashed from canonical DoF keys supplied by the caller.
"""
import numpy as np

from .rng import uniform_from_keys, normal_from_keys


def uniform(keys, seed, lo=-1.0, hi=1.0, stream=0):
    """Seeded U[lo,hi) value per DoF key."""
    return uniform_from_keys(seed, keys, lo, hi, stream=stream)


def cube_k(xyz):
    """k(x,y,z) = 1 + 0.5 sin(2 pi x) cos(2 pi y) z (P2 div(k grad) on the unit cube)."""
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    return 1.0 + 0.5 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) * z


def shell_mu(keys, xyz, seed, sigma=0.3):
    """mu = exp(-3 r) * exp(sigma g), g ~ N(0,1) per node, r = |x| (shell viscosity)."""
    r = np.linalg.norm(xyz, axis=-1)
    return np.exp(-3.0 * r) * np.exp(sigma * normal_from_keys(seed, keys))


def perturbed_k(keys, seed, amp=0.9):
    """k = 1 + amp * U[-1,1) per node (nodal coefficient of the adjoint workload)."""
    return 1.0 + amp * uniform_from_keys(seed, keys)


def batch_levels(count=32, seed=9, lo=3, hi=8):
    """Uneven refinement levels of the batched workload, drawn from {lo..hi-1}."""
    return np.random.default_rng(seed).integers(lo, hi, count)


def batch_k_params(count=32, seed=10):
    """Per-instance smooth-coefficient parameters (a_i in U[-2,2]^3, phi_i in U[0,2pi))."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-2.0, 2.0, (count, 3))
    phi = rng.uniform(0.0, 2 * np.pi, count)
    return a, phi


def batch_k(xyz, a, phi):
    """k_i(x) = 1 + 0.5 sin(2 pi a_i.x + phi_i) for one instance."""
    return 1.0 + 0.5 * np.sin(2 * np.pi * (xyz @ a) + phi)


def n1_coeff(xyz):
    """alpha and beta of the N1 curl-curl + mass operator at node positions, concatenated
    (smooth and positive; the operator reads them at the vertex points)."""
    alpha = 1 + 0.5 * np.sin(2 * np.pi * xyz[:, 0]) * np.cos(np.pi * xyz[:, 1]) + 0.2 * xyz[:, 2]
    beta = 0.6 + 0.3 * np.cos(np.pi * (xyz[:, 0] + 2 * xyz[:, 2]))
    return np.concatenate([alpha, beta])
