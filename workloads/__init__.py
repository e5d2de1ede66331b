"""Seeded synthetic inputs shared by the test suite and the benchmark.

Meshes, coefficient formulas, key-hashed random vectors and quadrature rules
(problem data).  This package holds no finite-element arithmetic: node
positions and canonical DoF keys are computed by whichever side consumes the
inputs, and passed in here.
"""
from .rng import uniform_from_keys, normal_from_keys, hash_keys, splitmix64  # noqa: F401
from . import meshes, fields, quadrature  # noqa: F401
