"""Counter-based random numbers keyed by canonical DoF keys.

A DoF shared by several macro-tetrahedra appears once per macro in the
macro-local layout.  Drawing its value from a hash of its canonical key (and
not from its position in an array) makes every copy receive the same value
and lets two independent programs that enumerate the DoFs differently build
the same input vector.

The generator is SplitMix64 (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), applied as a hash chain over
the key's integers.  Nothing here knows about finite elements.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x):
    """One SplitMix64 output step applied elementwise to a uint64 array."""
    with np.errstate(over="ignore"):
        z = (np.asarray(x, dtype=np.uint64) + _GOLDEN).astype(np.uint64)
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def hash_keys(seed, keys, stream=0):
    """uint64 hash of each row of an integer key array (rows are keys)."""
    keys = np.asarray(keys, dtype=np.int64)
    if keys.ndim == 1:
        keys = keys[:, None]
    h = splitmix64(np.full(keys.shape[0], np.uint64(seed) * np.uint64(1000003)
                           + np.uint64(stream), dtype=np.uint64))
    for c in range(keys.shape[1]):
        h = splitmix64(h ^ keys[:, c].astype(np.uint64))
    return h


def uniform_from_keys(seed, keys, lo=-1.0, hi=1.0, stream=0):
    """Values in [lo, hi) from the top 53 bits of the key hash."""
    h = hash_keys(seed, keys, stream)
    u = (h >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return lo + (hi - lo) * u


def normal_from_keys(seed, keys, stream=0):
    """Standard normal values (Box-Muller on two independent hash streams)."""
    u1 = uniform_from_keys(seed, keys, 0.0, 1.0, stream=2 * stream + 1)
    u2 = uniform_from_keys(seed, keys, 0.0, 1.0, stream=2 * stream + 2)
    u1 = np.maximum(u1, 1e-300)
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
