"""Seeded random test vectors shared by the tests, smoke() and bench.py.

Holds no arithmetic of the method: only numpy's PCG64 draws of vectors that
are passed, byte for byte, both to the HIP library and to the CPU oracle.
"""
import numpy as np


def normal_vector(n, seed):
    """n FP64 draws from N(0, 1) (numpy default_rng(seed))."""
    return np.random.default_rng(seed).standard_normal(int(n))


def uniform_vector(n, seed, lo=-1.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, int(n))


def sparse_vector(n, k, seed):
    """n-vector with k nonzero N(0,1) entries at distinct random positions."""
    rng = np.random.default_rng(seed)
    v = np.zeros(int(n))
    idx = rng.choice(int(n), size=min(int(k), int(n)), replace=False)
    v[idx] = rng.standard_normal(idx.size)
    return v
