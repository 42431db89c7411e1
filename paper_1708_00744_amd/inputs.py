"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This module holds none of the method's arithmetic: it only draws random
numbers with numpy's generators (Philox bit generator, keyed by seed and
walker id) and shapes them into positions, matrices, rows, uniforms and
arrival times.  Both the product path and the oracle may receive these
arrays as inputs.
"""
import numpy as np


def _gen(seed, stream=0):
    key = np.array([np.uint64(seed), np.uint64(stream)], dtype=np.uint64)
    return np.random.Generator(np.random.Philox(key=key))


def positions(seed, walker, n, L):
    """Electron positions uniform in the periodic box [0, L)^3, shape (n, 3)."""
    return _gen(seed, 1_000_000 + walker).uniform(0.0, L, size=(n, 3))


def dense_matrix(seed, n, kind="uniform"):
    """A generic dense n x n FP64 matrix (entries uniform in [-1, 1])."""
    g = _gen(seed, 2)
    if kind == "uniform":
        return g.uniform(-1.0, 1.0, size=(n, n))
    if kind == "normal":
        return g.standard_normal((n, n))
    raise ValueError(kind)


def integer_matrix(seed, n, lo=-3, hi=3):
    """Integer-valued n x n matrix (as float64) for exact rational checks."""
    return _gen(seed, 3).integers(lo, hi + 1, size=(n, n)).astype(np.float64)


def rows(seed, m, n, kind="uniform", lo=-3, hi=3):
    """m proposal rows of length n."""
    g = _gen(seed, 4)
    if kind == "uniform":
        return g.uniform(-1.0, 1.0, size=(m, n))
    if kind == "integer":
        return g.integers(lo, hi + 1, size=(m, n)).astype(np.float64)
    raise ValueError(kind)


def uniforms(seed, m):
    """m Metropolis uniforms in [0, 1)."""
    return _gen(seed, 5).random(m)


def normals(seed, shape):
    return _gen(seed, 6).standard_normal(shape)


def electron_order(seed, n, m):
    """m electron indices in [0, n) (host-driven tests that visit electrons out of order)."""
    return _gen(seed, 7).integers(0, n, size=m)


def poisson_arrivals(seed, count, rate_per_s):
    """Arrival times (s) of a Poisson process with the given rate."""
    gaps = _gen(seed, 8).exponential(1.0 / rate_per_s, size=count)
    return np.cumsum(gaps)


def serving_mix(seed, count, sizes=(128, 256, 512, 1024, 2048), acc_lo=0.5, acc_hi=0.99):
    """Per-request matrix size (uniform over `sizes`), target acceptance
    (uniform in [acc_lo, acc_hi]) and request seed."""
    g = _gen(seed, 9)
    n = g.choice(np.asarray(sizes), size=count)
    acc = g.uniform(acc_lo, acc_hi, size=count)
    seeds = g.integers(1, 2**62, size=count, dtype=np.int64).astype(np.uint64)
    return n, acc, seeds
