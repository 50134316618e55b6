"""Seeded synthetic inputs shared by the library's callers and its tests.

This module draws random numbers and nothing else: it holds none of the
transform or scheme arithmetic, imports nothing else from the package, and
is the only code the tests share with the product.  Seeds follow one
convention: 0 = data, 1 = secret/keys, 2 = errors, 3 = arrivals.
"""
import numpy as np


def rng(seed, stream=0):
    return np.random.Generator(np.random.PCG64([int(seed), int(stream)]))


def uniform_residues(seed, moduli, shape, stream=0):
    """uint32 [len(moduli)][*shape], limb l uniform in [0, moduli[l])."""
    g = rng(seed, stream)
    shape = tuple(int(s) for s in np.atleast_1d(shape))
    out = np.empty((len(moduli),) + shape, dtype=np.uint32)
    for i, q in enumerate(moduli):
        out[i] = g.integers(0, int(q), size=shape, dtype=np.uint64).astype(np.uint32)
    return out


def ternary_secret(seed, n, hamming_weight, stream=0):
    """int8 [n]: `hamming_weight` distinct uniform positions, each +-1."""
    g = rng(seed, stream)
    s = np.zeros(n, dtype=np.int8)
    pos = g.choice(n, size=hamming_weight, replace=False)
    s[pos] = np.where(g.integers(0, 2, size=hamming_weight) == 0, -1, 1)
    return s


def gaussian_error(seed, shape, sigma=3.2, bound=19, stream=0):
    """int32 rounded N(0, sigma^2), rejection-truncated to |e| <= bound."""
    g = rng(seed, stream)
    shape = tuple(int(s) for s in np.atleast_1d(shape))
    e = np.rint(g.normal(0.0, sigma, size=shape)).astype(np.int64)
    bad = np.abs(e) > bound
    while bad.any():
        e[bad] = np.rint(g.normal(0.0, sigma, size=int(bad.sum()))).astype(np.int64)
        bad = np.abs(e) > bound
    return e.astype(np.int32)


def small_messages(seed, shape, bound=16, stream=0):
    """int32 uniform in [-bound, bound]."""
    g = rng(seed, stream)
    shape = tuple(int(s) for s in np.atleast_1d(shape))
    return g.integers(-bound, bound + 1, size=shape, dtype=np.int64).astype(np.int32)


def poisson_arrivals(seed, rate_per_s, count, stream=0):
    """Arrival times (s) of a Poisson process: cumulative exponential gaps."""
    g = rng(seed, stream)
    return np.cumsum(g.exponential(1.0 / float(rate_per_s), size=int(count)))


def request_mix(seed, count, log_ns=(13, 14, 15, 16), max_level=24, rotations=(1, 2, 4, 8, 16, 32, 64, 128),
                hmult_share=0.5, stream=0):
    """Serving requests: op (0 = HMULT, 1 = rotate), log2 N, level in
    1..max_level, rotation amount.  Returns a dict of int arrays."""
    g = rng(seed, stream)
    count = int(count)
    return {
        "op": (g.random(count) >= hmult_share).astype(np.int32),
        "log_n": g.choice(np.asarray(log_ns), size=count).astype(np.int32),
        "level": g.integers(1, max_level + 1, size=count).astype(np.int32),
        "rot": g.choice(np.asarray(rotations), size=count).astype(np.int32),
    }
