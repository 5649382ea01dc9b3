"""Counter-based SplitMix64 stream for seeded synthetic inputs.

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): the k-th output (k = 0, 1, ...) of a stream seeded
with ``s`` is ``mix(s + (k + 1) * GAMMA)`` with GAMMA = 0x9E3779B97F4A7C15 and
``mix`` the variant-13 finaliser of MurmurHash3 used by that paper.  Because the
output is a pure function of (seed, k), any element of a block can be produced
independently, on the host here and, in the eigensolver library, on the device.

Uniform doubles use the top 53 bits: u = (z >> 11) * 2**-53 in [0, 1).
This module holds none of the eigensolver's arithmetic.
"""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def mix64(z):
    """MurmurHash3-style 64-bit finaliser (SplitMix64 output function)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed, k):
    """k-th output (array-valued k allowed) of the stream seeded with ``seed``."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = np.uint64(seed) + (k + np.uint64(1)) * GAMMA
    return mix64(state)


def uniform01(seed, k):
    """Doubles in [0, 1) from the top 53 bits of the k-th output."""
    z = splitmix64(seed, k)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def uniform_pm1(seed, k):
    """Doubles in [-1, 1)."""
    return 2.0 * uniform01(seed, k) - 1.0


def random_block(seed, n, q):
    """N x q row-major block of U(-1, 1) values.

    Element (row i, column j) is output k = j * n + i of the stream, so column j
    does not depend on q.
    """
    i = np.arange(n, dtype=np.uint64)[:, None]
    j = np.arange(q, dtype=np.uint64)[None, :]
    return uniform_pm1(seed, j * np.uint64(n) + i)


def derive_seed(seed, tag):
    """Seed of an independent sub-stream (e.g. per request of a stream)."""
    return int(mix64(np.uint64(seed) ^ mix64(np.uint64(tag) + GAMMA)))
