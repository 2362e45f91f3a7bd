"""Philox4x64-10 counter-based random numbers (Salmon, Moraes, Dror & Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), written from the
published definition with Python integers.

Test infrastructure only (see the package header).

The hybrid chain draws one uniform number per random decision: the initial
S^z index of each environment site of sample 0 and the outcome of each
environment-site collapse (Markov Chain Sampling Algorithm, step 4).  The
counter words are (chain, sample, MPS position, purpose) with purpose 0 for
the initial state and 1 for a collapse; the key is (seed, 0).  The uniform
number is the top 53 bits of the first output word times 2^-53.

Pin: bit-identical to numpy.random.Philox (an independent implementation
of the same published generator).
"""
from __future__ import annotations

MASK64 = (1 << 64) - 1
M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15   # golden ratio
W1 = 0xBB67AE8584CAA73B   # sqrt(3) - 1

PURPOSE_INIT = 0
PURPOSE_COLLAPSE = 1


def _mulhilo(a: int, b: int):
    p = a * b
    return (p >> 64) & MASK64, p & MASK64


def philox4x64(counter, key, rounds: int = 10):
    """Encrypt a 4-word counter with a 2-word key; returns 4 words."""
    c0, c1, c2, c3 = [int(x) & MASK64 for x in counter]
    k0, k1 = [int(x) & MASK64 for x in key]
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + W0) & MASK64
            k1 = (k1 + W1) & MASK64
        hi0, lo0 = _mulhilo(M0, c0)
        hi1, lo1 = _mulhilo(M1, c2)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def uniform(seed: int, chain: int, sample: int, pos: int,
            purpose: int) -> float:
    """u in [0,1) for one decision."""
    x = philox4x64((chain, sample, pos, purpose), (seed, 0))[0]
    return (x >> 11) * (1.0 / 9007199254740992.0)
