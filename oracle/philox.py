"""Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), from its published
definition, in Python integers.

Test infrastructure (see the package docstring).

One round maps the counter (x0, x1, x2, x3) with key (k0, k1) to
(hi(M1*x2) ^ x1 ^ k0, lo(M1*x2), hi(M0*x0) ^ x3 ^ k1, lo(M0*x0)); the key is
advanced by the Weyl constants (W0, W1) between rounds; ten rounds.
"""
from __future__ import annotations

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
MASK = (1 << 64) - 1


def philox4x64_10(ctr, key):
    x0, x1, x2, x3 = (int(c) & MASK for c in ctr)
    k0, k1 = (int(k) & MASK for k in key)
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * x0
        p1 = M1 * x2
        x0, x1, x2, x3 = ((p1 >> 64) ^ x1 ^ k0, p1 & MASK, (p0 >> 64) ^ x3 ^ k1, p0 & MASK)
    return x0, x1, x2, x3


def uniform53(r):
    """Uniform double in [0, 1) from the top 53 bits of a 64-bit word."""
    return (int(r) >> 11) * (1.0 / (1 << 53))


def index_below(r, n):
    """floor(U * n) for U = (r >> 11) / 2^53, in exact integer arithmetic."""
    return ((int(r) >> 11) * int(n)) >> 53
