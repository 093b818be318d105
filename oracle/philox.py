"""Philox4x64-10 counter-based generator, written from its published definition
(Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).

Oracle code (test infrastructure only).

The method draws one uniform per sampled site (paper, SM Alg. 1 and Alg. 2: a
spin is set to +1 when ``random() < q``) and one uniform per Metropolis-Hastings
decision (Alg. 2, ``random() < P_acc``).  Both implementations derive these
uniforms from the same counter-based generator so that the same proposal is
drawn on both sides.

Stream layout (our reading; the paper does not fix an RNG):

* key     = (seed, chain)
* counter = (draw, z, sweep, purpose); purpose 0 = site draw (draw = y*Lx + x),
  purpose 1 = MH decision (draw = 0); with several candidates per
  environment, candidate k draws its sites with purpose 2k and its MH uniform
  with purpose 2k + 1 (candidate 0 is the single-candidate update)
* the uniform is taken from output word 0:  U = ((w >> 11) + 0.5) * 2^-53,
  so 0 < U < 1.
"""
from __future__ import annotations

MASK64 = (1 << 64) - 1
_M0 = 0xD2E7470EE14C6C93
_M1 = 0xCA5A826395121157
_W0 = 0x9E3779B97F4A7C15
_W1 = 0xBB67AE8584CAA73B

PURPOSE_SITE = 0
PURPOSE_MH = 1


def philox4x64_10(counter, key):
    """One Philox4x64 block with 10 rounds: returns four 64-bit words."""
    c0, c1, c2, c3 = (int(v) & MASK64 for v in counter)
    k0, k1 = (int(v) & MASK64 for v in key)
    for _ in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + _W0) & MASK64
        k1 = (k1 + _W1) & MASK64
    return c0, c1, c2, c3


def word_to_uniform(w: int) -> float:
    """Top 53 bits of a 64-bit word mapped to the open interval (0, 1)."""
    return ((w >> 11) + 0.5) * (2.0 ** -53)


def uniform(seed: int, chain: int, sweep: int, z: int, purpose: int, draw: int) -> float:
    w = philox4x64_10((draw, z, sweep, purpose), (seed, chain))[0]
    return word_to_uniform(w)
