"""Oracle: SplitMix64 counter-based generator.  TEST INFRASTRUCTURE ONLY.

The paper fixes no randomness source.  Keys, noise and encryption masks are
drawn from SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014) used as a counter generator:
word(seed, dom, i) is output i of the stream whose state starts at
mix(seed + dom*gamma).  Domains: 1 = secret t, 2 = matrix B, 3 = LWE error e,
4 = encryption masks R.
"""
from __future__ import annotations

GAMMA = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1


def mix(z: int) -> int:
    z &= M64
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & M64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & M64
    z ^= z >> 31
    return z


def word(seed: int, dom: int, i: int) -> int:
    return mix(mix(seed + dom * GAMMA) + (i + 1) * GAMMA)


def zq_element(seed: int, dom: int, e: int, k: int) -> int:
    """Uniform element of Z_{2^k}: ceil(k/64) consecutive words of the
    domain, little-endian, the top word masked to the remaining bits."""
    L = (k + 63) // 64
    v = 0
    for w in range(L):
        v |= word(seed, dom, e * L + w) << (64 * w)
    return v & ((1 << k) - 1)


def ternary(seed: int, dom: int, j: int) -> int:
    """e_j = bit(2j) - bit(2j+1) of the domain's bit stream: P(-1)=P(1)=1/4,
    P(0)=1/2."""
    b0 = (word(seed, dom, (2 * j) // 64) >> ((2 * j) % 64)) & 1
    b1 = (word(seed, dom, (2 * j + 1) // 64) >> ((2 * j + 1) % 64)) & 1
    return b0 - b1
