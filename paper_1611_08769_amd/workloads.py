"""Seeded synthetic inputs for the encrypted FFT.

This module only draws signals: it holds none of the transform's or the
scheme's arithmetic, and both the library's callers and the tests' oracle
consume what it returns (real-valued float64 signals; each side quantises
them with its own code).

The paper's experiments use random complex signals with values in [0, 1]
(section "Experimental Results", 8 to 128 points) and ten 16x16 images that
are not published.  The generators below produce signals of the same shapes;
images are uniform 8-bit pixels scaled to [0, 1).

Uniforms come from SplitMix64 (Steele, Lea and Flood 2014) in counter mode,
domain 5: u_i = (word(seed, 5, i) >> 11) * 2^-53.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

_GAMMA = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def _mix(z: int) -> int:
    z &= _M64
    z ^= z >> 30
    z = (z * 0xBF58476D1CE4E5B9) & _M64
    z ^= z >> 27
    z = (z * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


class Uniforms:
    """Stream of float64 uniforms in [0, 1) from domain 5 of a seed."""

    def __init__(self, seed: int):
        self.base = _mix((seed + 5 * _GAMMA) & _M64)
        self.i = 0

    def next(self, n: int) -> np.ndarray:
        out = np.empty(n, dtype=np.float64)
        for j in range(n):
            w = _mix((self.base + (self.i + 1) * _GAMMA) & _M64)
            self.i += 1
            out[j] = (w >> 11) * (2.0 ** -53)
        return out


@dataclass
class Signal:
    """One transform request: dims 1 (length points) or 2 (length x length
    image), F-bit words with f fractional bits."""
    dims: int
    length: int
    F: int
    f: int
    re: np.ndarray            # float64, shape (length,) or (length, length)
    im: np.ndarray | None     # None for real input

    @property
    def is_complex(self) -> bool:
        return self.im is not None

    @property
    def points(self) -> int:
        return self.length if self.dims == 1 else self.length * self.length


def uniform_pm1(seed: int, n: int, F: int, f: int, complex_: bool, length=None, stream=None):
    """Uniform in [-1, 1) (real, or independent real/imaginary parts)."""
    u = stream or Uniforms(seed)
    re = 2.0 * u.next(n) - 1.0
    im = (2.0 * u.next(n) - 1.0) if complex_ else None
    return Signal(1, length or n, F, f, re, im)


def gaussian_clipped(seed: int, n: int, F: int, f: int, sigma: float = 0.25):
    """Complex signal, real and imaginary parts N(0, sigma^2) by Box-Muller
    from consecutive uniform pairs, clipped to [-1, 1 - 2^-f]."""
    u = Uniforms(seed)
    vals = np.empty(2 * n)
    for i in range(n):
        u1, u2 = u.next(2)
        r = math.sqrt(-2.0 * math.log(1.0 - u1))
        vals[2 * i] = sigma * r * math.cos(2.0 * math.pi * u2)
        vals[2 * i + 1] = sigma * r * math.sin(2.0 * math.pi * u2)
    vals = np.clip(vals, -1.0, 1.0 - 2.0 ** -f)
    return Signal(1, n, F, f, vals[0::2].copy(), vals[1::2].copy())


def image(seed: int, side: int, F: int, f: int, stream=None):
    """Real image of uniform integer pixels 0..255 scaled by 1/256."""
    u = stream or Uniforms(seed)
    pix = np.floor(256.0 * u.next(side * side))
    return Signal(2, side, F, f, (pix / 256.0).reshape(side, side), None)


# ---------------------------------------------------------------------------
# the named workloads
# ---------------------------------------------------------------------------
WORKLOADS = {
    "fft1d_n8_real_q8.4": "1D N=8 real, U[-1,1), Q(8,4), n_lwe=1",
    "fft1d_n64_cplx_q16.8": "1D N=64 complex, N(0,0.25^2) clipped, Q(16,8), n_lwe=3",
    "fft2d_16x16_real_q16.8": "2D 16x16 image, pixels 0..255 / 256, Q(16,8), n_lwe=1",
}


# Key and encryption seeds of request i of the batched and served mixes.
BATCH_SEED0 = 1000
SERVE_SEED0 = 5000


def workload(name: str):
    """(Signal, n_lwe, seed) of a named single-request workload, or of one
    request of the batched or served mix: "batch4_req<i>" is request i of
    batch_requests(4, ...), "serve5_req<i>" request i of served_requests(5,
    ...), each with n_lwe = 1 and the seed its mix gives it."""
    if name == "fft1d_n8_real_q8.4":
        return uniform_pm1(1, 8, 8, 4, False), 1, 1
    if name == "fft1d_n64_cplx_q16.8":
        return gaussian_clipped(2, 64, 16, 8), 3, 2
    if name == "fft2d_16x16_real_q16.8":
        return image(3, 16, 16, 8), 1, 3
    if name.startswith("batch4_req"):
        i = int(name[len("batch4_req"):])
        return batch_requests(4, i + 1)[i], 1, BATCH_SEED0 + i
    if name.startswith("serve5_req"):
        i = int(name[len("serve5_req"):])
        return served_requests(5, i + 1)[i], 1, SERVE_SEED0 + i
    raise KeyError(name)


def batch_requests(seed: int = 4, count: int = 256, lengths=(8, 16, 32, 64, 128)):
    """Independent 1D requests: length uniform in `lengths` (default
    {8..128}), F uniform in {12, 16, 24} with f = F/2, complex inputs uniform
    in [-1, 1)."""
    u = Uniforms(seed)
    reqs = []
    for _ in range(count):
        a, b = u.next(2)
        n = lengths[min(int(a * len(lengths)), len(lengths) - 1)]
        F = (12, 16, 24)[min(int(b * 3), 2)]
        reqs.append(uniform_pm1(seed, n, F, F // 2, True, stream=u))
    return reqs


def served_requests(seed: int = 5, count: int = 40):
    """Mixed serving traffic: half 1D requests (length uniform in
    {16, 32, 64, 128, 256}, complex inputs uniform in [-1, 1)), half 2D
    images (side uniform in {8, 16, 32}, pixels as in image()), all Q(16,8)."""
    u = Uniforms(seed)
    reqs = []
    for _ in range(count):
        a, b = u.next(2)
        if a < 0.5:
            n = (16, 32, 64, 128, 256)[min(int(b * 5), 4)]
            reqs.append(uniform_pm1(seed, n, 16, 8, True, stream=u))
        else:
            side = (8, 16, 32)[min(int(b * 3), 2)]
            reqs.append(image(seed, side, 16, 8, stream=u))
    return reqs


def poisson_arrivals(seed: int, count: int, rate: float) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process of the given rate:
    exponential gaps -ln(1 - u) / rate from domain-5 uniforms of seed."""
    u = Uniforms(seed).next(count)
    return np.cumsum(-np.log1p(-u) / rate)


def unit_complex(seed: int, n: int, F: int = 32, f: int = 16, stream=None):
    """Complex signal with real and imaginary parts uniform in [0, 1): the
    inputs of the paper's one-dimensional accuracy experiment (section
    "Experimental Results"), in its 32-bit format with 16 fractional bits."""
    u = stream or Uniforms(seed)
    return Signal(1, n, F, f, u.next(n), u.next(n))



@dataclass
class RingDraws:
    """Random draws of ring-GSW key generation and encryption, for n
    ciphertexts of rows x d coefficients: the secret's coefficients
    (ternary, signed), uniform masks in [0, modulus), signed errors in
    [-err_bound, err_bound] and the plaintext bits.  Both the library and the
    oracle take these as inputs; neither draws its own."""
    s: np.ndarray      # (d,) int64 in {-1, 0, 1}
    a: np.ndarray      # (n, rows, d) uint64 in [0, modulus)
    e: np.ndarray      # (n, rows, d) int64 in [-err_bound, err_bound]
    bits: np.ndarray   # (n,) uint8 in {0, 1}


def ring_draws(seed: int, n: int, d: int, rows: int, modulus: int, err_bound: int = 2, bits=None) -> RingDraws:
    """Seeded draws (numpy PCG64) for n ring ciphertexts; bits default to
    uniform random bits."""
    g = np.random.Generator(np.random.PCG64(seed))
    s = g.integers(-1, 2, size=d, dtype=np.int64)
    a = g.integers(0, modulus, size=(n, rows, d), dtype=np.uint64)
    e = g.integers(-err_bound, err_bound + 1, size=(n, rows, d), dtype=np.int64)
    if bits is None:
        bits = g.integers(0, 2, size=n, dtype=np.uint8)
    return RingDraws(s, a, e, np.ascontiguousarray(np.asarray(bits, dtype=np.uint8)))
