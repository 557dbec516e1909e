"""Oracle: plaintext two's-complement fixed-point FFT (the plain definition of
what the encrypted circuit decrypts to).  TEST INFRASTRUCTURE ONLY.

Paper, section "FFT in FHE": numbers are F-bit binary words with a power-of-two
scale (fixed point), addition/subtraction keep the fractional width, a
multiplication sign-extends to 2F bits and keeps the middle bits (an implicit
division by the scale), the FFT bit-reverses its input and runs log2(N)
butterfly stages with plaintext twiddles.  Section "Error Analysis": the only
error source is the float-to-fixed conversion ("truncation"); Theorem 2 bounds
the error by Delta*(N/2)*(log N + X_b + 1).

Everything here is int64 numpy arithmetic, vectorised over a leading batch
axis, wrapping mod 2^F like the gate circuit (adders drop the carry-out, the
multiplier drops high bits).
"""
from __future__ import annotations

import math

import numpy as np


def wrap(v, F):
    """Reduce to the signed F-bit range [-2^(F-1), 2^(F-1))."""
    v = np.asarray(v, dtype=np.int64)
    m = np.int64(1) << F
    return ((v + (m >> 1)) % m) - (m >> 1)


def quantize(x, F, f):
    """floor(x * 2^f): the paper's truncation of a real to Q(F, f).  Raises
    if a value does not fit F bits."""
    q = np.floor(np.asarray(x, dtype=np.float64) * float(1 << f)).astype(np.int64)
    lo, hi = -(1 << (F - 1)), (1 << (F - 1))
    if np.any(q < lo) or np.any(q >= hi):
        raise ValueError("input does not fit Q(%d,%d)" % (F, f))
    return q


def fx_add(a, b, F):
    return wrap(a + b, F)


def fx_sub(a, b, F):
    return wrap(a - b, F)


def fx_mul(x, c, F, f):
    """floor(x*c / 2^f) mod 2^F with x, c signed: the middle bits [f, f+F) of
    the 2F-bit two's-complement product (numpy's >> on int64 is an
    arithmetic shift, i.e. floor division by 2^f)."""
    return wrap((np.asarray(x, dtype=np.int64) * np.int64(c)) >> f, F)


def round_half_away(v: float) -> int:
    a = math.floor(abs(v) + 0.5)
    return int(a) if v >= 0 else -int(a)


def twiddle(j: int, m: int, f: int):
    """exp(-2 pi i j/m) quantised to Q(., f), rounded half away from zero."""
    ang = 2.0 * math.pi * j / m
    return (round_half_away(math.cos(ang) * (1 << f)),
            round_half_away(-math.sin(ang) * (1 << f)))


def twiddle_tie_margin(m: int, f: int) -> float:
    """Smallest distance of |w|*2^f to a rounding tie over the stage's
    twiddles (0 would make the rounding direction ambiguous)."""
    best = 1.0
    for j in range(m // 2):
        ang = 2.0 * math.pi * j / m
        for v in (math.cos(ang), -math.sin(ang)):
            fr = abs(v) * (1 << f)
            fr -= math.floor(fr)
            best = min(best, abs(fr - 0.5))
    return best


def _bitrev(i, lg):
    r = 0
    for _ in range(lg):
        r = (r << 1) | (i & 1)
        i >>= 1
    return r


def fft1d_fixed(re, im, F, f):
    """Radix-2 DIT FFT over the last axis of int64 arrays (batch, N)."""
    re = np.asarray(re, dtype=np.int64)
    im = np.asarray(im, dtype=np.int64)
    N = re.shape[-1]
    lg = N.bit_length() - 1
    assert 1 << lg == N
    perm = [_bitrev(i, lg) for i in range(N)]
    xr = re[..., perm].copy()
    xi = im[..., perm].copy()
    one = 1 << f
    for s in range(1, lg + 1):
        m = 1 << s
        h = m // 2
        for g in range(0, N, m):
            for j in range(h):
                cr, ci = twiddle(j, m, f)
                p, q = g + j, g + j + h
                ar, ai = xr[..., p].copy(), xi[..., p].copy()
                br, bi = xr[..., q].copy(), xi[..., q].copy()
                if (cr, ci) == (one, 0):
                    tr, ti = br, bi
                elif (cr, ci) == (0, -one):
                    tr, ti = bi, wrap(-br, F)
                else:
                    tr = fx_sub(fx_mul(br, cr, F, f), fx_mul(bi, ci, F, f), F)
                    ti = fx_add(fx_mul(bi, cr, F, f), fx_mul(br, ci, F, f), F)
                xr[..., p] = fx_add(ar, tr, F)
                xi[..., p] = fx_add(ai, ti, F)
                xr[..., q] = fx_sub(ar, tr, F)
                xi[..., q] = fx_sub(ai, ti, F)
    return xr, xi


def fft2d_fixed(re, im, F, f):
    """Row-column 2D FFT of (batch, S, S) arrays: every row, then every
    column, no rescaling between the passes."""
    re = np.asarray(re, dtype=np.int64)
    im = np.asarray(im, dtype=np.int64)
    r1, i1 = fft1d_fixed(re, im, F, f)
    r2, i2 = fft1d_fixed(np.swapaxes(r1, -1, -2), np.swapaxes(i1, -1, -2), F, f)
    return np.swapaxes(r2, -1, -2), np.swapaxes(i2, -1, -2)


def fft_fixed(dims, re, im, F, f):
    if dims == 1:
        return fft1d_fixed(re, im, F, f)
    return fft2d_fixed(re, im, F, f)


# ---------------------------------------------------------------------------
# error analysis
# ---------------------------------------------------------------------------
def error_bound(N: int, f: int, xb: float) -> float:
    """Theorem 2: Delta*(N/2)*(log2 N + X_b + 1) with Delta = 2^-f."""
    return (2.0 ** -f) * (N / 2.0) * (math.log2(N) + xb + 1.0)


def wrapped_error(fixed_val, exact, F, f):
    """|fixed/2^f - exact| measured modulo the representable range 2^(F-f)
    (the circuit wraps mod 2^F, so a true value outside the range is compared
    after the same wrap)."""
    span = 2.0 ** (F - f)
    d = np.asarray(fixed_val, dtype=np.float64) / (1 << f) - np.asarray(exact)
    d = (d + span / 2) % span - span / 2
    return np.abs(d)


def error_stats(errs):
    """Total, mean, population variance and standard deviation of absolute
    errors (the columns of Table 1)."""
    e = np.asarray(errs, dtype=np.float64).ravel()
    return dict(total=float(e.sum()), mean=float(e.mean()),
                var=float(e.var()), sd=float(e.std()))


# ---------------------------------------------------------------------------
# bits <-> words
# ---------------------------------------------------------------------------
def words_to_bits(vals, F):
    """Signed words -> list of bits, word-major, LSB first."""
    out = []
    for v in np.asarray(vals, dtype=np.int64).ravel():
        u = int(v) & ((1 << F) - 1)
        out.extend((u >> i) & 1 for i in range(F))
    return out


def bits_to_words(bits, F):
    bits = list(bits)
    assert len(bits) % F == 0
    out = []
    for w in range(len(bits) // F):
        u = 0
        for i in range(F):
            u |= (bits[w * F + i] & 1) << i
        if u >= 1 << (F - 1):
            u -= 1 << F
        out.append(u)
    return np.array(out, dtype=np.int64)
