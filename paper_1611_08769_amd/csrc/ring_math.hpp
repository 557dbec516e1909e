// Arithmetic of R_p = Z_p[X]/(X^d + 1), p = 2^62 - 2^16 + 1, shared by the
// ring-GSW kernels and their host-side table set-up.
//
// p is prime and 2^16 divides p - 1, so Z_p holds a primitive 2d-th root of
// unity psi for every d <= 2^15, and the negacyclic product of two
// polynomials is a pointwise product after the transform
//   A_k = sum_t a_t psi^t omega^(t k),  omega = psi^2
// (the "twisted" cyclic transform).  The transforms below fold the twist into
// their twiddles: the forward one is Cooley-Tukey from natural order to
// bit-reversed order with twiddles psi^brv(m+i), the inverse one
// Gentleman-Sande from bit-reversed to natural order with psi^-brv(m+i),
// followed by a scaling by d^-1 (the merged negacyclic NTT of Poppelmann,
// Oder and Guneysu, Latincrypt 2015, and Longa and Naehrig, CANS 2016).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace sfft {
namespace ring {

constexpr uint64_t kP = 0x3FFFFFFFFFFF0001ULL;  // 2^62 - 2^16 + 1
constexpr int kEll = 62;                         // bits of p: the gadget's length
constexpr int kRows = 2 * kEll;                  // rows of a ciphertext
constexpr uint64_t kM62 = (1ULL << 62) - 1;
constexpr int kMaxLogD = 11;                     // d <= 2048

__host__ __device__ __forceinline__ uint64_t addp(uint64_t a, uint64_t b)
{
    uint64_t s = a + b;  // a, b < p < 2^62: no wrap
    return s >= kP ? s - kP : s;
}

__host__ __device__ __forceinline__ uint64_t subp(uint64_t a, uint64_t b) { return a >= b ? a - b : a + kP - b; }

// 128-bit product of a, b < 2^62 from four 32 x 32 -> 64-bit partial
// products (one v_mad_u64_u32 each on the device): the cross terms are below
// 2^62, so their sum cannot wrap.
__host__ __device__ __forceinline__ void mul128(uint64_t a, uint64_t b, uint64_t* lo, uint64_t* hi)
{
    const uint64_t al = (uint32_t)a, ah = a >> 32, bl = (uint32_t)b, bh = b >> 32;
    const uint64_t mid = al * bh + ah * bl;   // < 2^63
    const uint64_t p0 = al * bl;
    const uint64_t l = p0 + (mid << 32);
    *lo = l;
    *hi = ah * bh + (mid >> 32) + (l < p0);
}

// a*b mod p for a, b < p.  With 2^62 = 2^16 - 1 (mod p), a 124-bit product
// x = xh*2^62 + xl reduces as xh*2^16 - xh + xl; xh*2^16 splits once more at
// bit 62 the same way.  Every intermediate stays below 2^64.
__host__ __device__ __forceinline__ uint64_t mulp(uint64_t a, uint64_t b)
{
    uint64_t lo, hi;
    mul128(a, b, &lo, &hi);
    const uint64_t xl = lo & kM62;
    const uint64_t xh = (hi << 2) | (lo >> 62);     // < 2^62
    const uint64_t yh = xh >> 46;                   // xh*2^16 = yh*2^62 + yl
    const uint64_t yl = (xh << 16) & kM62;
    const uint64_t xr = xh >= kP ? xh - kP : xh;    // xh mod p
    // z = xl + yl + yh*(2^16 - 1) + (p - xr) = x (mod p), z < 2^63 + 2^62 + 2^32
    const uint64_t z = xl + yl + ((yh << 16) - yh) + (kP - xr);
    const uint64_t zh = z >> 62, zl = z & kM62;     // zh <= 2
    const uint64_t w = zl + ((zh << 16) - zh);      // < 2^62 + 2^18 < 2p
    return w >= kP ? w - kP : w;
}

// x mod p for a 128-bit x = hi*2^64 + lo below 2^126 (a sum of up to four
// products of residues).  x = xh*2^62 + xl with xh < 2^64; xh*2^62 = xh*(2^16 - 1)
// and xh*2^16 splits again at bit 62; -xh enters as p - (xh mod p).
__host__ __device__ __forceinline__ uint64_t red126(uint64_t lo, uint64_t hi)
{
    const uint64_t xl = lo & kM62;
    const uint64_t xh = (hi << 2) | (lo >> 62);
    const uint64_t yh = xh >> 46, yl = (xh << 16) & kM62;
    uint64_t xr = (xh & kM62) + (((xh >> 62) << 16) - (xh >> 62));  // xh mod p, below 2p
    xr = xr >= kP ? xr - kP : xr;
    const uint64_t z = xl + yl + ((yh << 16) - yh) + (kP - xr);      // < 3*2^62 + 2^34
    const uint64_t zh = z >> 62, zl = z & kM62;
    const uint64_t w = zl + ((zh << 16) - zh);
    return w >= kP ? w - kP : w;
}

// (hi, lo) += a*b for residues a, b (no reduction).
__host__ __device__ __forceinline__ void mac128(uint64_t a, uint64_t b, uint64_t* lo, uint64_t* hi)
{
    uint64_t l, h;
    mul128(a, b, &l, &h);
    const uint64_t s = *lo + l;
    *hi += h + (s < l);
    *lo = s;
}

// A constant multiplier w < p with its Shoup quotient ws = floor(w * 2^64 / p)
// (V. Shoup, NTL; D. Harvey, "Faster arithmetic for number-theoretic
// transforms", J. Symb. Comp. 2014).
struct Tw {
    uint64_t w, ws;
};

// a*w mod p for a < p by Shoup's method: q = floor(a*ws / 2^64) estimates
// floor(a*w / p) from below by at most 1, so a*w - q*p (computed mod 2^64)
// lies in [0, 2p).  q is taken from three of the four partial products of
// a*ws (the dropped low one moves it down by at most 1 more), so the
// remainder lies in [0, 3p) before the final corrections.  q*p mod 2^64 is
// (q << 62) - (q << 16) + q.
__host__ __device__ __forceinline__ uint64_t mulw(uint64_t a, Tw t)
{
    const uint64_t al = (uint32_t)a, ah = a >> 32, wl = (uint32_t)t.ws, wh = t.ws >> 32;
    const uint64_t m1 = al * wh, m2 = ah * wl;
    const uint64_t ms = m1 + m2;
    const uint64_t q = ah * wh + (ms >> 32) + ((uint64_t)(ms < m1) << 32);
    uint64_t r = a * t.w - ((q << 62) - (q << 16) + q);
    r = r >= 2 * kP ? r - 2 * kP : r;
    return r >= kP ? r - kP : r;
}

inline uint64_t powp(uint64_t a, uint64_t e)
{
    uint64_t r = 1;
    while (e) {
        if (e & 1) r = mulp(r, a);
        a = mulp(a, a);
        e >>= 1;
    }
    return r;
}

// Residue of a small signed integer.
__host__ __device__ __forceinline__ uint64_t from_signed(int64_t v)
{
    return v >= 0 ? (uint64_t)v % kP : kP - (uint64_t)(-v) % kP;
}

// ---- transforms, one LDS round at a time --------------------------------
// The caller runs the rounds in order with a barrier after each; a round
// spreads its butterflies over nt threads (thread tid takes every nt-th).
// np polynomials of 2^LOGD coefficients lie back to back at a.  tw holds the
// 2^LOGD twiddles of the direction, index m + i for group i of a stage with
// m groups.

// Cooley-Tukey butterfly (x, y) -> (x + w*y, x - w*y); Gentleman-Sande
// butterfly (x, y) -> (x + y, (x - y)*w).
__host__ __device__ __forceinline__ void bf_ct(uint64_t& x, uint64_t& y, Tw t)
{
    const uint64_t v = mulw(y, t);
    y = subp(x, v);
    x = addp(x, v);
}
__host__ __device__ __forceinline__ void bf_gs(uint64_t& x, uint64_t& y, Tw t)
{
    const uint64_t u = x;
    x = addp(u, y);
    y = mulw(subp(u, y), t);
}
// A Cooley-Tukey butterfly whose y is 0 or 1 (a digit): the product is a select.
__host__ __device__ __forceinline__ void bf_ct_bit(uint64_t& x, uint64_t& y, Tw t)
{
    const uint64_t v = y ? t.w : 0;
    y = subp(x, v);
    x = addp(x, v);
}

// Forward round starting at stage s (natural -> bit-reversed order): stages s
// and s+1 as radix-4 on quadruples, or stage s alone when it is the last.
// binary: the inputs are 0/1 (only meaningful for s = 0).
template <int LOGD, int NP>
__host__ __device__ __forceinline__ void fwd_round(uint64_t* a, int s, const Tw* tw, int tid, int nt, bool binary)
{
    constexpr int D = 1 << LOGD;
    if (s + 1 < LOGD) {
        const int t = D >> (s + 1), h = t >> 1, m = 1 << s;
        constexpr int Q = D >> 2;
        for (int b = tid; b < NP * Q; b += nt) {
            const int q = b / Q, bb = b % Q;
            const int i = bb / h, j = bb % h;
            uint64_t* p = a + q * D + 2 * i * t + j;
            uint64_t x0 = p[0], x1 = p[h], x2 = p[t], x3 = p[t + h];
            const Tw w1 = tw[m + i];
            if (binary && s == 0) {
                bf_ct_bit(x0, x2, w1);
                bf_ct_bit(x1, x3, w1);
            } else {
                bf_ct(x0, x2, w1);
                bf_ct(x1, x3, w1);
            }
            bf_ct(x0, x1, tw[2 * m + 2 * i]);
            bf_ct(x2, x3, tw[2 * m + 2 * i + 1]);
            p[0] = x0;
            p[h] = x1;
            p[t] = x2;
            p[t + h] = x3;
        }
    } else if (s < LOGD) {
        constexpr int H = D >> 1;
        for (int b = tid; b < NP * H; b += nt) {
            const int q = b / H, i = b % H;
            uint64_t* p = a + q * D + 2 * i;
            if (binary && s == 0)
                bf_ct_bit(p[0], p[1], tw[H + i]);
            else
                bf_ct(p[0], p[1], tw[H + i]);
        }
    }
}

// Inverse round (bit-reversed -> natural order): pair = stages s and s-1 as
// radix-4, else stage s alone.
template <int LOGD, int NP>
__host__ __device__ __forceinline__ void inv_round(uint64_t* a, int s, bool pair, const Tw* tw, int tid, int nt)
{
    constexpr int D = 1 << LOGD;
    if (pair) {
        const int t = D >> (s + 1), m = 1 << s;
        constexpr int Q = D >> 2;
        for (int b = tid; b < NP * Q; b += nt) {
            const int q = b / Q, bb = b % Q;
            const int i2 = bb / t, j = bb % t;
            uint64_t* p = a + q * D + 4 * i2 * t + j;
            uint64_t x0 = p[0], x1 = p[t], x2 = p[2 * t], x3 = p[3 * t];
            bf_gs(x0, x1, tw[m + 2 * i2]);
            bf_gs(x2, x3, tw[m + 2 * i2 + 1]);
            const Tw w2 = tw[(m >> 1) + i2];
            bf_gs(x0, x2, w2);
            bf_gs(x1, x3, w2);
            p[0] = x0;
            p[t] = x1;
            p[2 * t] = x2;
            p[3 * t] = x3;
        }
    } else {
        const int t = D >> (s + 1), m = 1 << s;
        for (int b = tid; b < NP * (D >> 1); b += nt) {
            const int q = b / (D >> 1), bb = b % (D >> 1);
            const int i = bb / t, j = bb % t;
            uint64_t* p = a + q * D + 2 * i * t + j;
            bf_gs(p[0], p[t], tw[m + i]);
        }
    }
}

// Round schedules.  Forward: rounds start at s = 0, 2, 4, ... (< LOGD).
// Inverse: with LOGD odd, stage LOGD-1 alone first; then pairs (s, s-1) for s
// descending by 2 down to 1.
template <int LOGD>
__host__ __device__ __forceinline__ int inv_stage(int r, bool* pair)
{
    if (LOGD & 1) {
        *pair = r > 0;
        return r == 0 ? LOGD - 1 : LOGD - 2 - 2 * (r - 1);
    }
    *pair = true;
    return LOGD - 1 - 2 * r;
}
constexpr int rounds_of(int logd) { return (logd + 1) / 2; }

}  // namespace ring
}  // namespace sfft
