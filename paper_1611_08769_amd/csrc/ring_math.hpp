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

}  // namespace ring
}  // namespace sfft
