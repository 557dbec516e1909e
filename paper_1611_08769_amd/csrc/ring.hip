// Ring-GSW gates on gfx950: GSW13 over R_p = Z_p[X]/(X^d + 1),
// p = 2^62 - 2^16 + 1 (GSW13's ring instantiation of the scheme of the
// paper's section "Notation and Background"; gates as in Lemma "binary
// gates").
//
// A ciphertext is 2*ell rows x 2 columns of polynomials (ell = 62), stored
// (row, column, coefficient) as uint64 residues in [0, p).  The product of
// two ciphertexts is P = G^-1(L) * R, where G^-1 splits every coefficient of
// L into its ell bits: row i of P is the sum over the 2*ell digit
// polynomials D_ij (bit j mod ell of L[i][j div ell]) of D_ij * R[j], each a
// negacyclic product.  The kernels compute it in the transform domain:
//   k_ring_fwd      forward transform of every polynomial of R (once per gate)
//   k_ring_product  one workgroup per (ciphertext, row i): for each digit,
//                   build D_ij in LDS, transform it there, multiply-accumulate
//                   against R's transformed row j in registers; then the
//                   inverse transform of the two accumulated polynomials and
//                   the gate's affine epilogue in the coefficient domain.
//                   Twiddles are read from the (L1-resident) global tables,
//                   which keeps the workgroup's LDS at 48 KB for d = 1024
//                   (three workgroups per CU).
//   k_ring_linear   NOT and XADD (no product)
//   k_ring_encrypt  one workgroup per (ciphertext, row): a*s by transforms,
//                   plus the error and the gadget
// and the refresh of LWE ciphertexts mod p (refresh is only mentioned by the
// paper's section "Error Analysis"; this is the FHEW/TFHE construction with
// these ring-GSW ciphertexts as the key):
//   k_ring_br_init       modulus switch to 2d, accumulator and rotations
//   k_ring_blind_rotate  one workgroup per accumulator runs all its CMux
//                        steps, each one row of the same product
//   k_ring_extract       coefficient 0 as an LWE ciphertext (ring secret)
//   k_ring_keyswitch     back to the LWE secret
// (k_ring_br_init also forms the linear combination of two ciphertexts that
// turns a refresh into a bootstrapped AND, OR, NAND or XOR gate)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "netlist.hpp"
#include "ring_math.hpp"
#include "sfft.h"

int sfft_fail(int code, const std::string& msg);
int sfft_hip_fail(hipError_t e, const char* where);
bool sfft_shape_check(const sfft_shape* s, std::string* why);
sfft::Shape sfft_shape_of(const sfft_shape* s);

using namespace sfft::ring;

namespace {

constexpr int kT = 256;  // threads per workgroup

// Transform tables of one d, on the device: forward twiddles psi^brv(k)
// [0, d), inverse twiddles psi^-brv(k) [d, 2d), each with its Shoup
// quotient, and d^-1.
struct TwView {
    const Tw* fwd;
    const Tw* inv;
    Tw dinv;
};

__device__ __forceinline__ void copy_lds(uint64_t* dst, const uint64_t* src, int count)
{
    for (int t = threadIdx.x; t < count; t += kT) dst[t] = src[t];
}

// Forward transforms (natural -> bit-reversed order) of NP polynomials held
// back to back in LDS, two stages per barrier.  binary: the inputs are 0/1,
// so the first stage's products are selects.
template <int LOGD, int NP>
__device__ __forceinline__ void fwd_lds(uint64_t* a, const Tw* tw, bool binary)
{
#pragma unroll
    for (int s = 0; s < LOGD; s += 2) {
        fwd_round<LOGD, NP>(a, s, tw, threadIdx.x, kT, binary);
        __syncthreads();
    }
}

// Inverse transforms (bit-reversed -> natural order, without the d^-1
// scaling) of NP polynomials in LDS.
template <int LOGD, int NP>
__device__ __forceinline__ void inv_lds(uint64_t* a, const Tw* tw)
{
#pragma unroll
    for (int r = 0; r < rounds_of(LOGD); ++r) {
        bool pair;
        const int s = inv_stage<LOGD>(r, &pair);
        inv_round<LOGD, NP>(a, s, pair, tw, threadIdx.x, kT);
        __syncthreads();
    }
}

// Workgroup order -> (ciphertext, row), keeping the rows of one ciphertext on
// one XCD (workgroups are dealt to the 8 XCDs round robin) so that the rows
// share that XCD's L2 copy of the transformed right operand.
__device__ __forceinline__ int64_t xcd_order(int64_t b, int64_t nb)
{
    const int64_t nb8 = nb & ~(int64_t)7;
    return b < nb8 ? (b & 7) * (nb8 >> 3) + (b >> 3) : b;
}

// Gadget entry of (row, column, coefficient t).
__device__ __forceinline__ uint64_t gadget(int row, int col, int t)
{
    return (t == 0 && col == row / kEll) ? (1ULL << (row % kEll)) : 0;
}

__device__ __forceinline__ uint64_t epilogue(int op, uint64_t P, uint64_t l, uint64_t r, uint64_t g)
{
    switch (op) {
    case 4: case 9: return P;
    case 5: return subp(addp(l, r), addp(P, P));
    case 6: return subp(addp(l, r), P);
    default: return subp(g, P);  // 8: NAND
    }
}

// Digit polynomials per pass of the product kernel: 4, or 2 at d = 2048
// (LDS).  Buffers: at least 2 (the two accumulators at the end).
template <int LOGD>
struct ProdShape {
    static constexpr int D = 1 << LOGD;
    static constexpr int DG = LOGD >= 11 ? 2 : 4;   // also bounds the unreduced pointwise sums (<= 4 terms)
    static constexpr int NB = DG > 2 ? DG : 2;
    static constexpr int PER = D >= kT ? D / kT : 1;        // coefficients per thread
    static constexpr size_t lds = (size_t)(2 * D + NB * D) * 8;  // L row, digits
};

// Forward transforms of rows (both columns of each) of src into dst.
template <int LOGD>
__global__ __launch_bounds__(kT) void k_ring_fwd(const uint64_t* __restrict__ src, uint64_t* __restrict__ dst,
                                                 TwView tw)
{
    constexpr int D = 1 << LOGD;
    extern __shared__ uint64_t lds[];
    Tw* t_f = reinterpret_cast<Tw*>(lds);
    uint64_t* buf = lds + 2 * D;
    const int64_t row = blockIdx.x;
    copy_lds(lds, reinterpret_cast<const uint64_t*>(tw.fwd), 2 * D);
    copy_lds(buf, src + row * 2 * D, 2 * D);
    __syncthreads();
    fwd_lds<LOGD, 2>(buf, t_f, false);
    uint64_t* o = dst + row * 2 * D;
    for (int t = threadIdx.x; t < 2 * D; t += kT) o[t] = buf[t];
}

// One row of G^-1(L) * R: src(col, t) gives coefficient t of column col of
// the row of L (a pair of polynomials), and rn holds R's 2*ell rows
// transformed (2D words each).  For each group of DG digit polynomials (bit j
// mod ell of the row's column j div ell), transform them in dig and
// multiply-accumulate against rn in registers; at the end the two sums are
// transformed back and left, not yet scaled by d^-1, in dig[0, 2D).  Starts
// and ends with a barrier.
template <int LOGD, typename Src>
__device__ __forceinline__ void row_product(Src src, const uint64_t* __restrict__ rn, uint64_t* dig,
                                            const TwView& tw)
{
    using S = ProdShape<LOGD>;
    constexpr int D = S::D, DG = S::DG, PER = S::PER;
    uint64_t acc0[PER], acc1[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) acc0[q] = acc1[q] = 0;
    __syncthreads();

    for (int jj0 = 0; jj0 < kRows; jj0 += DG) {
        // digit polynomials jj0 .. jj0+DG-1: bit (jj mod ell) of column jj div ell
        for (int b = threadIdx.x; b < DG * D; b += kT) {
            const int jj = jj0 + b / D, t = b % D;
            dig[b] = (src(jj / kEll, t) >> (jj % kEll)) & 1;
        }
        __syncthreads();
        fwd_lds<LOGD, DG>(dig, tw.fwd, true);
        // pointwise products against R's transformed rows jj0..jj0+DG-1,
        // summed unreduced (DG <= 4 products stay below 2^126), reduced once
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int k = threadIdx.x + q * kT;
            if (D >= kT || k < D) {
                uint64_t l0 = 0, h0 = 0, l1 = 0, h1 = 0;
#pragma unroll
                for (int g = 0; g < DG; ++g) {
                    const uint64_t* r0 = rn + (int64_t)(jj0 + g) * 2 * D;
                    const uint64_t x = dig[g * D + k];
                    mac128(x, r0[k], &l0, &h0);
                    mac128(x, r0[D + k], &l1, &h1);
                }
                acc0[q] = addp(acc0[q], red126(l0, h0));
                acc1[q] = addp(acc1[q], red126(l1, h1));
            }
        }
        __syncthreads();
    }

    // both accumulated polynomials back to coefficients
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int k = threadIdx.x + q * kT;
        if (D >= kT || k < D) {
            dig[k] = acc0[q];
            dig[D + k] = acc1[q];
        }
    }
    __syncthreads();
    inv_lds<LOGD, 2>(dig, tw.inv);
}

// out[c] = op(L[c], R[c]) for the product gates (AND, XOR, OR, NAND,
// PRODUCT).  Rn: R's rows, transformed.
template <int LOGD>
__global__ __launch_bounds__(kT) void k_ring_product(const uint64_t* __restrict__ L, const uint64_t* __restrict__ R,
                                                     const uint64_t* __restrict__ Rn, uint64_t* __restrict__ out,
                                                     int64_t nblocks, TwView tw, int op)
{
    constexpr int D = 1 << LOGD;
    extern __shared__ uint64_t lds[];
    uint64_t* lrow = lds;                   // row i of L: 2D
    uint64_t* dig = lrow + 2 * D;           // NB polynomials
    const int64_t lb = xcd_order(blockIdx.x, nblocks);
    const int64_t c = lb / kRows;
    const int i = (int)(lb % kRows);
    const int64_t row_off = (c * kRows + i) * 2 * D;

    copy_lds(lrow, L + row_off, 2 * D);
    row_product<LOGD>([lrow](int col, int t) { return lrow[col * D + t]; }, Rn + c * kRows * 2 * D, dig, tw);

    const uint64_t* rrow = R + row_off;
    uint64_t* orow = out + row_off;
    for (int b = threadIdx.x; b < 2 * D; b += kT) {
        const int col = b / D, t = b % D;
        const uint64_t P = mulw(dig[b], tw.dinv);
        orow[b] = epilogue(op, P, lrow[b], rrow[b], gadget(i, col, t));
    }
}

// Blind rotation of m ring-LWE accumulators (2D words each, in place) by a
// key of n ring-GSW ciphertexts, transformed (bkt: n x 2*ell rows of 2D
// words).  Workgroup j runs all n steps of accumulator j:
//   acc <- acc + G^-1(X^r acc - acc) * bk[i],  r = rot[j*n + i] mod 2D
// (the CMux of bk[i]'s bit between acc and X^r acc; X^D = -1).
template <int LOGD>
__global__ __launch_bounds__(kT) void k_ring_blind_rotate(const uint64_t* __restrict__ bkt, int64_t n,
                                                          const int32_t* __restrict__ rot, uint64_t* __restrict__ acc,
                                                          TwView tw)
{
    constexpr int D = 1 << LOGD;
    extern __shared__ uint64_t lds[];
    uint64_t* a = lds;            // the accumulator: 2D
    uint64_t* dig = a + 2 * D;    // NB polynomials
    const int64_t j = blockIdx.x;
    uint64_t* ga = acc + j * 2 * D;
    copy_lds(a, ga, 2 * D);
    for (int64_t i = 0; i < n; ++i) {
        const int r = ((rot[j * n + i] % (2 * D)) + 2 * D) % (2 * D);
        // coefficient t of column col of X^r a - a, formed where the digits
        // are taken (X^r a at t is +a[u], or -a[u - D] past the wrap)
        auto dif = [a, r](int col, int t) {
            const int u = (t - r + 2 * D) % (2 * D);
            const uint64_t v = u < D ? a[col * D + u] : subp(0, a[col * D + u - D]);
            return subp(v, a[col * D + t]);
        };
        row_product<LOGD>(dif, bkt + i * kRows * 2 * D, dig, tw);
        for (int b = threadIdx.x; b < 2 * D; b += kT) a[b] = addp(a[b], mulw(dig[b], tw.dinv));
        __syncthreads();
    }
    for (int b = threadIdx.x; b < 2 * D; b += kT) ga[b] = a[b];
}

// floor((x * 2D + floor(p/2)) / p) mod 2D for x < p: x switched to the
// modulus 2D with rounding.  y = x*2D + floor(p/2) < 2^75 is split at bit 62;
// with 2^62 = p + 2^16 - 1 the quotient estimate y >> 62 leaves a remainder
// below 2p, corrected once.
template <int LOGD>
__device__ __forceinline__ int32_t switch_2d(uint64_t x)
{
    constexpr uint64_t half = kP / 2;
    const uint64_t lo0 = x << (LOGD + 1), hi0 = x >> (63 - LOGD);
    const uint64_t lo = lo0 + half, hi = hi0 + (lo < lo0);
    uint64_t q = (hi << 2) | (lo >> 62);
    uint64_t r = (lo & kM62) + ((q << 16) - q);
    if (r >= kP) ++q;
    return (int32_t)(q & ((2u << LOGD) - 1));
}

// cx * v for a small signed coefficient cx in {-1, 0, 1, 2}.
__device__ __forceinline__ uint64_t small_mul(int cx, uint64_t v)
{
    return cx == 1 ? v : cx == 2 ? addp(v, v) : cx == -1 ? subp(0, v) : 0;
}

// The linear combination of a bootstrapped gate (bits encoded as mu * 2 *
// floor(p/8)): c = cx*x + cy*y + (0, .., 0, k*floor(p/8)).
__host__ __device__ __forceinline__ void gate_combination(int gate, int* cx, int* cy, uint64_t* cb)
{
    int k;
    switch (gate) {
    case 4: *cx = 1, *cy = 1, k = -1; break;   // AND
    case 6: *cx = 1, *cy = 1, k = 1; break;    // OR
    case 8: *cx = -1, *cy = -1, k = 5; break;  // NAND
    default: *cx = 2, *cy = 2, k = 0; break;   // XOR (and XADD)
    }
    *cb = k >= 0 ? (uint64_t)k * (kP / 8) : kP - (uint64_t)(-k) * (kP / 8);
}

// Gate bootstrapping, step 1: for LWE ciphertext j, c = cx*x_j + cy*y_j
// (+ cb on b) with c = (a_0..a_{n-1}, b), the rotations -a~_i mod 2D and
// the accumulator (X^(b~ + D/2) * TV, 0), TV = delta * (1 + X + ... +
// X^(D-1)).  y may be null (cy = 0).
template <int LOGD>
__global__ __launch_bounds__(kT) void k_ring_br_init(const uint64_t* __restrict__ x, const uint64_t* __restrict__ y,
                                                     const int32_t* __restrict__ xi, const int32_t* __restrict__ yi,
                                                     const int32_t* __restrict__ gk, int cx, int cy, uint64_t cb,
                                                     int64_t n, int32_t* __restrict__ rot, uint64_t* __restrict__ acc,
                                                     uint64_t delta)
{
    constexpr int D = 1 << LOGD;
    const int64_t j = blockIdx.x;
    if (gk) gate_combination(gk[j], &cx, &cy, &cb);   // per-row gate (mixed-gate calls)
    // operand j is row j, or row xi[j] / yi[j] of a slot array
    const uint64_t* xc = x + (xi ? (int64_t)xi[j] : j) * (n + 1);
    const uint64_t* yc = y ? y + (yi ? (int64_t)yi[j] : j) * (n + 1) : nullptr;
    auto coord = [&](int64_t i) {
        const uint64_t v = small_mul(cx, xc[i]);
        return yc ? addp(v, small_mul(cy, yc[i])) : v;
    };
    for (int64_t i = threadIdx.x; i < n; i += kT) rot[j * n + i] = (2 * D - switch_2d<LOGD>(coord(i))) % (2 * D);
    const int k = (switch_2d<LOGD>(addp(coord(n), cb)) + D / 2) % (2 * D);
    uint64_t* a = acc + j * 2 * D;
    for (int u = threadIdx.x; u < D; u += kT) {
        a[u] = ((u - k + 2 * D) % (2 * D)) < D ? delta : kP - delta;
        a[D + u] = 0;
    }
}

// Gate bootstrapping, step 3: coefficient 0 of accumulator j as an LWE
// ciphertext under the ring secret's coefficients, (a_0, -a_{D-1}, ...,
// -a_1, b_0 + delta).
template <int LOGD>
__global__ __launch_bounds__(kT) void k_ring_extract(const uint64_t* __restrict__ acc, uint64_t* __restrict__ out,
                                                     uint64_t delta)
{
    constexpr int D = 1 << LOGD;
    const int64_t j = blockIdx.x;
    const uint64_t* a = acc + j * 2 * D;
    uint64_t* o = out + j * (D + 1);
    for (int t = threadIdx.x; t <= D; t += kT)
        o[t] = t == D ? addp(a[0], delta) : (t == 0 ? a[D] : subp(0, a[2 * D - t]));
}

// Key switching of LWE ciphertext j (a'_0..a'_{d-1}, b') under the ring
// secret to the LWE secret of ksk ([t][k][n+1]: an encryption of
// s_ring[t] * 16^k): out = (0, .., 0, b') - sum_{t,k} digit_k(a'_t) ksk[t][k].
// One workgroup per ciphertext, a thread per output coordinate; the a'_t
// sit in LDS, the key is read coalesced along the coordinate (L2-resident
// across workgroups), and each coordinate's sum of d*16 products of a 4-bit
// digit by a residue (below 2^80) is kept unreduced and reduced once.
constexpr int kKsDigits = 16;  // base-16 digits of a residue below 2^64
__global__ __launch_bounds__(kT) void k_ring_keyswitch(const uint64_t* __restrict__ ksk, const uint64_t* __restrict__ in,
                                                       uint64_t* __restrict__ out, const int32_t* __restrict__ oi, int d,
                                                       int64_t n)
{
    extern __shared__ uint64_t lds[];
    const int64_t j = blockIdx.x;
    const uint64_t* c = in + j * (d + 1);
    copy_lds(lds, c, d + 1);
    __syncthreads();
    for (int64_t q = threadIdx.x; q <= n; q += kT) {
        uint64_t lo = 0, hi = 0;
        for (int t = 0; t < d; ++t) {
            const uint64_t at = lds[t];
            const uint64_t* kp = ksk + (int64_t)t * kKsDigits * (n + 1) + q;
#pragma unroll
            for (int k = 0; k < kKsDigits; ++k) mac128((at >> (4 * k)) & 15, kp[k * (n + 1)], &lo, &hi);
        }
        out[(oi ? (int64_t)oi[j] : j) * (n + 1) + q] = subp(q == n ? lds[d] : 0, red126(lo, hi));
    }
}

// Row moves of the FFT executor (rows of w words): dst[di ? di[j] : j] =
// src[si ? si[j] : j], and NOT rows dst[di[j]] = (0, .., 0, 2 floor(p/8)) -
// src[si[j]]; slots 0 and 1 set to the trivial encryptions of 0 and 1.
__global__ __launch_bounds__(kT) void k_ring_rows(const uint64_t* __restrict__ src, const int32_t* __restrict__ si,
                                                  uint64_t* __restrict__ dst, const int32_t* __restrict__ di,
                                                  int64_t count, int64_t w, int negate)
{
    const int64_t total = count * w, stride = (int64_t)gridDim.x * kT;
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < total; e += stride) {
        const int64_t j = e / w, q = e % w;
        const uint64_t v = src[(si ? (int64_t)si[j] : j) * w + q];
        dst[(di ? (int64_t)di[j] : j) * w + q] = negate ? subp(q == w - 1 ? 2 * (kP / 8) : 0, v) : v;
    }
}
__global__ __launch_bounds__(kT) void k_ring_consts(uint64_t* __restrict__ slots, int64_t w)
{
    for (int64_t q = threadIdx.x; q < 2 * w; q += kT) slots[q] = q == 2 * w - 1 ? 2 * (kP / 8) : 0;
}

// NOT (3): G - X;  XADD (7): X + Y.  Elementwise over n ciphertexts.
__global__ __launch_bounds__(kT) void k_ring_linear(const uint64_t* __restrict__ X, const uint64_t* __restrict__ Y,
                                                    uint64_t* __restrict__ out, int64_t count, int d, int logd,
                                                    int op)
{
    const int64_t stride = (int64_t)gridDim.x * kT;
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < count; e += stride) {
        if (op == 3) {
            const int t = (int)(e & (d - 1));
            const int64_t rc = e >> logd;                 // (ct*rows + row)*2 + col
            const int col = (int)(rc & 1), row = (int)((rc >> 1) % kRows);
            out[e] = subp(gadget(row, col, t), X[e]);
        } else {
            out[e] = addp(X[e], Y[e]);
        }
    }
}

// Encryption of bits[c] under secret s (signed coefficients): row r of
// ciphertext c is (a_r*s + e_r, a_r) + bits[c]*G[r].
template <int LOGD>
__global__ __launch_bounds__(kT) void k_ring_encrypt(const int64_t* __restrict__ s, const uint64_t* __restrict__ A,
                                                     const int64_t* __restrict__ E, const uint8_t* __restrict__ bits,
                                                     uint64_t* __restrict__ out, TwView tw)
{
    constexpr int D = 1 << LOGD;
    extern __shared__ uint64_t lds[];
    Tw* t_w = reinterpret_cast<Tw*>(lds);
    uint64_t* buf = lds + 2 * D;  // a_r, then s
    const int64_t cr = blockIdx.x;   // c*rows + r
    const int64_t c = cr / kRows;
    const int r = (int)(cr % kRows);
    const uint64_t* a = A + cr * D;
    copy_lds(lds, reinterpret_cast<const uint64_t*>(tw.fwd), 2 * D);
    for (int t = threadIdx.x; t < D; t += kT) {
        buf[t] = a[t];
        buf[D + t] = from_signed(s[t]);
    }
    __syncthreads();
    fwd_lds<LOGD, 2>(buf, t_w, false);
    for (int t = threadIdx.x; t < D; t += kT) buf[t] = mulp(buf[t], buf[D + t]);
    copy_lds(lds, reinterpret_cast<const uint64_t*>(tw.inv), 2 * D);
    __syncthreads();
    inv_lds<LOGD, 1>(buf, t_w);
    const uint64_t m = bits[c] & 1;
    const int64_t* e = E + cr * D;
    uint64_t* o = out + cr * 2 * D;
    for (int t = threadIdx.x; t < D; t += kT) {
        const uint64_t g0 = m ? gadget(r, 0, t) : 0, g1 = m ? gadget(r, 1, t) : 0;
        o[t] = addp(addp(mulw(buf[t], tw.dinv), from_signed(e[t])), g0);
        o[D + t] = addp(a[t], g1);
    }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

int log2_exact(int d)
{
    if (d < 1 || d > (1 << kMaxLogD) || (d & (d - 1))) return -1;
    int l = 0;
    while ((1 << l) < d) ++l;
    return l;
}

int brv(int x, int bits)
{
    int r = 0;
    for (int i = 0; i < bits; ++i) r = (r << 1) | ((x >> i) & 1);
    return r;
}

// A primitive 2d-th root of unity: g^((p-1)/(2d)) for a generator g of Z_p^*
// (p - 1 = 2^16 * 3 * 47 * 178481 * 2796203).
uint64_t root_2d(int d)
{
    static const uint64_t f[] = {2, 3, 47, 178481, 2796203};
    for (uint64_t g = 2;; ++g) {
        bool gen = true;
        for (uint64_t q : f)
            if (powp(g, (kP - 1) / q) == 1) {
                gen = false;
                break;
            }
        if (gen) return powp(g, (kP - 1) / (2 * (uint64_t)d));
    }
}

Tw shoup(uint64_t w) { return Tw{w, (uint64_t)(((unsigned __int128)w << 64) / kP)}; }

std::mutex g_tw_mu;
std::map<std::pair<int, int>, Tw*> g_tw;  // (device, d) -> tables

int tables(int d, int logd, TwView* tv)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return sfft_hip_fail(e, "hipGetDevice");
    std::lock_guard<std::mutex> lk(g_tw_mu);
    auto it = g_tw.find({dev, d});
    Tw* p = nullptr;
    if (it != g_tw.end()) {
        p = it->second;
    } else {
        std::vector<Tw> h(2 * (size_t)d);
        const uint64_t psi = root_2d(d), ipsi = powp(psi, kP - 2);
        for (int k = 0; k < d; ++k) {
            h[k] = shoup(powp(psi, (uint64_t)brv(k, logd)));
            h[d + k] = shoup(powp(ipsi, (uint64_t)brv(k, logd)));
        }
        e = hipMalloc(&p, h.size() * sizeof(Tw));
        if (e != hipSuccess) return sfft_hip_fail(e, "ring tables");
        e = hipMemcpy(p, h.data(), h.size() * sizeof(Tw), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(p);
            return sfft_hip_fail(e, "ring tables");
        }
        g_tw[{dev, d}] = p;
    }
    tv->fwd = p;
    tv->inv = p + d;
    tv->dinv = shoup(powp((uint64_t)d, kP - 2));
    return SFFT_OK;
}

// Lets a kernel take up to 160 KB of LDS.
template <typename K>
hipError_t allow_lds(K kernel)
{
    return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
}

template <int LOGD>
hipError_t launch_gate(const uint64_t* L, const uint64_t* R, uint64_t* Rn, uint64_t* out, int64_t n, TwView tv, int op,
                       hipStream_t s)
{
    constexpr int D = 1 << LOGD;
    // once per instantiation (thread-safe static initialisation)
    static const hipError_t attr = [] {
        hipError_t e = allow_lds(k_ring_fwd<LOGD>);
        return e == hipSuccess ? allow_lds(k_ring_product<LOGD>) : e;
    }();
    hipError_t e = attr;
    if (e != hipSuccess) return e;
    const int64_t nb = n * kRows;
    hipLaunchKernelGGL(k_ring_fwd<LOGD>, dim3((unsigned)nb), dim3(kT), (size_t)4 * D * 8, s, R, Rn, tv);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ring_product<LOGD>, dim3((unsigned)nb), dim3(kT), ProdShape<LOGD>::lds, s, L, R, Rn, out, nb,
                       tv, op);
    return hipGetLastError();
}

template <int LOGD>
hipError_t launch_bk_prepare(const uint64_t* bk, int64_t n, uint64_t* bkt, TwView tv, hipStream_t s)
{
    constexpr int D = 1 << LOGD;
    static const hipError_t attr = allow_lds(k_ring_fwd<LOGD>);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(k_ring_fwd<LOGD>, dim3((unsigned)(n * kRows)), dim3(kT), (size_t)4 * D * 8, s, bk, bkt, tv);
    return hipGetLastError();
}

template <int LOGD>
hipError_t launch_blind_rotate(const uint64_t* bkt, int64_t n, const int32_t* rot, uint64_t* acc, int64_t m, TwView tv,
                               hipStream_t s)
{
    constexpr int D = 1 << LOGD;
    static const hipError_t attr = allow_lds(k_ring_blind_rotate<LOGD>);
    if (attr != hipSuccess) return attr;
    const size_t lds = (size_t)(2 * D) * 8 + (size_t)ProdShape<LOGD>::NB * D * 8;
    hipLaunchKernelGGL(k_ring_blind_rotate<LOGD>, dim3((unsigned)m), dim3(kT), lds, s, bkt, n, rot, acc, tv);
    return hipGetLastError();
}

// The combination (cx, cy, cb) of x and y, switched, blind-rotated and
// extracted with accumulator value delta.
struct Combine {
    const uint64_t* x;
    const uint64_t* y;
    int cx, cy;
    uint64_t cb, delta;
    const int32_t* xi = nullptr;  // row indices into x / y (null: row j)
    const int32_t* yi = nullptr;
    const int32_t* gk = nullptr;  // per-row gate codes (null: cx, cy, cb for every row)
};

template <int LOGD>
hipError_t launch_bootstrap(const uint64_t* bkt, int64_t n, const Combine& cm, int64_t m, uint64_t* out, uint64_t* acc,
                            int32_t* rot, TwView tv, hipStream_t s)
{
    hipLaunchKernelGGL(k_ring_br_init<LOGD>, dim3((unsigned)m), dim3(kT), 0, s, cm.x, cm.y, cm.xi, cm.yi, cm.gk, cm.cx,
                       cm.cy, cm.cb, n, rot, acc, cm.delta);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (n > 0 && (e = launch_blind_rotate<LOGD>(bkt, n, rot, acc, m, tv, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ring_extract<LOGD>, dim3((unsigned)m), dim3(kT), 0, s, acc, out, cm.delta);
    return hipGetLastError();
}

template <int LOGD>
hipError_t launch_encrypt(const int64_t* sd, const uint64_t* a, const int64_t* ed, const uint8_t* bits, int64_t n,
                          uint64_t* ct, TwView tv, hipStream_t s)
{
    constexpr int D = 1 << LOGD;
    static const hipError_t attr = allow_lds(k_ring_encrypt<LOGD>);
    hipError_t e = attr;
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ring_encrypt<LOGD>, dim3((unsigned)(n * kRows)), dim3(kT), (size_t)4 * D * 8, s, sd, a, ed,
                       bits, ct, tv);
    return hipGetLastError();
}

// Calls F<LOGD>::run(args...) for the run-time logd (0..kMaxLogD).
#define SFFT_RING_DISPATCH(logd, CALL)                                                                            \
    switch (logd) {                                                                                               \
    case 0: CALL(0); case 1: CALL(1); case 2: CALL(2); case 3: CALL(3); case 4: CALL(4); case 5: CALL(5);        \
    case 6: CALL(6); case 7: CALL(7); case 8: CALL(8); case 9: CALL(9); case 10: CALL(10); default: CALL(11);    \
    }

int check_d(int32_t d, int* logd)
{
    *logd = log2_exact(d);
    if (*logd < 0) return sfft_fail(SFFT_EINVAL, "d must be a power of two in [1, 2048]");
    return SFFT_OK;
}

int64_t ct_words_of(int d) { return (int64_t)kRows * 2 * d; }

// Blocks of one launch: grids are split below 2^31 workgroups.
constexpr int64_t kMaxGrid = 1 << 30;

// ---- FFT plans on bootstrapped gates ---------------------------------------
// Every node of the (shared) FFT netlist gets a slot of n+1 words: slot v
// holds node v's LWE ciphertext.  Binary nodes are levelised (a NOT takes
// its operand's level) and each level's binary nodes, of whatever kinds,
// form one batched bootstrapped gate (every row carries its gate code):
// operands gathered from the slots by index, outputs key-switched straight
// into theirs.  NOTs run after their level's gates, in
// rank order (a NOT of a NOT of the same level one rank later).
struct RingStep {
    bool is_not;
    int count;
    int64_t x, y, o, g;  // offsets of the index arrays and gate codes (NOT: x = sources, o = destinations)
};
struct RingPlanHost {
    int d = 0, logd = 0;
    int64_t n = 0, nodes = 0, gates = 0, n_in = 0, n_out = 0, max_batch = 0;
    int32_t levels = 0, calls = 0;
    int64_t in_off = 0, out_off = 0;
    std::vector<int32_t> idx;
    std::vector<RingStep> steps;
    int64_t ws_bytes() const
    {
        const int64_t slots = nodes * (n + 1) * 8, scratch = max_batch * (2 * d * 8 + (d + 1) * 8 + n * 4);
        return ((slots + 255) & ~(int64_t)255) + scratch;
    }
};

int ring_plan_build(const sfft_shape* shape, int32_t d, int64_t n, RingPlanHost* pl)
{
    std::string why;
    if (!sfft_shape_check(shape, &why)) return sfft_fail(SFFT_EINVAL, why);
    int logd, rc;
    if ((rc = check_d(d, &logd)) != SFFT_OK) return rc;
    if (n < 1) return sfft_fail(SFFT_EINVAL, "n must be >= 1");
    const sfft::Compact c = sfft::share(sfft::compact(sfft::build_fft_netlist(sfft_shape_of(shape))));
    const int64_t N = (int64_t)c.size();
    std::vector<int32_t> depth(N, 0), rank(N, 0);
    int32_t L = 0;
    for (int64_t v = 0; v < N; ++v) {
        const int8_t t = c.t[v];
        if (t == sfft::T_NOT) {
            depth[v] = depth[c.a[v]];
            rank[v] = c.t[c.a[v]] == sfft::T_NOT && depth[c.a[v]] == depth[v] ? rank[c.a[v]] + 1 : 0;
        } else if (t >= sfft::T_AND) {
            depth[v] = std::max(depth[c.a[v]], depth[c.b[v]]) + 1;
        }
        L = std::max(L, depth[v]);
    }
    pl->d = d, pl->logd = logd, pl->n = n, pl->nodes = N, pl->levels = L;
    pl->n_in = c.n_inputs, pl->n_out = (int64_t)c.outputs.size();
    auto push = [&](const std::vector<int32_t>& v) {
        const int64_t off = (int64_t)pl->idx.size();
        pl->idx.insert(pl->idx.end(), v.begin(), v.end());
        return off;
    };
    std::vector<int32_t> ins(c.n_inputs, 0);
    for (int64_t v = 0; v < N; ++v)
        if (c.t[v] == sfft::T_IN) ins[c.a[v]] = (int32_t)v;
    pl->in_off = push(ins);
    pl->out_off = push(std::vector<int32_t>(c.outputs.begin(), c.outputs.end()));
    for (int32_t lev = 0; lev <= L; ++lev) {
        if (lev > 0) {
            // every binary node of the level in one call, each with its gate
            std::vector<int32_t> xs, ys, os, gs;
            for (int64_t v = 0; v < N; ++v) {
                const int8_t t = c.t[v];
                if (depth[v] != lev || t < sfft::T_AND) continue;
                xs.push_back(c.a[v]);
                ys.push_back(c.b[v]);
                os.push_back((int32_t)v);
                gs.push_back(t == sfft::T_XADD ? sfft::T_XOR : t);   // the gate codes are the node types
            }
            if (!xs.empty()) {
                RingStep st{false, (int)xs.size(), push(xs), push(ys), push(os), push(gs)};
                pl->steps.push_back(st);
                pl->gates += (int64_t)xs.size();
                pl->max_batch = std::max(pl->max_batch, (int64_t)xs.size());
                ++pl->calls;
            }
        }
        for (int r = 0;; ++r) {
            std::vector<int32_t> src, dst;
            for (int64_t v = 0; v < N; ++v)
                if (c.t[v] == sfft::T_NOT && depth[v] == lev && rank[v] == r) {
                    src.push_back(c.a[v]);
                    dst.push_back((int32_t)v);
                }
            if (src.empty()) break;
            pl->steps.push_back(RingStep{true, (int)src.size(), push(src), 0, push(dst), 0});
        }
    }
    return SFFT_OK;
}

}  // namespace

struct sfft_ring_plan {
    RingPlanHost h;
    int32_t* dev = nullptr;  // the index arrays
};

extern "C" {

int sfft_ring_plan_analyze(const sfft_shape* shape, int32_t d, int64_t n, sfft_ring_plan_info* info)
{
    if (!info) return sfft_fail(SFFT_EINVAL, "null info");
    RingPlanHost h;
    int rc;
    try {
        if ((rc = ring_plan_build(shape, d, n, &h)) != SFFT_OK) return rc;
    } catch (const std::bad_alloc&) {
        return sfft_fail(SFFT_ENOMEM, "host allocation failed");
    }
    info->nodes = h.nodes, info->gates = h.gates, info->levels = h.levels, info->calls = h.calls;
    info->max_batch = h.max_batch, info->n_inputs = h.n_in, info->n_outputs = h.n_out, info->ws_bytes = h.ws_bytes();
    return SFFT_OK;
}

int sfft_ring_plan_create(const sfft_shape* shape, int32_t d, int64_t n, sfft_ring_plan** out)
{
    if (!out) return sfft_fail(SFFT_EINVAL, "null output");
    *out = nullptr;
    sfft_ring_plan* pl = nullptr;
    try {
        pl = new sfft_ring_plan();
        int rc = ring_plan_build(shape, d, n, &pl->h);
        if (rc != SFFT_OK) {
            delete pl;
            return rc;
        }
    } catch (const std::bad_alloc&) {
        delete pl;
        return sfft_fail(SFFT_ENOMEM, "host allocation failed");
    }
    const size_t bytes = pl->h.idx.size() * sizeof(int32_t);
    hipError_t e = hipMalloc(&pl->dev, bytes ? bytes : 4);
    if (e == hipSuccess && bytes) e = hipMemcpy(pl->dev, pl->h.idx.data(), bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (pl->dev) (void)hipFree(pl->dev);
        delete pl;
        return sfft_hip_fail(e, "sfft_ring_plan_create");
    }
    *out = pl;
    return SFFT_OK;
}

void sfft_ring_plan_destroy(sfft_ring_plan* plan)
{
    if (!plan) return;
    if (plan->dev) (void)hipFree(plan->dev);
    delete plan;
}

int sfft_ring_fft_execute(const sfft_ring_plan* plan, const uint64_t* bkt_dev, const uint64_t* ksk_dev,
                          const uint64_t* in_dev, uint64_t* out_dev, void* ws_dev, int64_t ws_bytes, void* hip_stream)
{
    if (!plan || !bkt_dev || !ksk_dev || !in_dev || !out_dev || !ws_dev) return sfft_fail(SFFT_EINVAL, "null argument");
    const RingPlanHost& h = plan->h;
    if (ws_bytes < h.ws_bytes()) return sfft_fail(SFFT_EINVAL, "workspace too small");
    TwView tv;
    int rc;
    if ((rc = tables(h.d, h.logd, &tv)) != SFFT_OK) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t w = h.n + 1;
    uint64_t* slots = (uint64_t*)ws_dev;
    uint8_t* scratch = (uint8_t*)ws_dev + ((h.nodes * w * 8 + 255) & ~(int64_t)255);
    uint64_t* acc = (uint64_t*)scratch;
    uint64_t* mid = acc + h.max_batch * 2 * h.d;
    int32_t* rot = (int32_t*)(mid + h.max_batch * (h.d + 1));
    const int32_t* I = plan->dev;
    auto rows = [&](const uint64_t* src, const int32_t* si, uint64_t* dst, const int32_t* di, int64_t count, int neg) {
        const int64_t blocks = std::min<int64_t>((count * w + kT - 1) / kT, 1 << 16);
        hipLaunchKernelGGL(k_ring_rows, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(kT), 0, s, src, si, dst, di,
                           count, w, neg);
        return hipGetLastError();
    };
    hipLaunchKernelGGL(k_ring_consts, dim3(1), dim3(kT), 0, s, slots, w);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess && h.n_in > 0) e = rows(in_dev, nullptr, slots, I + h.in_off, h.n_in, 0);
    const uint64_t q8 = kP / 8;
    for (const RingStep& st : h.steps) {
        if (e != hipSuccess) break;
        if (st.is_not) {
            e = rows(slots, I + st.x, slots, I + st.o, st.count, 1);
            continue;
        }
        Combine cm{slots, slots, 0, 0, 0, q8, I + st.x, I + st.y, I + st.g};
#define SFFT_PBS(L) { e = launch_bootstrap<L>(bkt_dev, h.n, cm, st.count, mid, acc, rot, tv, s); break; }
        SFFT_RING_DISPATCH(h.logd, SFFT_PBS)
#undef SFFT_PBS
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(k_ring_keyswitch, dim3((unsigned)st.count), dim3(kT), (size_t)(h.d + 1) * 8, s, ksk_dev, mid,
                           slots, I + st.o, h.d, h.n);
        e = hipGetLastError();
    }
    if (e == hipSuccess && h.n_out > 0) e = rows(slots, I + h.out_off, out_dev, nullptr, h.n_out, 0);
    return e == hipSuccess ? SFFT_OK : sfft_hip_fail(e, "sfft_ring_fft_execute");
}


int64_t sfft_ring_ct_words(int32_t d)
{
    int logd;
    if (check_d(d, &logd) != SFFT_OK) return SFFT_EINVAL;
    return ct_words_of(d);
}

int sfft_ring_workspace_bytes(int32_t d, int64_t n, int64_t* bytes)
{
    int logd;
    if (check_d(d, &logd) != SFFT_OK) return SFFT_EINVAL;
    if (n < 0 || !bytes) return sfft_fail(SFFT_EINVAL, "n < 0 or null output");
    *bytes = n * ct_words_of(d) * 8;
    return SFFT_OK;
}

int sfft_ring_encrypt(int32_t d, const int64_t* s_dev, const uint64_t* a_dev, const int64_t* e_dev,
                      const uint8_t* bits_dev, int64_t n, uint64_t* ct_dev, void* hip_stream)
{
    int logd, rc;
    if ((rc = check_d(d, &logd)) != SFFT_OK) return rc;
    if (n < 0) return sfft_fail(SFFT_EINVAL, "n < 0");
    if (n == 0) return SFFT_OK;
    if (!s_dev || !a_dev || !e_dev || !bits_dev || !ct_dev) return sfft_fail(SFFT_EINVAL, "null buffer");
    if (n * kRows > kMaxGrid) return sfft_fail(SFFT_EINVAL, "too many ciphertexts for one call");
    TwView tv;
    if ((rc = tables(d, logd, &tv)) != SFFT_OK) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipSuccess;
#define SFFT_ENC(L) { e = launch_encrypt<L>(s_dev, a_dev, e_dev, bits_dev, n, ct_dev, tv, s); break; }
    SFFT_RING_DISPATCH(logd, SFFT_ENC)
#undef SFFT_ENC
    return e == hipSuccess ? SFFT_OK : sfft_hip_fail(e, "k_ring_encrypt");
}

int sfft_ring_gate(int32_t d, int32_t gate, const uint64_t* x_dev, const uint64_t* y_dev, uint64_t* out_dev,
                   int64_t n, void* ws_dev, int64_t ws_bytes, void* hip_stream)
{
    int logd, rc;
    if ((rc = check_d(d, &logd)) != SFFT_OK) return rc;
    if (gate < 3 || gate > 9) return sfft_fail(SFFT_EINVAL, "gate must be 3..9");
    if (n < 0) return sfft_fail(SFFT_EINVAL, "n < 0");
    if (n == 0) return SFFT_OK;
    const bool linear = gate == 3 || gate == 7;
    if (!x_dev || !out_dev || (gate != 3 && !y_dev)) return sfft_fail(SFFT_EINVAL, "null buffer");
    if (out_dev == x_dev || out_dev == y_dev) return sfft_fail(SFFT_EINVAL, "out must not alias an operand");
    if (n * kRows > kMaxGrid) return sfft_fail(SFFT_EINVAL, "too many ciphertexts for one call");
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e;
    const int64_t words = n * ct_words_of(d);
    if (linear) {
        const int64_t blocks = std::min<int64_t>((words + kT - 1) / kT, 1 << 20);
        hipLaunchKernelGGL(k_ring_linear, dim3((unsigned)blocks), dim3(kT), 0, s, x_dev, y_dev, out_dev, words, d,
                           logd, gate);
        e = hipGetLastError();
        return e == hipSuccess ? SFFT_OK : sfft_hip_fail(e, "k_ring_linear");
    }
    if (!ws_dev || ws_bytes < words * 8) return sfft_fail(SFFT_EINVAL, "workspace missing or too small");
    TwView tv;
    if ((rc = tables(d, logd, &tv)) != SFFT_OK) return rc;
    uint64_t* rn = (uint64_t*)ws_dev;
#define SFFT_GATE(L) { e = launch_gate<L>(x_dev, y_dev, rn, out_dev, n, tv, gate, s); break; }
    SFFT_RING_DISPATCH(logd, SFFT_GATE)
#undef SFFT_GATE
    return e == hipSuccess ? SFFT_OK : sfft_hip_fail(e, "k_ring_product");
}

int sfft_ring_bk_prepare(int32_t d, const uint64_t* bk_dev, int64_t n, uint64_t* bkt_dev, void* hip_stream)
{
    int logd, rc;
    if ((rc = check_d(d, &logd)) != SFFT_OK) return rc;
    if (n < 0) return sfft_fail(SFFT_EINVAL, "n < 0");
    if (n == 0) return SFFT_OK;
    if (!bk_dev || !bkt_dev) return sfft_fail(SFFT_EINVAL, "null buffer");
    if (bkt_dev == bk_dev) return sfft_fail(SFFT_EINVAL, "bkt must not alias bk");
    if (n * kRows > kMaxGrid) return sfft_fail(SFFT_EINVAL, "too many key ciphertexts for one call");
    TwView tv;
    if ((rc = tables(d, logd, &tv)) != SFFT_OK) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipSuccess;
#define SFFT_BKP(L) { e = launch_bk_prepare<L>(bk_dev, n, bkt_dev, tv, s); break; }
    SFFT_RING_DISPATCH(logd, SFFT_BKP)
#undef SFFT_BKP
    return e == hipSuccess ? SFFT_OK : sfft_hip_fail(e, "k_ring_fwd");
}

int sfft_ring_blind_rotate(int32_t d, const uint64_t* bkt_dev, int64_t n, const int32_t* rot_dev, uint64_t* acc_dev,
                           int64_t m, void* hip_stream)
{
    int logd, rc;
    if ((rc = check_d(d, &logd)) != SFFT_OK) return rc;
    if (n < 0 || m < 0) return sfft_fail(SFFT_EINVAL, "n < 0 or m < 0");
    if (n == 0 || m == 0) return SFFT_OK;
    if (!bkt_dev || !rot_dev || !acc_dev) return sfft_fail(SFFT_EINVAL, "null buffer");
    if (m > kMaxGrid) return sfft_fail(SFFT_EINVAL, "too many accumulators for one call");
    TwView tv;
    if ((rc = tables(d, logd, &tv)) != SFFT_OK) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipSuccess;
#define SFFT_BR(L) { e = launch_blind_rotate<L>(bkt_dev, n, rot_dev, acc_dev, m, tv, s); break; }
    SFFT_RING_DISPATCH(logd, SFFT_BR)
#undef SFFT_BR
    return e == hipSuccess ? SFFT_OK : sfft_hip_fail(e, "k_ring_blind_rotate");
}

int sfft_ring_bootstrap_workspace_bytes(int32_t d, int64_t n, int64_t m, int64_t* bytes)
{
    int logd, rc;
    if ((rc = check_d(d, &logd)) != SFFT_OK) return rc;
    if (n < 0 || m < 0 || !bytes) return sfft_fail(SFFT_EINVAL, "n < 0, m < 0 or null output");
    *bytes = m * 2 * d * 8 + m * n * 4;
    return SFFT_OK;
}

int sfft_ring_bootstrap(int32_t d, const uint64_t* bkt_dev, int64_t n, const uint64_t* lwe_dev, int64_t m,
                        uint64_t* out_dev, void* ws_dev, int64_t ws_bytes, void* hip_stream)
{
    int logd, rc;
    if ((rc = check_d(d, &logd)) != SFFT_OK) return rc;
    if (n < 0 || m < 0) return sfft_fail(SFFT_EINVAL, "n < 0 or m < 0");
    if (m == 0) return SFFT_OK;
    if (!lwe_dev || !out_dev || !ws_dev || (n > 0 && !bkt_dev)) return sfft_fail(SFFT_EINVAL, "null buffer");
    if (m > kMaxGrid) return sfft_fail(SFFT_EINVAL, "too many ciphertexts for one call");
    if (ws_bytes < m * 2 * d * 8 + m * n * 4) return sfft_fail(SFFT_EINVAL, "workspace too small");
    TwView tv;
    if ((rc = tables(d, logd, &tv)) != SFFT_OK) return rc;
    uint64_t* acc = (uint64_t*)ws_dev;
    int32_t* rot = (int32_t*)(acc + m * 2 * d);
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipSuccess;
    const Combine cm{lwe_dev, nullptr, 1, 0, 0, kP / 4};
#define SFFT_BS(L) { e = launch_bootstrap<L>(bkt_dev, n, cm, m, out_dev, acc, rot, tv, s); break; }
    SFFT_RING_DISPATCH(logd, SFFT_BS)
#undef SFFT_BS
    return e == hipSuccess ? SFFT_OK : sfft_hip_fail(e, "ring bootstrap");
}

int sfft_ring_keyswitch(int32_t d, int64_t n, const uint64_t* ksk_dev, const uint64_t* in_dev, int64_t m,
                        uint64_t* out_dev, void* hip_stream)
{
    int logd, rc;
    if ((rc = check_d(d, &logd)) != SFFT_OK) return rc;
    if (n < 0 || m < 0) return sfft_fail(SFFT_EINVAL, "n < 0 or m < 0");
    if (m == 0) return SFFT_OK;
    if (!ksk_dev || !in_dev || !out_dev) return sfft_fail(SFFT_EINVAL, "null buffer");
    if (m > kMaxGrid) return sfft_fail(SFFT_EINVAL, "too many ciphertexts for one call");
    hipStream_t s = (hipStream_t)hip_stream;
    hipLaunchKernelGGL(k_ring_keyswitch, dim3((unsigned)m), dim3(kT), (size_t)(d + 1) * 8, s, ksk_dev, in_dev, out_dev,
                       (const int32_t*)nullptr, (int)d, n);
    hipError_t e = hipGetLastError();
    return e == hipSuccess ? SFFT_OK : sfft_hip_fail(e, "k_ring_keyswitch");
}

int sfft_ring_gate_bootstrap_workspace_bytes(int32_t d, int64_t n, int64_t m, int64_t* bytes)
{
    int logd, rc;
    if ((rc = check_d(d, &logd)) != SFFT_OK) return rc;
    if (n < 0 || m < 0 || !bytes) return sfft_fail(SFFT_EINVAL, "n < 0, m < 0 or null output");
    *bytes = m * 2 * d * 8 + m * (d + 1) * 8 + m * n * 4;
    return SFFT_OK;
}

int sfft_ring_gate_bootstrap(int32_t d, int32_t gate, const uint64_t* bkt_dev, int64_t n, const uint64_t* ksk_dev,
                             const uint64_t* x_dev, const uint64_t* y_dev, int64_t m, uint64_t* out_dev, void* ws_dev,
                             int64_t ws_bytes, void* hip_stream)
{
    int logd, rc;
    if ((rc = check_d(d, &logd)) != SFFT_OK) return rc;
    if (gate != 4 && gate != 5 && gate != 6 && gate != 8)
        return sfft_fail(SFFT_EINVAL, "gate must be 4 (AND), 5 (XOR), 6 (OR) or 8 (NAND)");
    int cx, cy;
    uint64_t cb;
    gate_combination(gate, &cx, &cy, &cb);
    if (n < 0 || m < 0) return sfft_fail(SFFT_EINVAL, "n < 0 or m < 0");
    if (m == 0) return SFFT_OK;
    if (!x_dev || !y_dev || !out_dev || !ksk_dev || !ws_dev || (n > 0 && !bkt_dev))
        return sfft_fail(SFFT_EINVAL, "null buffer");
    if (m > kMaxGrid) return sfft_fail(SFFT_EINVAL, "too many ciphertexts for one call");
    if (ws_bytes < m * 2 * d * 8 + m * (d + 1) * 8 + m * n * 4) return sfft_fail(SFFT_EINVAL, "workspace too small");
    TwView tv;
    if ((rc = tables(d, logd, &tv)) != SFFT_OK) return rc;
    const Combine cm{x_dev, y_dev, cx, cy, cb, kP / 8};
    uint64_t* acc = (uint64_t*)ws_dev;
    uint64_t* mid = acc + m * 2 * d;
    int32_t* rot = (int32_t*)(mid + m * (d + 1));
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e = hipSuccess;
#define SFFT_GBS(L) { e = launch_bootstrap<L>(bkt_dev, n, cm, m, mid, acc, rot, tv, s); break; }
    SFFT_RING_DISPATCH(logd, SFFT_GBS)
#undef SFFT_GBS
    if (e != hipSuccess) return sfft_hip_fail(e, "ring gate bootstrap");
    return sfft_ring_keyswitch(d, n, ksk_dev, mid, m, out_dev, hip_stream);
}

int sfft_ring_decrypt(int32_t d, const int64_t* s_host, const uint64_t* ct, int64_t n, int ct_on_device,
                      uint8_t* bits_out)
{
    int logd, rc;
    if ((rc = check_d(d, &logd)) != SFFT_OK) return rc;
    if (n < 0) return sfft_fail(SFFT_EINVAL, "n < 0");
    if (n == 0) return SFFT_OK;
    if (!s_host || !ct || !bits_out) return sfft_fail(SFFT_EINVAL, "null buffer");
    std::vector<uint64_t> row(2 * (size_t)d);
    const int r = kEll - 1;  // gadget 2^(ell-1) on column 0
    for (int64_t c = 0; c < n; ++c) {
        const uint64_t* src = ct + (c * kRows + r) * 2 * d;
        if (ct_on_device) {
            hipError_t e = hipMemcpy(row.data(), src, row.size() * 8, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return sfft_hip_fail(e, "sfft_ring_decrypt");
        } else {
            std::memcpy(row.data(), src, row.size() * 8);
        }
        // coefficient 0 of c0 - c1*s:  (c1*s)_0 = c1_0 s_0 - sum_{t>0} c1_t s_(d-t)
        uint64_t cs = mulp(row[d], from_signed(s_host[0]));
        for (int t = 1; t < d; ++t) cs = subp(cs, mulp(row[d + t], from_signed(s_host[d - t])));
        const uint64_t x = subp(row[0], cs);
        const uint64_t mag = x <= kP / 2 ? x : kP - x;
        bits_out[c] = mag > kP / 4;
    }
    return SFFT_OK;
}

}  // extern "C"
