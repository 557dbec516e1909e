// gfx950 kernels for GSW13 ciphertext arithmetic over q = 2^k.
//
// The gate product (paper, section "Time/Space Complexities": a NAND is a
// matrix-matrix product, cubic in the ciphertext dimension) is
//     P = BitDecomp(L) * R  mod 2^k,
// an Nct x Nct bit matrix times an Nct x (n+1) matrix of k-bit integers.  Row
// r of P is the sum of the rows j of R selected by the bits of row r of L.
//
// Method: four bits of a row of L select one of the 16 subset sums of four
// consecutive rows of R (the method of Arlazarov, Dinic, Kronrod and Faradzev,
// 1970).  A workgroup builds those subset-sum tables for 32 consecutive rows
// of R in LDS (8 tables x 16 entries, carried mod 2^k per element), then every
// lane adds one table entry per 4 bits of its L rows into 32-bit limb
// accumulators with separate carry counters.  Integer VALU only: per table
// word one LDS read, one add with carry-out and one add of the carry.
//
// Epilogue (fused): the limb sums and carry counters of each (row, element)
// are resolved into P mod 2^k and combined, still limb by limb, into up to
// four outputs a L + b R + c P + g G + e E (AND, XOR, OR, NOT, XADD forms).
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace sfft {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kGroups = 8;  // 4-bit groups per 32-row chunk of R

__device__ __forceinline__ uint32_t* ctp(const Bufs& b, int32_t ref)
{
    const uint32_t u = (uint32_t)ref;
    const uint32_t buf = u >> 29;
    const uint64_t idx = u & 0x1FFFFFFFu;
    uint32_t* base = buf == B_IN ? b.in : buf == B_OUT ? b.out : buf == B_WS ? b.ws : b.aux;
    return base + idx * (uint64_t)b.ct_words;
}

__device__ __forceinline__ uint64_t sm_mix(uint64_t z)
{
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

struct MuBits {
    uint32_t w[kMaxEncPerLaunch / 32];
};

// Output row `row`, element e: resolve P from limb sums (acc, cnt pairs in
// `sums`) and write every output of the item.
__device__ void epilogue_element(const Bufs& bufs, const Geo& g, const ProdItem& it, const uint32_t* sums,
                                 const uint32_t* Lp, const uint32_t* Rp, int row, int e, uint64_t dst_shift)
{
    const int br = row / g.k, tr = row % g.k;
    const size_t rowoff = (size_t)row * g.W;
    uint64_t cp = 0;
    int64_t carry[kMaxOut];
    uint32_t* dst[kMaxOut];
    const uint32_t* Ep[kMaxOut];
#pragma unroll
    for (int o = 0; o < kMaxOut; o++) {
        carry[o] = 0;
        dst[o] = o < it.nout ? ctp(bufs, it.dst[o]) + dst_shift : nullptr;
        Ep[o] = (o < it.nout && it.E[o] >= 0) ? ctp(bufs, it.E[o]) : nullptr;
    }
    bool needL = false, needR = false;
    for (int o = 0; o < it.nout; o++) {
        needL |= it.cL[o] != 0;
        needR |= it.cR[o] != 0;
    }
    for (int l = 0; l < g.kw; l++) {
        const int w = e * g.kw + l;
        const uint64_t t = (uint64_t)sums[2 * w] + cp;
        const uint32_t P = (uint32_t)t;
        cp = (t >> 32) + sums[2 * w + 1];
        const uint32_t Gv = (e == br && l == (tr >> 5)) ? (1u << (tr & 31)) : 0u;
        const size_t off = rowoff + w;
        const uint32_t Lv = needL ? Lp[off] : 0u;
        const uint32_t Rv = needR ? Rp[off] : 0u;
#pragma unroll
        for (int o = 0; o < kMaxOut; o++) {
            if (o >= it.nout) break;
            int64_t s = carry[o] + (int64_t)it.cL[o] * Lv + (int64_t)it.cR[o] * Rv + (int64_t)it.cP[o] * P +
                        (int64_t)it.cG[o] * Gv;
            if (Ep[o]) s += (int64_t)it.cE[o] * Ep[o][off];
            dst[o][off] = (uint32_t)s;
            carry[o] = s >> 32;
        }
    }
}

template <int WPL, int RPLMAX, bool ENC>
__global__ void __launch_bounds__(kThreads) k_product(Bufs bufs, Geo g, const ProdItem* __restrict__ items,
                                                      ProdItem one, int rpl, uint64_t seed, uint64_t first_id,
                                                      MuBits mu)
{
    extern __shared__ uint32_t lds[];
    ProdItem it = items ? items[blockIdx.y] : one;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int W = g.W;
    const int LPR = W / WPL;
    const int RPW = 64 / LPR;
    const bool active = lane < RPW * LPR;
    const int sub = lane % LPR, rloc = lane / LPR;
    const int w0 = sub * WPL;
    const int TR = kWaves * RPW * rpl;
    const int row_base = blockIdx.x * TR;

    uint64_t dst_shift = 0, ct_id = 0;
    if (ENC) {
        ct_id = first_id + blockIdx.y;
        dst_shift = (uint64_t)blockIdx.y * (uint64_t)bufs.ct_words;
        it.cG[0] = (int8_t)((mu.w[blockIdx.y >> 5] >> (blockIdx.y & 31)) & 1u);
    }
    const uint32_t* Lp = ENC ? nullptr : ctp(bufs, it.L);
    const uint32_t* Rp = ctp(bufs, it.R);
    const uint64_t M64 = (uint64_t)(g.nct + 63) / 64;
    const uint64_t enc_base = sm_mix(seed + 4ull * 0x9E3779B97F4A7C15ull);

    uint32_t acc[RPLMAX][WPL], cnt[RPLMAX][WPL];
#pragma unroll
    for (int i = 0; i < RPLMAX; i++)
#pragma unroll
        for (int u = 0; u < WPL; u++) acc[i][u] = cnt[i][u] = 0;

    uint32_t* T = lds;
    const int nchunks = g.nct / 32;
    const int ntask = kGroups * 16 * g.n1;
    for (int c = 0; c < nchunks; c++) {
        __syncthreads();
        for (int task = tid; task < ntask; task += kThreads) {
            const int e = task % g.n1;
            const int v = (task / g.n1) & 15;
            const int grp = task / (16 * g.n1);
            const uint32_t* r0 = Rp + (size_t)(c * 32 + grp * 4) * W + e * g.kw;
            uint32_t* dst = T + (grp * 16 + v) * W + e * g.kw;
            uint64_t carry = 0;
            for (int l = 0; l < g.kw; l++) {
                uint64_t s = carry;
                if (v & 1) s += r0[l];
                if (v & 2) s += r0[W + l];
                if (v & 4) s += r0[2 * W + l];
                if (v & 8) s += r0[3 * W + l];
                dst[l] = (uint32_t)s;
                carry = s >> 32;
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < RPLMAX; i++) {
            if (i >= rpl) break;
            const int row = row_base + (wave * rpl + i) * RPW + rloc;
            uint32_t Lw = 0;
            if (active && row < g.nct) {
                if (ENC) {
                    const uint64_t widx = ct_id * (uint64_t)g.nct * M64 + (uint64_t)row * M64 + (uint64_t)(c >> 1);
                    const uint64_t wd = sm_mix(enc_base + (widx + 1) * 0x9E3779B97F4A7C15ull);
                    Lw = (uint32_t)(wd >> (32 * (c & 1)));
                } else {
                    Lw = Lp[(size_t)row * W + c];
                }
            }
#pragma unroll
            for (int grp = 0; grp < kGroups; grp++) {
                const uint32_t idx = (Lw >> (4 * grp)) & 15u;
                const uint32_t* t = T + (grp * 16 + idx) * W + w0;
#pragma unroll
                for (int u = 0; u < WPL; u++) {
                    const uint32_t x = t[u];
                    const uint64_t s = (uint64_t)acc[i][u] + x;
                    acc[i][u] = (uint32_t)s;
                    cnt[i][u] += (uint32_t)(s >> 32);
                }
            }
        }
    }

    // epilogue: stage one row-iteration of limb sums per wave in LDS, then
    // one lane per (row, element) resolves carries and writes the outputs
    __syncthreads();
    uint32_t* E = lds + wave * (RPW * W * 2);
    for (int i = 0; i < rpl; i++) {
        if (active) {
#pragma unroll
            for (int u = 0; u < WPL; u++) {
                E[(rloc * W + w0 + u) * 2] = acc[i][u];
                E[(rloc * W + w0 + u) * 2 + 1] = cnt[i][u];
            }
        }
        __syncthreads();
        for (int task = lane; task < RPW * g.n1; task += 64) {
            const int rl = task / g.n1, e = task % g.n1;
            const int row = row_base + (wave * rpl + i) * RPW + rl;
            if (row < g.nct) epilogue_element(bufs, g, it, E + rl * W * 2, Lp, Rp, row, e, dst_shift);
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kThreads) k_linear(Bufs bufs, Geo g, const LinItem* __restrict__ items, LinItem one)
{
    const LinItem it = items ? items[blockIdx.y] : one;
    const int task = blockIdx.x * kThreads + threadIdx.x;
    if (task >= g.nct * g.n1) return;
    const int row = task / g.n1, e = task % g.n1;
    const int br = row / g.k, tr = row % g.k;
    uint32_t* dst = ctp(bufs, it.dst);
    const uint32_t* X = it.X >= 0 ? ctp(bufs, it.X) : nullptr;
    const uint32_t* Y = it.Y >= 0 ? ctp(bufs, it.Y) : nullptr;
    int64_t carry = 0;
    for (int l = 0; l < g.kw; l++) {
        const size_t off = (size_t)row * g.W + e * g.kw + l;
        int64_t s = carry;
        if (X) s += (int64_t)it.cX * X[off];
        if (Y) s += (int64_t)it.cY * Y[off];
        if (e == br && l == (tr >> 5)) s += (int64_t)it.cG * (int64_t)(1u << (tr & 31));
        dst[off] = (uint32_t)s;
        carry = s >> 32;
    }
}

template <int WPL, int RPLMAX, bool ENC>
hipError_t launch_t(const Bufs& b, const Geo& g, const ProdCfg& cfg, const ProdItem* d_items, const ProdItem& one,
                    int64_t count, uint64_t seed, uint64_t first_id, const MuBits* mu, hipStream_t s)
{
    static int attr_bytes = 64 * 1024;
    if (cfg.lds_bytes > attr_bytes) {
        hipError_t e = hipFuncSetAttribute((const void*)k_product<WPL, RPLMAX, ENC>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, cfg.lds_bytes);
        if (e != hipSuccess) return e;
        attr_bytes = cfg.lds_bytes;
    }
    const int tiles = (g.nct + cfg.tr - 1) / cfg.tr;
    MuBits none{};
    for (int64_t b0 = 0; b0 < count; b0 += 65535) {
        const int64_t n = count - b0 < 65535 ? count - b0 : 65535;
        dim3 grid(tiles, (unsigned)n);
        hipLaunchKernelGGL((k_product<WPL, RPLMAX, ENC>), grid, dim3(kThreads), cfg.lds_bytes, s, b, g,
                           d_items ? d_items + b0 : nullptr, one, cfg.rpl, seed, first_id + (uint64_t)b0,
                           mu ? *mu : none);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <bool ENC>
hipError_t dispatch(const Bufs& b, const Geo& g, const ProdCfg& cfg, const ProdItem* d_items, const ProdItem& one,
                    int64_t count, uint64_t seed, uint64_t first_id, const MuBits* mu, hipStream_t s)
{
    switch (cfg.wpl) {
#define CASE(WPL, RPLMAX) \
    case WPL: return launch_t<WPL, RPLMAX, ENC>(b, g, cfg, d_items, one, count, seed, first_id, mu, s);
        CASE(1, 8)
        CASE(2, 8)
        CASE(3, 8)
        CASE(4, 8)
        CASE(6, 8)
        CASE(8, 8)
        CASE(11, 8)
        CASE(13, 7)
#undef CASE
    default: return hipErrorInvalidValue;
    }
}

}  // namespace

int rplmax_for(int wpl) { return wpl == 13 ? 7 : 8; }

bool product_config(const Geo& g, ProdCfg* cfg)
{
    static const int cands[] = {13, 11, 8, 6, 4, 3, 2, 1};
    if (g.nct % 32 != 0 || g.W * 32 != g.nct) return false;
    for (int wpl : cands) {
        if (g.W % wpl) continue;
        const int lpr = g.W / wpl;
        if (lpr > 64) continue;
        const int rpw = 64 / lpr;
        // rows per lane: enough rows per workgroup to amortise the tables,
        // not more than the product has
        int rpl = rplmax_for(wpl);
        while (rpl > 1 && kWaves * rpw * (rpl - 1) >= g.nct) rpl--;
        cfg->wpl = wpl;
        cfg->rpl = rpl;
        cfg->rpw = rpw;
        cfg->tr = kWaves * rpw * rpl;
        const int tbl = kGroups * 16 * g.W;
        const int epi = kWaves * rpw * g.W * 2;
        cfg->lds_bytes = 4 * (tbl > epi ? tbl : epi);
        return cfg->lds_bytes <= 160 * 1024;
    }
    return false;
}

hipError_t launch_products(const Bufs& b, const Geo& g, const ProdCfg& cfg, const ProdItem* d_items, int64_t count,
                           hipStream_t s)
{
    if (count <= 0) return hipSuccess;
    ProdItem none{};
    return dispatch<false>(b, g, cfg, d_items, none, count, 0, 0, nullptr, s);
}

hipError_t launch_product_one(const Bufs& b, const Geo& g, const ProdCfg& cfg, const ProdItem& item, hipStream_t s)
{
    return dispatch<false>(b, g, cfg, nullptr, item, 1, 0, 0, nullptr, s);
}

hipError_t launch_linear(const Bufs& b, const Geo& g, const LinItem* d_items, int64_t count, hipStream_t s)
{
    LinItem none{};
    const int blocks = (g.nct * g.n1 + kThreads - 1) / kThreads;
    for (int64_t b0 = 0; b0 < count; b0 += 65535) {
        const int64_t n = count - b0 < 65535 ? count - b0 : 65535;
        hipLaunchKernelGGL(k_linear, dim3(blocks, (unsigned)n), dim3(kThreads), 0, s, b, g, d_items + b0, none);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_linear_one(const Bufs& b, const Geo& g, const LinItem& item, hipStream_t s)
{
    const int blocks = (g.nct * g.n1 + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_linear, dim3(blocks, 1), dim3(kThreads), 0, s, b, g, (const LinItem*)nullptr, item);
    return hipGetLastError();
}

hipError_t launch_encrypt(const Bufs& b, const Geo& g, const ProdCfg& cfg, const uint32_t* bits, int n_ct,
                          uint64_t seed, uint64_t first_id, hipStream_t s)
{
    if (n_ct <= 0) return hipSuccess;
    if (n_ct > kMaxEncPerLaunch) return hipErrorInvalidValue;
    MuBits mu{};
    for (int i = 0; i < (n_ct + 31) / 32; i++) mu.w[i] = bits[i];
    ProdItem one{};
    one.L = -1;
    one.R = ct_ref(B_AUX, 0);
    one.nout = 1;
    one.dst[0] = ct_ref(B_OUT, 0);
    one.E[0] = -1;
    one.cP[0] = 1;
    for (int i = 1; i < kMaxOut; i++) one.dst[i] = one.E[i] = -1;
    return dispatch<true>(b, g, cfg, nullptr, one, n_ct, seed, first_id, &mu, s);
}

}  // namespace sfft
