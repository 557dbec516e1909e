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
// 1970).  Per chunk of 32 rows of R, a workgroup re-encodes the rows into
// 30-bit digits (a sum of four digits fits 32 bits, so the tables need no
// carries) and builds 8 tables x 16 subset sums in LDS, while the next
// chunk's rows of R and words of L are already in flight into registers.
// Each half-wave owns one output row and reads 32 consecutive digits of one
// table entry per lookup (no LDS bank conflicts); every lane adds the digit
// into a 64-bit accumulator (one v_mad_u64_u32, no carry flag).  Integer
// VALU and LDS only.
//
// Epilogue (fused): per (row, element) the exact digit sums are carried into
// P mod 2^k limb by limb and combined into up to four outputs
// a L + b R + c P + g G + e E (AND, XOR, OR, NOT, NAND, XADD forms).
#include <hip/hip_runtime.h>

#include "device.hpp"

namespace sfft {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kGroups = 8;          // 4-bit groups per 32-row chunk of R
constexpr int kDigitBits = 30;      // 4 * (2^30 - 1) < 2^32
constexpr uint32_t kDigitMask = (1u << kDigitBits) - 1u;
constexpr int kMaxChunkWords = 4096;  // 32 rows of R, W <= 128 words per row
constexpr int kMaxDigitSlots = 128;   // digits per row incl. padding
constexpr int kPassMinRows = 64;      // rows staged per epilogue pass (at least)

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

// Output row `row`, element e: carry the exact digit sums A[0..nd) (digit d
// weighs 2^(30 d)) into the limbs of P mod 2^k and write every output of the
// item, limb by limb with signed carries.
__device__ void finish_element(const Bufs& bufs, const Geo& g, const ProdItem& it, const uint64_t* A, int nd,
                               const uint32_t* Lp, const uint32_t* Rp, int row, int e, uint64_t dst_shift)
{
    const int br = row / g.k, tr = row % g.k;
    const size_t base = (size_t)row * g.W + (size_t)e * g.kw;
    int64_t carry[kMaxOut];
    uint32_t* dst[kMaxOut];
    const uint32_t* Ep[kMaxOut];
    bool needL = false, needR = false;
#pragma unroll
    for (int o = 0; o < kMaxOut; o++) {
        carry[o] = 0;
        dst[o] = o < it.nout ? ctp(bufs, it.dst[o]) + dst_shift : nullptr;
        Ep[o] = (o < it.nout && it.E[o] >= 0) ? ctp(bufs, it.E[o]) : nullptr;
        if (o < it.nout) {
            needL |= it.cL[o] != 0;
            needR |= it.cR[o] != 0;
        }
    }
    auto emit = [&](int l, uint32_t P) {
        const size_t off = base + l;
        const uint32_t Gv = (e == br && l == (tr >> 5)) ? (1u << (tr & 31)) : 0u;
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
    };
    unsigned __int128 V = 0;  // pending bits from position `pos` up
    int pos = 0, l = 0;
    for (int d = 0; d < nd; d++) {
        V += (unsigned __int128)A[d] << (kDigitBits * d - pos);
        while (l < g.kw && pos + 32 <= kDigitBits * (d + 1)) {
            emit(l++, (uint32_t)V);
            V >>= 32;
            pos += 32;
        }
    }
    while (l < g.kw) {
        emit(l++, (uint32_t)V);
        V >>= 32;
    }
}

// THREADS threads per workgroup, LPR lanes per output row, DPL digit slots
// per lane held as DPL/4 groups of 4 consecutive digits (lane slot group
// q covers digits 4 (lane % LPR + LPR q) .. +3, read with one ds_read_b128),
// up to RPLMAX rows per lane.
template <int THREADS, int LPR, int DPL, int RPLMAX, bool ENC>
__global__ void __launch_bounds__(THREADS) k_product(Geo g, KCfg kc, const ProdSeg* __restrict__ segs, int nseg,
                                                     ProdSeg seg0, ProdItem one, uint32_t ybase, uint64_t seed,
                                                     uint64_t first_id, MuBits mu)
{
    constexpr int NW = THREADS / 64;
    constexpr int RPW = 64 / LPR;      // rows per wave per row-iteration
    constexpr int NQ = DPL / 4;        // 16-byte table reads per lookup
    constexpr int st = LPR * DPL;      // digit slots per table entry
    constexpr int RPF = (kMaxChunkWords + THREADS - 1) / THREADS;
    constexpr int BT = (kGroups * kMaxDigitSlots + THREADS - 1) / THREADS;
    constexpr int LR = (NW * RPW * RPLMAX + THREADS - 1) / THREADS;
    constexpr int PI = (kPassMinRows + NW * RPW - 1) / (NW * RPW);  // row-iterations per epilogue pass
    constexpr int PASS_ROWS = NW * RPW * PI;
    static_assert(DPL % 4 == 0, "digit slots come in groups of 4");

    extern __shared__ uint32_t lds[];
    // work item of this workgroup: segment (a request's buffers and items) by
    // binary search over the segments' first global item index
    const uint32_t y = blockIdx.y + ybase;
    ProdSeg sg = seg0;
    if (nseg > 1) {
        int lo = 0, hi = nseg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (segs[mid].first <= y) lo = mid;
            else hi = mid - 1;
        }
        sg = segs[lo];
    }
    const Bufs bufs = sg.bufs;
    ProdItem it = sg.items ? sg.items[y - sg.first] : one;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rsub = lane / LPR, lq = lane % LPR;
    const int W = g.W, kw = g.kw, nd = kc.nd, wd = kc.wd;
    const int rpl = kc.rpl, TR = kc.tr;
    const int row_base = blockIdx.x * TR;

    uint64_t dst_shift = 0, ct_id = 0;
    if (ENC) {
        ct_id = first_id + y;
        dst_shift = (uint64_t)y * (uint64_t)bufs.ct_words;
        it.cG[0] = (int8_t)((mu.w[y >> 5] >> (y & 31)) & 1u);
    }
    const uint32_t* Lp = ENC ? nullptr : ctp(bufs, it.L);
    const uint32_t* Rp = ctp(bufs, it.R);
    const uint64_t M64 = (uint64_t)(g.nct + 63) / 64;
    const uint64_t enc_base = sm_mix(seed + 4ull * 0x9E3779B97F4A7C15ull);

    // Ls is double-buffered by chunk parity: a wave still looking up chunk c
    // reads its half while faster waves stage chunk c+1 into the other.
    uint32_t* Rs = lds;            // 32 x W raw words of the chunk's rows of R
    uint32_t* Ls = Rs + 32 * W;    // 2 x TR words of L (a chunk's 32 bits of each row); TR % 4 == 0
    uint32_t* T = Ls + 2 * TR;     // 8 groups x 16 subset sums x st digit slots, 16-byte aligned
    for (int q = tid; q < kGroups * 16 * st; q += THREADS) T[q] = 0;  // empty subsets, padding slots

    // table tasks of this thread: (group, digit slot) -> word offset and shift
    int bt_off[BT], bt_sh[BT], bt_dst[BT];
    bool bt_ok[BT], bt_hi[BT];
#pragma unroll
    for (int q = 0; q < BT; q++) {
        const int task = tid + q * THREADS;
        bt_ok[q] = task < kGroups * wd;
        const int slot = bt_ok[q] ? task % wd : 0, grp = bt_ok[q] ? task / wd : 0;
        const int e = slot / nd, d = slot % nd, o = kDigitBits * d;
        bt_off[q] = grp * 4 * W + e * kw + (o >> 5);
        bt_sh[q] = o & 31;
        bt_hi[q] = (o >> 5) + 1 < kw;
        bt_dst[q] = grp * 16 * st + slot;
    }

    uint64_t acc[RPLMAX][DPL];
#pragma unroll
    for (int i = 0; i < RPLMAX; i++)
#pragma unroll
        for (int u = 0; u < DPL; u++) acc[i][u] = 0;

    const int nchunks = g.nct / 32;
    const int chunk_words = 32 * W;
    uint32_t rpf[RPF];
    uint32_t lpf[LR];
    auto load_R = [&](int c) {
        const uint32_t* src = Rp + (size_t)c * chunk_words;
#pragma unroll
        for (int q = 0; q < RPF; q++) {
            const int idx = tid + q * THREADS;
            rpf[q] = idx < chunk_words ? src[idx] : 0u;
        }
    };
    auto load_L = [&](int c) {
#pragma unroll
        for (int q = 0; q < LR; q++) {
            const int lr = tid + q * THREADS;
            const int row = row_base + lr;
            uint32_t v = 0;
            if (lr < TR && row < g.nct) {
                if (ENC) {
                    const uint64_t widx = ct_id * (uint64_t)g.nct * M64 + (uint64_t)row * M64 + (uint64_t)(c >> 1);
                    const uint64_t wd64 = sm_mix(enc_base + (widx + 1) * 0x9E3779B97F4A7C15ull);
                    v = (uint32_t)(wd64 >> (32 * (c & 1)));
                } else {
                    v = Lp[(size_t)row * W + c];
                }
            }
            lpf[q] = v;
        }
    };

    load_R(0);
    load_L(0);
    for (int c = 0; c < nchunks; c++) {
        // stage this chunk; start loading the next one
#pragma unroll
        for (int q = 0; q < RPF; q++) {
            const int idx = tid + q * THREADS;
            if (idx < chunk_words) Rs[idx] = rpf[q];
        }
        uint32_t* Lc = Ls + (c & 1) * TR;
#pragma unroll
        for (int q = 0; q < LR; q++)
            if (tid + q * THREADS < TR) Lc[tid + q * THREADS] = lpf[q];
        if (c + 1 < nchunks) {
            load_R(c + 1);
            load_L(c + 1);
        }
        __syncthreads();
        // digits of 4 rows at one slot -> the 15 non-empty subset sums
#pragma unroll
        for (int q = 0; q < BT; q++) {
            if (!bt_ok[q]) continue;
            const uint32_t* r = Rs + bt_off[q];
            uint32_t d[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const uint32_t lo = r[j * W];
                const uint32_t hi = bt_hi[q] ? r[j * W + 1] : 0u;
                d[j] = __builtin_amdgcn_alignbit(hi, lo, bt_sh[q]) & kDigitMask;
            }
            uint32_t* tb = T + bt_dst[q];
            const uint32_t s01 = d[0] + d[1], s02 = d[0] + d[2], s12 = d[1] + d[2], s012 = s01 + d[2];
            tb[1 * st] = d[0];
            tb[2 * st] = d[1];
            tb[3 * st] = s01;
            tb[4 * st] = d[2];
            tb[5 * st] = s02;
            tb[6 * st] = s12;
            tb[7 * st] = s012;
            tb[8 * st] = d[3];
            tb[9 * st] = d[0] + d[3];
            tb[10 * st] = d[1] + d[3];
            tb[11 * st] = s01 + d[3];
            tb[12 * st] = d[2] + d[3];
            tb[13 * st] = s02 + d[3];
            tb[14 * st] = s12 + d[3];
            tb[15 * st] = s012 + d[3];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < RPLMAX; i++) {
            if (i < rpl) {
                const uint32_t Lw = Lc[(wave * rpl + i) * RPW + rsub];
#pragma unroll
                for (int grp = 0; grp < kGroups; grp++) {
                    const uint32_t idx = __builtin_amdgcn_ubfe(Lw, 4 * grp, 4);
                    const uint4* t = reinterpret_cast<const uint4*>(T + (grp * 16 + idx) * st) + lq;
#pragma unroll
                    for (int q = 0; q < NQ; q++) {
                        const uint4 x = t[q * LPR];
                        acc[i][4 * q + 0] = (uint64_t)x.x * kc.one + acc[i][4 * q + 0];
                        acc[i][4 * q + 1] = (uint64_t)x.y * kc.one + acc[i][4 * q + 1];
                        acc[i][4 * q + 2] = (uint64_t)x.z * kc.one + acc[i][4 * q + 2];
                        acc[i][4 * q + 3] = (uint64_t)x.w * kc.one + acc[i][4 * q + 3];
                    }
                }
            }
        }
    }

    // epilogue in passes of PI row-iterations: stage the digit sums in LDS,
    // then one thread per (row, element) finishes it
    uint64_t* E = reinterpret_cast<uint64_t*>(lds);
#pragma unroll
    for (int p = 0; p < (RPLMAX + PI - 1) / PI; p++) {
        if (p * PI >= rpl) continue;  // uniform across the workgroup
        __syncthreads();
#pragma unroll
        for (int ii = 0; ii < PI; ii++) {
            const int i = p * PI + ii;
            if (i < RPLMAX && i < rpl) {
                const int pr = (wave * PI + ii) * RPW + rsub;
#pragma unroll
                for (int q = 0; q < NQ; q++)
#pragma unroll
                    for (int c4 = 0; c4 < 4; c4++) E[pr * st + 4 * (lq + LPR * q) + c4] = acc[i][4 * q + c4];
            }
        }
        __syncthreads();
        for (int task = tid; task < PASS_ROWS * g.n1; task += THREADS) {
            const int pr = task / g.n1, e = task % g.n1;
            const int wv = pr / (PI * RPW), ii = (pr / RPW) % PI, rs = pr % RPW;
            const int i = p * PI + ii;
            if (i >= rpl) continue;
            const int row = row_base + (wv * rpl + i) * RPW + rs;
            if (row >= g.nct) continue;
            finish_element(bufs, g, it, E + pr * st + e * nd, nd, Lp, Rp, row, e, dst_shift);
        }
    }
}

__global__ void __launch_bounds__(kThreads) k_linear(Geo g, const LinSeg* __restrict__ segs, int nseg, LinSeg seg0,
                                                     LinItem one, uint32_t ybase)
{
    const uint32_t y = blockIdx.y + ybase;
    LinSeg sg = seg0;
    if (nseg > 1) {
        int lo = 0, hi = nseg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (segs[mid].first <= y) lo = mid;
            else hi = mid - 1;
        }
        sg = segs[lo];
    }
    const Bufs bufs = sg.bufs;
    const LinItem it = sg.items ? sg.items[y - sg.first] : one;
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

template <int THREADS, int LPR, int DPL, int RPLMAX, bool ENC>
hipError_t launch_t(const Geo& g, const ProdCfg& cfg, const ProdSeg* d_segs, int nseg, const ProdSeg& seg0,
                    const ProdItem& one, int64_t total, uint64_t seed, uint64_t first_id, const MuBits* mu,
                    hipStream_t s)
{
    static int attr_bytes = 64 * 1024;
    if (cfg.lds_bytes > attr_bytes) {
        hipError_t e = hipFuncSetAttribute((const void*)k_product<THREADS, LPR, DPL, RPLMAX, ENC>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, cfg.lds_bytes);
        if (e != hipSuccess) return e;
        attr_bytes = cfg.lds_bytes;
    }
    const int tiles = (g.nct + cfg.tr - 1) / cfg.tr;
    const KCfg kc{cfg.nd, cfg.wd, cfg.st, cfg.rpl, cfg.tr, 1u};
    MuBits none{};
    for (int64_t b0 = 0; b0 < total; b0 += 65535) {
        const int64_t n = total - b0 < 65535 ? total - b0 : 65535;
        dim3 grid(tiles, (unsigned)n);
        hipLaunchKernelGGL((k_product<THREADS, LPR, DPL, RPLMAX, ENC>), grid, dim3(THREADS), cfg.lds_bytes, s, g, kc,
                           d_segs, nseg, seg0, one, (uint32_t)b0, seed, first_id, mu ? *mu : none);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Tilings: (threads, lanes per row, digit slots per lane, rows per lane).
struct Tiling {
    int threads, lpr, dpl, rplmax;
};
constexpr Tiling kTilings[] = {
    {256, 4, 4, 8},    // rows of <= 16 digits
    {256, 8, 4, 16},   // <= 32
    {256, 8, 8, 8},    // <= 64
    {256, 8, 12, 5},   // <= 96
    {256, 8, 16, 4},   // <= 128
};

template <bool ENC>
hipError_t dispatch(const Geo& g, const ProdCfg& cfg, const ProdSeg* d_segs, int nseg, const ProdSeg& seg0,
                    const ProdItem& one, int64_t total, uint64_t seed, uint64_t first_id, const MuBits* mu,
                    hipStream_t s)
{
#define CASE(I)                                                                                              \
    if (cfg.tiling == I)                                                                                     \
        return launch_t<kTilings[I].threads, kTilings[I].lpr, kTilings[I].dpl, kTilings[I].rplmax, ENC>(     \
            g, cfg, d_segs, nseg, seg0, one, total, seed, first_id, mu, s);
    CASE(0)
    CASE(1)
    CASE(2)
    CASE(3)
    CASE(4)
#undef CASE
    return hipErrorInvalidValue;
}

}  // namespace

bool product_config(const Geo& g, ProdCfg* cfg)
{
    if (g.nct % 32 != 0 || g.W * 32 != g.nct || 32 * g.W > kMaxChunkWords) return false;
    const int nd = (g.k + kDigitBits - 1) / kDigitBits;
    const int wd = g.n1 * nd;
    int ti = -1;
    for (int i = 0; i < (int)(sizeof(kTilings) / sizeof(kTilings[0])); i++)
        if (kTilings[i].lpr * kTilings[i].dpl >= wd) {
            ti = i;
            break;
        }
    if (ti < 0) return false;
    const Tiling& t = kTilings[ti];
    cfg->tiling = ti;
    cfg->nd = nd;
    cfg->wd = wd;
    cfg->lpr = t.lpr;
    cfg->dpl = t.dpl;
    cfg->st = t.lpr * t.dpl;
    cfg->rpw = 64 / t.lpr;
    const int per_iter = (t.threads / 64) * cfg->rpw;
    int rpl = (g.nct + per_iter - 1) / per_iter;
    if (rpl > t.rplmax) rpl = t.rplmax;
    cfg->rpl = rpl;
    cfg->tr = per_iter * rpl;
    const int pi = (kPassMinRows + per_iter - 1) / per_iter;
    const int main_words = 32 * g.W + 2 * cfg->tr + kGroups * 16 * cfg->st;
    const int epi_words = 2 * per_iter * pi * cfg->st;
    cfg->lds_bytes = 4 * (main_words > epi_words ? main_words : epi_words);
    return cfg->lds_bytes <= 160 * 1024;
}

hipError_t launch_products(const Geo& g, const ProdCfg& cfg, const ProdSeg* d_segs, int nseg,
                           const ProdSeg& seg0, int64_t total, hipStream_t s)
{
    if (total <= 0) return hipSuccess;
    ProdItem none{};
    return dispatch<false>(g, cfg, d_segs, nseg, seg0, none, total, 0, 0, nullptr, s);
}

hipError_t launch_product_one(const Bufs& b, const Geo& g, const ProdCfg& cfg, const ProdItem& item, hipStream_t s)
{
    const ProdSeg seg0{nullptr, b, 0, 0};
    return dispatch<false>(g, cfg, nullptr, 1, seg0, item, 1, 0, 0, nullptr, s);
}

hipError_t launch_linear(const Geo& g, const LinSeg* d_segs, int nseg, const LinSeg& seg0, int64_t total,
                         hipStream_t s)
{
    LinItem none{};
    const int blocks = (g.nct * g.n1 + kThreads - 1) / kThreads;
    for (int64_t b0 = 0; b0 < total; b0 += 65535) {
        const int64_t n = total - b0 < 65535 ? total - b0 : 65535;
        hipLaunchKernelGGL(k_linear, dim3(blocks, (unsigned)n), dim3(kThreads), 0, s, g, d_segs, nseg, seg0, none,
                           (uint32_t)b0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_linear_one(const Bufs& b, const Geo& g, const LinItem& item, hipStream_t s)
{
    const int blocks = (g.nct * g.n1 + kThreads - 1) / kThreads;
    const LinSeg seg0{nullptr, b, 0, 0};
    hipLaunchKernelGGL(k_linear, dim3(blocks, 1), dim3(kThreads), 0, s, g, (const LinSeg*)nullptr, 1, seg0, item,
                       0u);
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
    const ProdSeg seg0{nullptr, b, 0, 0};
    return dispatch<true>(g, cfg, nullptr, 1, seg0, one, n_ct, seed, first_id, &mu, s);
}

}  // namespace sfft
