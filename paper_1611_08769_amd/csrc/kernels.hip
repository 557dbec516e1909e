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
// 1970).  A workgroup owns a tile of output rows and walks R in chunks of 16
// or 32 rows.  Per chunk it re-encodes the rows into 30-bit digits (a sum of
// four digits fits 32 bits, so the tables need no carries) and builds the
// chunk's tables of subset sums in LDS, one table set ahead of the lookups,
// with one barrier per chunk.  Lanes of a row each read 4 consecutive digits
// of the selected entry with one ds_read_b128 and add them into 64-bit
// accumulators (v_mad_u64_u32 with a multiplier of one: no carry flags, no
// zero-extended register pairs).  Integer VALU and LDS only.
//
// Epilogue (fused): per (row, element) the exact digit sums become 32-bit
// column sums that feed, limb by limb, up to four outputs
// a L + b R + c P + g G + e E (AND, XOR, OR, NOT, NAND, XADD forms) mod 2^k.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>

#include "device.hpp"

namespace sfft {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kDigitBits = 30;      // 4 * (2^30 - 1) < 2^32
constexpr uint32_t kDigitMask = (1u << kDigitBits) - 1u;
constexpr int kMaxRowWords = 128;     // words per ciphertext row (W)
constexpr int kMaxDigitSlots = 128;   // digits per row incl. padding

// Ciphertext words in the global address space: loads and stores through
// these pointers compile to global (not flat) instructions, which the LDS
// wait counter does not track, so an LDS wait never waits for them.
typedef __attribute__((address_space(1))) uint32_t gword;

__device__ __forceinline__ gword* ctp(const Bufs& b, int32_t ref)
{
    const uint32_t u = (uint32_t)ref;
    const uint32_t buf = u >> 29;
    const uint64_t idx = u & 0x1FFFFFFFu;
    uint32_t* base = buf == B_IN ? b.in : buf == B_OUT ? b.out : buf == B_WS ? b.ws : b.aux;
    return (gword*)(base + idx * (uint64_t)b.ct_words);
}

// Index of the last segment whose key (first item or first workgroup) is
// <= y (the keys ascend), found by the whole wave at once: lane i tests segment base + i and
// the highest lane that passes is the answer.  One round of loads per 64
// segments instead of a chain of dependent loads.
template <class Seg, class Key>
__device__ __forceinline__ int find_segment(const Seg* segs, int nseg, uint32_t y, Key key)
{
    const int lane = threadIdx.x & 63;
    int found = 0;
    for (int base = 0; base < nseg; base += 64) {
        const int i = base + lane;
        const bool le = i < nseg && key(segs[i]) <= y;
        const uint64_t m = __ballot(le);
        if (m) found = base + 63 - __clzll(m);
        if (m != ~0ull) break;
    }
    // the same on every lane: keep it (and the segment) in scalar registers
    return __builtin_amdgcn_readfirstlane(found);
}

// Workgroups are handed to the 8 XCDs in turn (workgroup b to XCD b mod 8).
// Renumber them so that each XCD works through one contiguous range of the
// launch's (item, row tile) order: the row tiles of one product, which all
// read its whole right operand, then share one XCD's L2.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_order(uint32_t b, uint32_t n)
{
    const uint32_t x = b % kXcds, k = b / kXcds;
    const uint32_t per = n / kXcds, rem = n % kXcds;
    return x * per + (x < rem ? x : rem) + k;
}

// A copy of a value that is the same in every lane of the wave, taken word by
// word from the first active lane: the compiler keeps it in scalar registers
// instead of vector ones.
template <class T>
__device__ __forceinline__ T wave_uniform(const T& x)
{
    static_assert(sizeof(T) % 4 == 0, "whole words");
    T v;
    const uint32_t* src = reinterpret_cast<const uint32_t*>(&x);
    uint32_t* dst = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); i++) dst[i] = __builtin_amdgcn_readfirstlane(src[i]);
    return v;
}

// A work item read word by word through the global address space.
template <class T>
__device__ __forceinline__ T load_global(const T* p)
{
    static_assert(sizeof(T) % 4 == 0, "work items are whole words");
    T v;
    const gword* src = (const gword*)p;
    uint32_t* w = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); i++) w[i] = src[i];
    return v;
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

// Row-iterations per epilogue pass: as many as the workgroup's share of LDS
// (160 KB for 512 threads, 80 KB for 256, so that two of those fit a CU)
// holds as 64-bit digit sums, so that few accumulators stay live across the
// passes.
constexpr int pass_iters(int threads, int rpw, int st, int rpl)
{
    const int cap = 160 * 1024 * threads / 512;
    const int per = (threads / 64) * rpw * st * 8;
    const int pi = cap / per;
    return pi < 1 ? 1 : pi > rpl ? rpl : pi;
}

// Output row `row`, element e.  The exact digit sums A[0..nd) (digit d
// weighs 2^(30 d)) are split into 32-bit column sums, 16 digits onto 15 limbs
// (480 bits) at a time; every output a L + b R + c P + g G + e E of the item
// is formed from the column sums limb by limb with one signed carry chain per
// output, so that P is never carried on its own.  The words of L and R (and
// of each output's E) for up to 8 limbs are loaded before the arithmetic that
// uses them, so that their latencies overlap.
__device__ void finish_element(const Bufs& bufs, const Geo& g, const ProdItem& it, const uint64_t* A, int nd,
                               const gword* Lp, const gword* Rp, int row, int e, uint64_t dst_shift)
{
    const int br = row / g.k, tr = row % g.k;
    const size_t base = (size_t)row * g.W + (size_t)e * g.kw;
    int64_t carry[kMaxOut];
    bool needL = false, needR = false;
#pragma unroll
    for (int o = 0; o < kMaxOut; o++) {
        carry[o] = 0;
        if (o < it.nout) {
            needL |= it.cL[o] != 0;
            needR |= it.cR[o] != 0;
        }
    }
    uint64_t next0 = 0, next1 = 0;  // column sums that reach the next group's limbs 0 and 1
    for (int l0 = 0, d0 = 0; l0 < g.kw; l0 += 15, d0 += 16) {
        uint64_t col[17];
        col[0] = next0;
        col[1] = next1;
#pragma unroll
        for (int j = 2; j < 17; j++) col[j] = 0;
#pragma unroll
        for (int t = 0; t < 16; t++) {
            // digit d0 + t starts at bit 30 t of the group: limb j0, bit sh
            const uint64_t a = d0 + t < nd ? A[d0 + t] : 0;
            const int j0 = (30 * t) >> 5, sh = (30 * t) & 31;
            const uint64_t hi = sh ? a >> (32 - sh) : a >> 32;  // bits 32 and up of a 2^sh
            col[j0] += (uint32_t)(a << sh);
            col[j0 + 1] += (uint32_t)hi;
            col[j0 + 2] += hi >> 32;
        }
        next0 = col[15];
        next1 = col[16];
        // the group's limbs in two halves of at most 8
#pragma unroll
        for (int h = 0; h < 2; h++) {
            const int j1 = 8 * h, nh = h ? 7 : 8;
            const int lh = l0 + j1;
            const int nl = g.kw - lh < nh ? g.kw - lh : nh;
            if (nl <= 0) break;
            const size_t off = base + lh;
            uint32_t Lv[8], Rv[8];
#pragma unroll
            for (int j = 0; j < 8; j++) {
                Lv[j] = (needL && j < nl) ? Lp[off + j] : 0u;
                Rv[j] = (needR && j < nl) ? Rp[off + j] : 0u;
            }
#pragma unroll
            for (int o = 0; o < kMaxOut; o++) {
                if (o < it.nout) {
                    gword* dst = ctp(bufs, it.dst[o]) + dst_shift + off;
                    const gword* Ep = it.E[o] >= 0 ? ctp(bufs, it.E[o]) + off : nullptr;
                    uint32_t Ev[8];
#pragma unroll
                    for (int j = 0; j < 8; j++) Ev[j] = (Ep && j < nl) ? Ep[j] : 0u;
#pragma unroll
                    for (int j = 0; j < 8; j++) {
                        if (j < nl) {
                            const int l = lh + j;
                            const uint32_t Gv = (e == br && l == (tr >> 5)) ? (1u << (tr & 31)) : 0u;
                            const int64_t s = carry[o] + (int64_t)it.cL[o] * Lv[j] + (int64_t)it.cR[o] * Rv[j] +
                                              (int64_t)it.cP[o] * (int64_t)col[j1 + j] + (int64_t)it.cG[o] * Gv +
                                              (int64_t)it.cE[o] * Ev[j];
                            dst[j] = (uint32_t)s;
                            carry[o] = s >> 32;
                        }
                    }
                }
            }
        }
    }
}

// THREADS threads per workgroup; LPR lanes per output row; DPL digit slots
// per lane, held as DPL/4 quads of consecutive digits (quad q of a lane covers
// slots 4 (lane % LPR + LPR q) .. +3 and is read with one ds_read_b128); RPL
// rows per lane, so that a workgroup covers TR = (THREADS/64)(64/LPR) RPL rows
// of the product; CG 4-bit groups (4 CG rows of R) per chunk.
//
// Chunks are pipelined with one barrier per chunk: while the waves look up
// chunk c in one table set, they build chunk c+1's tables in the other from
// rows of R staged in LDS the chunk before, stage chunk c+2's rows of R and
// bits of L, and load chunk c+3's from memory into registers.  Within a chunk
// the lookups of consecutive (row, group) steps form a software pipeline PD
// steps deep: the table reads of step s + PD are issued before the additions
// of step s.
template <int THREADS, int LPR, int DPL, int RPL, int PD, int CG, bool ENC>
__global__ void __launch_bounds__(THREADS) k_product(KCfg kc, const ProdSeg* __restrict__ segs, int nseg,
                                                     ProdSeg seg0, ProdItem one, uint64_t seed, uint64_t first_id,
                                                     MuBits mu)
{
    constexpr int NW = THREADS / 64;
    constexpr int RPW = 64 / LPR;          // rows per wave per row-iteration
    constexpr int NQ = DPL / 4;            // 16-byte table reads per lookup
    constexpr int st = LPR * DPL;          // digit slots per table entry
    constexpr int SQ = st / 4;             // slot quads per table entry
    constexpr int TR = NW * RPW * RPL;     // rows per workgroup
    constexpr int CR = 4 * CG;             // rows of R per chunk
    constexpr int TSZ = CG * 16 * st;      // words per table set
    constexpr int NSTEP = RPL * CG;        // lookup steps per chunk
    constexpr int NTASK = CG * SQ;         // table-build tasks per chunk
    constexpr int RPF = (CR * kMaxRowWords + THREADS - 1) / THREADS;
    constexpr int LR = (TR + THREADS - 1) / THREADS;
    constexpr int PI = pass_iters(THREADS, RPW, st, RPL);  // row-iterations per epilogue pass
    constexpr int PASS_ROWS = NW * RPW * PI;
    static_assert(DPL % 4 == 0, "digit slots come in quads");
    static_assert(NTASK <= THREADS, "one table-build task per thread");
    static_assert(CG == 4 || CG == 8, "chunks of 16 or 32 rows of R");
    static_assert(PD >= 1 && PD < NSTEP, "pipeline depth");

    extern __shared__ uint32_t lds[];
    // work of this workgroup: virtual index v (XCD-grouped), its segment (a
    // request's buffers, geometry and items: the last whose first workgroup
    // is <= v), then item and row tile within the segment
    const uint32_t v = xcd_order(blockIdx.x, gridDim.x);
    ProdSeg sg = seg0;  // (a select between the two structs would copy both into vector registers)
    if (nseg > 1) sg = segs[find_segment(segs, nseg, v, [](const ProdSeg& q) { return q.first_block; })];
    const Geo g = sg.geo;
    const uint32_t tiles = ((uint32_t)g.nct + TR - 1) / TR;
    const uint32_t local = v - sg.first_block;
    const uint32_t yl = local / tiles;
    const uint32_t y = sg.first + yl;  // item index within the launch (numbers encryptions)
    const int row_base = (int)(local % tiles) * TR;
    const Bufs bufs = sg.bufs;
    ProdItem it = sg.items ? load_global(sg.items + yl) : one;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int rsub = lane / LPR, lq = lane % LPR;
    const int W = g.W, kw = g.kw, nd = sg.nd, wd = sg.wd;

    uint64_t dst_shift = 0, ct_id = 0;
    if (ENC) {
        ct_id = first_id + y;
        dst_shift = (uint64_t)y * (uint64_t)bufs.ct_words;
        it.cG[0] = (int8_t)((mu.w[y >> 5] >> (y & 31)) & 1u);
    }
    const gword* Lp = ENC ? nullptr : ctp(bufs, it.L);
    const gword* Rp = ctp(bufs, it.R);
    const uint64_t M64 = (uint64_t)(g.nct + 63) / 64;
    const uint64_t enc_base = sm_mix(seed + 4ull * 0x9E3779B97F4A7C15ull);

    const int chunk_words = CR * W;
    uint32_t* Rs = lds;                    // 2 x CR rows of R (raw words), by chunk parity
    uint32_t* Ls = Rs + 2 * chunk_words;   // 3 x TR: a chunk's CR bits of each row of L, by chunk mod 3
    uint32_t* T = Ls + 3 * TR;             // 2 table sets (CG groups x 16 subset sums x st slots), by chunk parity
    // entry 0 of every group is the empty subset; the build never writes it
    for (int q = tid; q < 2 * CG * st; q += THREADS) {
        const int grp = q / st;  // over both table sets
        T[grp * 16 * st + q % st] = 0;
    }

    // table-build task of this thread: group `grp`, slot quad `sq` (slots
    // 4 sq .. 4 sq + 3).  Tasks fill whole waves, so that the build costs as
    // few wave instructions as possible.  A digit's mask keeps its bits below
    // k (the top digit of an element ends early; its high word is then the
    // next element's and is masked away); padding slots beyond wd get mask 0.
    const bool bt_task = tid < NTASK;
    const int bt_grp = bt_task ? tid / SQ : 0, bt_sq = bt_task ? tid % SQ : 0;
    int bt_off[4], bt_sh[4];
    uint32_t bt_mask[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const int slot = 4 * bt_sq + u;
        const bool ok = bt_task && slot < wd;
        const int e = ok ? slot / nd : 0, d = ok ? slot % nd : 0, o = kDigitBits * d;
        bt_off[u] = bt_grp * 4 * W + e * kw + (o >> 5);
        bt_sh[u] = o & 31;
        const int bits = g.k - o < kDigitBits ? g.k - o : kDigitBits;
        bt_mask[u] = ok ? (uint32_t)((1ull << bits) - 1) : 0u;
    }
    const int bt_dst = bt_grp * 16 * st + 4 * bt_sq;

    uint64_t acc[RPL][DPL];
#pragma unroll
    for (int i = 0; i < RPL; i++)
#pragma unroll
        for (int u = 0; u < DPL; u++) acc[i][u] = 0;

    const int nchunks = g.nct / CR;
    uint32_t rpf[RPF];
    uint32_t lpf[LR];
    bool l_ok[LR];  // staged row of L lies in the product
#pragma unroll
    for (int q = 0; q < LR; q++) l_ok[q] = tid + q * THREADS < TR && row_base + tid + q * THREADS < g.nct;
    auto load_R = [&](int c) {
        const gword* src = Rp + (size_t)c * chunk_words;
#pragma unroll
        for (int q = 0; q < RPF; q++) {
            const int idx = tid + q * THREADS;
            rpf[q] = src[idx < chunk_words ? idx : chunk_words - 1];  // words past the chunk are not staged
        }
    };
    auto stage_R = [&](int c) {
        uint32_t* dst = Rs + (c & 1) * chunk_words;
#pragma unroll
        for (int q = 0; q < RPF; q++) {
            const int idx = tid + q * THREADS;
            if (idx < chunk_words) dst[idx] = rpf[q];
        }
    };
    // bits [CR c, CR c + CR) of each row of L, in the low CR bits
    auto load_L = [&](int c) {
        const int b = CR * c;
#pragma unroll
        for (int q = 0; q < LR; q++) {
            // rows past the product read row 0 and are staged as zero
            const int rowc = l_ok[q] ? row_base + tid + q * THREADS : 0;
            if (ENC) {
                const uint64_t widx = ct_id * (uint64_t)g.nct * M64 + (uint64_t)rowc * M64 + (uint64_t)(b >> 6);
                const uint64_t w64 = sm_mix(enc_base + (widx + 1) * 0x9E3779B97F4A7C15ull);
                lpf[q] = (uint32_t)(w64 >> (b & 63));
            } else {
                lpf[q] = Lp[(size_t)rowc * W + (b >> 5)] >> (b & 31);
            }
        }
    };
    // (the mask is applied here, not at the load, so that nothing waits for
    // the load before the chunk after it)
    auto stage_L = [&](int slot) {
#pragma unroll
        for (int q = 0; q < LR; q++)
            if (tid + q * THREADS < TR) Ls[slot * TR + tid + q * THREADS] = l_ok[q] ? lpf[q] : 0u;
    };
    // Table build for chunk c in two halves: build_read issues the LDS reads
    // of the digits' words (4 rows x 4 slots, low and high word), build_write
    // (after the chunk's staging work, which hides the reads' latency) cuts the
    // digits and stores the 15 non-empty subset sums, one 16-byte store per
    // entry.
    uint32_t b_lo[4][4], b_hi[4][4];
    auto build_read = [&](int c) {
        const uint32_t* Rb = Rs + (c & 1) * chunk_words;
#pragma unroll
        for (int j = 0; j < 4; j++)
#pragma unroll
            for (int u = 0; u < 4; u++) {
                b_lo[j][u] = Rb[bt_off[u] + j * W];
                b_hi[j][u] = Rb[bt_off[u] + j * W + 1];
            }
    };
    auto build_write = [&](int c) {
        uint32_t d[4][4];
#pragma unroll
        for (int j = 0; j < 4; j++)
#pragma unroll
            for (int u = 0; u < 4; u++) {
                d[j][u] = __builtin_amdgcn_alignbit(b_hi[j][u], b_lo[j][u], bt_sh[u]) & bt_mask[u];
            }
        uint4* tb = reinterpret_cast<uint4*>(T + (c & 1) * TSZ + bt_dst);
        // sums over subsets of rows {0, 1}, then entries v and v + 8 (v < 8)
        // written as soon as they are formed
        uint32_t a[4][4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            a[0][u] = 0;
            a[1][u] = d[0][u];
            a[2][u] = d[1][u];
            a[3][u] = d[0][u] + d[1][u];
        }
#pragma unroll
        for (int v = 0; v < 8; v++) {
            uint32_t sv[4];
#pragma unroll
            for (int u = 0; u < 4; u++) sv[u] = v < 4 ? a[v][u] : a[v - 4][u] + d[2][u];
            if (v > 0) tb[v * SQ] = make_uint4(sv[0], sv[1], sv[2], sv[3]);
            tb[(v + 8) * SQ] = make_uint4(sv[0] + d[3][0], sv[1] + d[3][1], sv[2] + d[3][2], sv[3] + d[3][3]);
        }
    };

    // prologue: chunks 0 and 1 staged, chunk 2 in registers, tables of chunk 0
    load_R(0);
    load_L(0);
    stage_R(0);
    stage_L(0);
    if (1 < nchunks) {
        load_R(1);
        load_L(1);
        stage_R(1);
        stage_L(1);
    }
    if (2 < nchunks) {
        load_R(2);
        load_L(2);
    }
    __syncthreads();
    if (bt_task) {
        build_read(0);
        build_write(0);
    }
    __syncthreads();

    int ls_c = 0, ls_c2 = 2;  // c mod 3, (c + 2) mod 3
    for (int c = 0; c < nchunks; c++) {
        const bool do_build = bt_task && c + 1 < nchunks;
        if (do_build) build_read(c + 1);
        if (c + 2 < nchunks) {
            stage_R(c + 2);
            stage_L(ls_c2);
        }
        if (c + 3 < nchunks) {
            load_R(c + 3);
            load_L(c + 3);
        }
        if (do_build) build_write(c + 1);
        // lookups: step s = (row-iteration s / CG, group s % CG)
        const uint32_t* Lc = Ls + ls_c * TR;
        const uint32_t* Tc = T + (c & 1) * TSZ;
        uint32_t Lw[RPL];
#pragma unroll
        for (int i = 0; i < RPL; i++) Lw[i] = Lc[(wave * RPL + i) * RPW + rsub];
        uint4 buf[PD + 1][NQ];
        auto issue = [&](int s, uint4* b) {
            const int i = s / CG, grp = s % CG;
            const uint32_t idx = __builtin_amdgcn_ubfe(Lw[i], 4 * grp, 4);
            const uint4* t = reinterpret_cast<const uint4*>(Tc + (grp * 16 + idx) * st) + lq;
#pragma unroll
            for (int q = 0; q < NQ; q++) b[q] = t[q * LPR];
        };
#pragma unroll
        for (int s = 0; s < PD; s++) issue(s, buf[s]);
#pragma unroll
        for (int s = 0; s < NSTEP; s++) {
            if (s + PD < NSTEP) issue(s + PD, buf[(s + PD) % (PD + 1)]);
            const int i = s / CG;
            const uint4* b = buf[s % (PD + 1)];
#pragma unroll
            for (int q = 0; q < NQ; q++) {
                acc[i][4 * q + 0] = (uint64_t)b[q].x * kc.one + acc[i][4 * q + 0];
                acc[i][4 * q + 1] = (uint64_t)b[q].y * kc.one + acc[i][4 * q + 1];
                acc[i][4 * q + 2] = (uint64_t)b[q].z * kc.one + acc[i][4 * q + 2];
                acc[i][4 * q + 3] = (uint64_t)b[q].w * kc.one + acc[i][4 * q + 3];
            }
        }
        ls_c = ls_c == 2 ? 0 : ls_c + 1;
        ls_c2 = ls_c2 == 2 ? 0 : ls_c2 + 1;
        __syncthreads();
    }

    // epilogue in passes of PI row-iterations: stage the digit sums in LDS,
    // then one thread per (row, element) finishes it
    // (the pass loop stays rolled; the accumulators, which need compile-time
    // indices, are staged under a uniform branch per pass)
    uint64_t* E = reinterpret_cast<uint64_t*>(lds);
    constexpr int NPASS = (RPL + PI - 1) / PI;
    for (int p = 0; p < NPASS; p++) {
        if (p > 0) __syncthreads();
#pragma unroll
        for (int pp = 0; pp < NPASS; pp++) {
            if (pp != p) continue;
#pragma unroll
            for (int ii = 0; ii < PI; ii++) {
                const int i = pp * PI + ii;
                if (i < RPL) {
                    const int pr = (wave * PI + ii) * RPW + rsub;
#pragma unroll
                    for (int q = 0; q < NQ; q++)
#pragma unroll
                        for (int c4 = 0; c4 < 4; c4++) E[pr * st + 4 * (lq + LPR * q) + c4] = acc[i][4 * q + c4];
                }
            }
        }
        __syncthreads();
        for (int tk = tid; tk < PASS_ROWS * g.n1; tk += THREADS) {
            const int pr = tk / g.n1, e = tk % g.n1;
            const int wv = pr / (PI * RPW), ii = (pr / RPW) % PI, rs = pr % RPW;
            const int i = p * PI + ii;
            if (i >= RPL) continue;
            const int row = row_base + (wv * RPL + i) * RPW + rs;
            if (row >= g.nct) continue;
            finish_element(bufs, g, it, E + pr * st + e * nd, nd, Lp, Rp, row, e, dst_shift);
        }
    }
}

// ---------------------------------------------------------------------------
// The product on the matrix cores.  P = BitDecomp(L) R is a dense integer
// matrix product: an Nct x Nct matrix of bits times the Nct x N matrix of the
// bytes of R (N = 4 W bytes per row), whose column sums S[r][b] (byte b of
// row r) give P = sum_b S[r][b] 2^(8 b) per element.  v_mfma_i32_32x32x32_i8
// multiplies signed bytes exactly into 32-bit sums; the bytes u of R enter as
// u - 128 (u xor 0x80), and 128 popcount(row r of L) is added back in the
// epilogue.  Column sums stay below Nct 255 < 2^31.
//
// Workgroup: RG x CG waves; a wave owns 64 rows (two 32-row fragments) of
// the tile and CF 32-column fragments, so a tile is TM = 64 RG rows by up to
// 32 CG CF byte columns.  R is walked in chunks of 64 rows: each chunk is
// loaded as 4x4 byte blocks, transposed in registers (v_perm) and stored in
// LDS column by column (64 bytes of a column contiguous, so that a lane's
// 16 bytes of a B fragment are one ds_read_b128), double-buffered with one
// barrier per chunk.  A lane's 16 bits of L for a fragment become 16 bytes of
// 0/1 by a multiply that spreads 4 bits to the 4 bytes of a word.
//
// Epilogue: the accumulators go to LDS in slabs of 32 rows, and one thread
// per (row, element) forms 32-bit limbs from 4 column sums at a time and
// feeds up to four outputs a L + b R + c P + g G + e E, one signed carry
// chain each, as in the lookup kernel.
typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef int32_t i32x16 __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) u32x4 gu32x4;  // 16 bytes of a ciphertext, global

constexpr int kMfmaChunk = 128;                 // rows of R per chunk
constexpr int kMfmaPitch = kMfmaChunk;          // LDS bytes per staged column

// A staged column n (or row of bits of L) keeps its 8 units of 16 bytes in
// the order unit ^ swz(n).  swz takes distinct values on the even and on the
// odd n of any 16 aligned consecutive n, so that the 16 lanes of a
// ds_read_b128 phase (16 consecutive columns) hit distinct 4-bank groups of
// the 64 banks, and distinct values on n = 16 w + k for w = 0..7, so that
// the dword stores of a staging wave spread over all banks (two lanes each).
__device__ __forceinline__ int mfma_swz(int n) { return ((n >> 1) + (n >> 4)) & 7; }
// The 16-byte units of a column of a 64-row chunk (4 units): unit ^
// swz64(n), so that 16 lanes reading one unit of 16 consecutive columns hit
// distinct 4-bank groups.
__device__ __forceinline__ int swz64(int n) { return (n >> 2) & 3; }
template <int KC>
__device__ __forceinline__ int chunk_swz(int n) { return KC == 128 ? mfma_swz(n) : swz64(n); }

// Epilogue layout of the column sums: a row of NF fragments takes SP =
// 32 NF + 8 words (rows 4 apart, as the two halves of a fragment's lanes
// store them, then fall on disjoint halves of the 64 banks).  Word w of a
// row (its four byte sums, 16 bytes) sits in unit mfma_sum_unit(w): the
// units of a quad stay in the quad, permuted so that 16 lanes reading word u
// of 16 consecutive quads hit distinct 4-bank groups.
__host__ __device__ constexpr int mfma_sum_pitch(int nf) { return 32 * nf + 8; }
__device__ __forceinline__ int mfma_sum_unit(int w) { return w ^ ((w >> 4) & 3); }
// LDS bytes of one operand's words in a pass of 32 rows (whole KB: the
// loads straight into LDS fill 1 KB per wave instruction).
__host__ __device__ constexpr int mfma_op_bytes(int W) { return (128 * W + 1023) / 1024 * 1024; }
// LDS bytes of the epilogue: a slab of 32 rows of column sums, one carry
// per quad of words and output, and two passes' words of L, R and up to
// kMaxE extra operands.
__host__ __device__ constexpr int mfma_epi_bytes(int nf, int W)
{
    return 32 * mfma_sum_pitch(nf) * 4 + kMaxOut * 8 * W * 4 + 2 * (2 + kMaxE) * mfma_op_bytes(W);
}
// LDS bytes of the 256-thread kernel (k_product_mfma2): its main loop's
// chunks in flight of 2 x 2 CF 1 KB units of R and of 128 rows' 64 bits of
// L, and its epilogue's passes of 16 pm rows (qp quads of words): column
// sums and two passes' quads of L, R and up to kMaxE extra operands.
// Chunks of R in flight: as many as about 78 KB hold, at most 6 (a chunk
// keeps the matrix cores busy for a short time, so the requests must be
// issued several chunks ahead to cover the memory latency).
__host__ __device__ constexpr int mfma2_depth(int cf)
{
    return (78 * 1024) / (4 * cf * 1024 + 1024) < 6 ? (78 * 1024) / (4 * cf * 1024 + 1024) : 6;
}
__host__ __device__ constexpr int mfma2_main_bytes(int cf) { return mfma2_depth(cf) * (4 * cf * 1024 + 128 * 8); }
__host__ __device__ constexpr int mfma2_epi_bytes(int cf, int qp, int pm)
{
    return 16 * pm * mfma_sum_pitch(2 * cf) * 4 + 2 * (2 + kMaxE) * ((16 * qp + 1023) / 1024 * 1024);
}

// r[i] holds bytes (i, 0..3) of a 4x4 byte block; c[j] gets bytes (0..3, j)
__device__ __forceinline__ void transpose4x4(const uint32_t r[4], uint32_t c[4])
{
    const uint32_t lo01 = __builtin_amdgcn_perm(r[1], r[0], 0x05010400u);
    const uint32_t hi01 = __builtin_amdgcn_perm(r[1], r[0], 0x07030602u);
    const uint32_t lo23 = __builtin_amdgcn_perm(r[3], r[2], 0x05010400u);
    const uint32_t hi23 = __builtin_amdgcn_perm(r[3], r[2], 0x07030602u);
    c[0] = __builtin_amdgcn_perm(lo23, lo01, 0x05040100u);
    c[1] = __builtin_amdgcn_perm(lo23, lo01, 0x07060302u);
    c[2] = __builtin_amdgcn_perm(hi23, hi01, 0x05040100u);
    c[3] = __builtin_amdgcn_perm(hi23, hi01, 0x07060302u);
}

// Direct loads from global memory into LDS: every lane of the wave loads
// BYTES bytes from its own address, and lane i's bytes land at
// lds_base + BYTES * i (lds_base the same for the whole wave).  They count
// as vector-memory operations of the wave (vmcnt) and write LDS without
// passing through registers.
typedef __attribute__((address_space(3))) void lds_void;
template <int BYTES>
__device__ __forceinline__ void load_to_lds(const void* src, void* lds_base)
{
    static_assert(BYTES == 4 || BYTES == 16, "4- or 16-byte lanes");
    if constexpr (BYTES == 16) __builtin_amdgcn_global_load_lds(src, (lds_void*)lds_base, 16, 0, 0);
    else __builtin_amdgcn_global_load_lds(src, (lds_void*)lds_base, 4, 0, 0);
}

// Wait until at most N vector-memory operations of this wave are
// outstanding (s_waitcnt: vmcnt in bits 3:0 and 15:14, expcnt (6:4) and
// lgkmcnt (11:8) left at their maxima, i.e. not waited for).
template <int N>
__device__ __forceinline__ void wait_vmcnt()
{
    static_assert(N >= 0 && N < 64, "vmcnt range");
    __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// Wait until at most n * STEP (n <= MAX / STEP, run-time) vector-memory
// operations of this wave are outstanding: the counts are immediates, so
// one s_waitcnt per possible n.
template <int MAX, int STEP>
__device__ __forceinline__ void wait_vmcnt_upto(int n)
{
    if constexpr (MAX >= STEP) {
        if (n >= MAX / STEP) {
            wait_vmcnt<MAX>();
            return;
        }
        wait_vmcnt_upto<MAX - STEP, STEP>(n);
    } else {
        wait_vmcnt<0>();
    }
}

// Workgroup barrier without the memory fence of __syncthreads (which would
// wait for every outstanding load, prefetches included); the empty asm
// statements keep the compiler from moving memory accesses across it.
__device__ __forceinline__ void barrier_only()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// Workgroup barrier after this wave's LDS accesses (lgkmcnt 0) but without
// waiting for its global loads or stores.
__device__ __forceinline__ void lds_barrier()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt(15 | (3 << 14) | (7 << 4));  // vmcnt and expcnt at their maxima, lgkmcnt 0
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
}

// 16 bits to 16 bytes of 0/1 (byte p = bit p): x * 0x204081 places bits
// 0..3 of a nibble at bits 0, 8, 16, 24 without carries.
__device__ __forceinline__ i32x4 spread_bits(uint32_t u)
{
    i32x4 a;
    a[0] = (int32_t)(((u & 15u) * 0x204081u) & 0x01010101u);
    a[1] = (int32_t)((((u >> 4) & 15u) * 0x204081u) & 0x01010101u);
    a[2] = (int32_t)((((u >> 8) & 15u) * 0x204081u) & 0x01010101u);
    a[3] = (int32_t)((((u >> 12) & 15u) * 0x204081u) & 0x01010101u);
    return a;
}

// Right operands of a launch's items into the matrix-core kernel's chunk
// layout, once per item instead of once per row tile: workgroup (y, c)
// loads chunk c (128 rows) of item y's R with 16-byte row loads (8 lanes per
// 128 contiguous bytes), transposes 4x4 byte blocks in registers (v_perm),
// stores them column by column into LDS (bytes xor 0x80, 16-byte units of a
// column XOR-swizzled) and copies the chunk out with 16-byte stores.
// KC = 128 for the 512-thread kernel's chunks; KC = 64 for the 256-thread
// kernel's, whose columns keep their 4 units in the order unit ^ swz64(n).
constexpr int kRtransThreads = 256;
template <int KC>
__global__ void __launch_bounds__(kRtransThreads) k_rtrans(const ProdSeg* __restrict__ segs, int nseg, ProdSeg seg0,
                                                           ProdItem one)
{
    constexpr int THREADS = kRtransThreads;
    constexpr int BP = KC;                                       // bytes per column of a chunk
    constexpr int JG = KC / 32;                                  // groups of 8 row quads
    constexpr int SPT = (KC / 4 * 24 + THREADS - 1) / THREADS;  // KC/4 row quads x up to 24 word quads (W <= 96)
    extern __shared__ uint32_t lds[];
    uint8_t* Ts = reinterpret_cast<uint8_t*>(lds);
    const uint32_t y = blockIdx.x;  // item within the launch
    ProdSeg sg = seg0;
    if (nseg > 1) sg = segs[find_segment(segs, nseg, y, [](const ProdSeg& q) { return q.first; })];
    const Geo g = sg.geo;
    const int c = blockIdx.y, W = g.W, nct = g.nct;
    if (KC * c >= nct) return;  // chunks past this item's rows
    const uint32_t yl = y - sg.first;
    const ProdItem it = sg.items ? load_global(sg.items + yl) : one;
    const gword* src = ctp(sg.bufs, it.R) + (size_t)(KC * c) * W;
    const int NF = (4 * W + 31) / 32, bsz = NF * 32 * BP;
    const int rows_c = nct - KC * c < KC ? nct - KC * c : KC;
    const bool quads = (W & 3) == 0;
    const int tid = threadIdx.x;
    // block i of this thread: rows 4 jq .. 4 jq + 3, words 4 wq .. 4 wq + 3;
    // within a wave 8 consecutive wq (128 bytes of a row) times 8 consecutive jq
    uint32_t rs[SPT][4][4];
#pragma unroll
    for (int i = 0; i < SPT; i++) {
        const int t = tid + i * THREADS, r = t >> 6;
        const int jq = ((t >> 3) & 7) + 8 * (r % JG), wq = (t & 7) + 8 * (r / JG);
        const bool ok = 4 * wq < W && 4 * jq < rows_c;
#pragma unroll
        for (int rr = 0; rr < 4; rr++) {
            const gword* p = src + (size_t)(4 * jq + rr) * W + 4 * wq;
            if (ok && quads) {
                const u32x4 x = *reinterpret_cast<const gu32x4*>(p);
                rs[i][rr][0] = x[0], rs[i][rr][1] = x[1], rs[i][rr][2] = x[2], rs[i][rr][3] = x[3];
            } else {
#pragma unroll
                for (int u = 0; u < 4; u++) rs[i][rr][u] = ok && 4 * wq + u < W ? p[u] : 0u;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < SPT; i++) {
        const int t = tid + i * THREADS, r = t >> 6;
        const int jq = ((t >> 3) & 7) + 8 * (r % JG), wq = (t & 7) + 8 * (r / JG);
        if (4 * wq < W && 4 * jq < rows_c) {
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const uint32_t blk[4] = {rs[i][0][u], rs[i][1][u], rs[i][2][u], rs[i][3][u]};
                uint32_t col[4];
                transpose4x4(blk, col);
#pragma unroll
                for (int cc = 0; cc < 4; cc++) {
                    const int n = 16 * wq + 4 * u + cc;
                    // columns past the row (a partial last unit) are never read
                    *reinterpret_cast<uint32_t*>(Ts + n * BP + 16 * ((jq >> 2) ^ chunk_swz<KC>(n)) + 4 * (jq & 3)) =
                        col[cc] ^ 0x80808080u;
                }
            }
        }
    }
    __syncthreads();
    uint8_t* dst = sg.rt + (size_t)yl * rt_item_bytes(g) + (size_t)c * bsz;
    for (int u = tid; 16 * u < bsz; u += THREADS)
        *(gu32x4*)(dst + 16 * u) = *reinterpret_cast<const u32x4*>(Ts + 16 * u);
}

// The work of one workgroup (virtual block v of the launch's flat order),
// shared by the launch per level and the whole-plan persistent kernel.
template <int RG, int CG, int CF, bool PRE>
__device__ __forceinline__ void product_mfma_block(const ProdSeg* __restrict__ segs, int nseg, const ProdSeg& seg0,
                                                   const ProdItem& one, int lds_bytes, uint32_t v)
{
    constexpr int THREADS = RG * CG * 64;
    constexpr int TM = 64 * RG;
    constexpr int KC = kMfmaChunk;
    constexpr int BP = kMfmaPitch;
    // staging of R per thread: PRE, 16-byte units of a chunk already in chunk
    // layout; else 4-row x 16-byte blocks transposed here (W <= 8 CG CF)
    constexpr int SPT_C = (32 * CG * CF * KC / 16 + THREADS - 1) / THREADS;
    constexpr int SPT_T = (KC / 4 * 2 * CG * CF + THREADS - 1) / THREADS;
    constexpr int SPT = PRE ? SPT_C : SPT_T;
    constexpr int APT = (TM * (KC / 32) + THREADS - 1) / THREADS;        // staged words of L per thread
    constexpr int EPT = (8 * 8 * CG * CF + THREADS - 1) / THREADS;  // epilogue quads of words per thread and pass
    constexpr int NP = SPT < KC / 32 ? SPT : KC / 32;                     // staging parts per chunk

    extern __shared__ uint32_t lds[];
    ProdSeg sg = seg0;  // (a select between the two structs would copy both into vector registers)
    if (nseg > 1) sg = segs[find_segment(segs, nseg, v, [](const ProdSeg& q) { return q.first_block; })];
    const Geo g = sg.geo;
    const uint32_t tiles = ((uint32_t)g.nct + TM - 1) / TM;
    const uint32_t local = v - sg.first_block;
    const uint32_t yl = local / tiles;
    const int row_base = (int)(local % tiles) * TM;
    const Bufs bufs = sg.bufs;
    const ProdItem it = sg.items ? load_global(sg.items + yl) : one;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wr = wave % RG, wc = wave / RG;
    const int half = lane >> 5;
    const int W = g.W, nct = g.nct;
    const int NF = (4 * W + 31) / 32;
    const int bsz = NF * 32 * BP;  // bytes per staged chunk of R
    const int nchunks = (nct + KC - 1) / KC;
    const bool quads = (W & 3) == 0;  // rows are whole 16-byte units
    const gword* Lp = ctp(bufs, it.L);
    const gword* Rp = ctp(bufs, it.R);

    // epilogue: a slab of 32 rows of column sums (SP words per row), a carry
    // per quad of words and output, the operands of two passes (segments of
    // one launch may differ in width)
    const int SP = mfma_sum_pitch(NF);
    const int main_bytes = PRE ? 3 * bsz + 3 * TM * 16 : 2 * bsz + 2 * TM * KC;
    const int e_bytes = mfma_epi_bytes(NF, W);
    uint8_t* Bs = reinterpret_cast<uint8_t*>(lds);  // 2 chunks of R, column by column
    uint8_t* As = Bs + 2 * bsz;                     // 2 chunks of bits of L as 0/1 bytes, KC bytes per row
    int32_t* Pc = reinterpret_cast<int32_t*>(Bs + (main_bytes > e_bytes ? main_bytes : e_bytes));  // popcount per row

    // Staging of R.  PRE: R comes already in chunk layout (k_rtrans), and
    // staging chunk c copies its bsz bytes, 16 per thread and unit, into
    // LDS.  Else each thread transposes 4x4 byte blocks of the raw rows here.
    // Loads and staging go in NP parts (part p: the units or blocks i with
    // i % NP == p); part p of chunk c + 1 is staged, and its registers
    // refilled with chunk c + 2, after a matrix step of chunk c, so that
    // every load has a whole chunk to arrive.
    const uint8_t* rtp = PRE ? sg.rt + (size_t)yl * rt_item_bytes(g) : nullptr;
    u32x4 rc[SPT_C];
    auto load_R_c = [&](int c, int part) {
        const uint8_t* src = rtp + (size_t)c * bsz;
#pragma unroll
        for (int i = 0; i < SPT_C; i++) {
            if (part >= 0 && i % NP != part) continue;
            const int u = tid + i * THREADS;
            if (16 * u < bsz) rc[i] = *(const gu32x4*)(src + 16 * u);
        }
    };
    // staging block i of this thread: rows 4 jq .. 4 jq + 3 of the chunk,
    // words 4 wq .. 4 wq + 3 (one 16-byte load per row).  Within a wave 8
    // consecutive wq (128 bytes of a row) times 8 consecutive jq.
    uint32_t rs[SPT_T][4][4];
    auto block_of = [&](int i, int& jq, int& wq) {
        const int t = tid + i * THREADS, r = t >> 6;
        jq = ((t >> 3) & 7) + 8 * (r & 3);
        wq = (t & 7) + 8 * (r >> 2);
    };
    // loads and staging go in NP parts (part p: the blocks i with i % NP ==
    // p); part p of chunk c + 1 is staged, and its registers refilled with
    // chunk c + 2, after matrix step kPartStep[p] of chunk c, so that every
    // load has a whole chunk to arrive
    auto load_R_t = [&](int c, int part) {
        const int rows_c = nct - KC * c < KC ? nct - KC * c : KC;
        const gword* src = Rp + (size_t)(KC * c) * W;
#pragma unroll
        for (int i = 0; i < SPT_T; i++) {
            if (part >= 0 && i % NP != part) continue;
            int jq, wq;
            block_of(i, jq, wq);
            const bool ok = 4 * wq < W && 4 * jq < rows_c;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const gword* p = src + (size_t)(4 * jq + r) * W + 4 * wq;
                if (ok && quads) {
                    const u32x4 x = *reinterpret_cast<const gu32x4*>(p);
                    rs[i][r][0] = x[0], rs[i][r][1] = x[1], rs[i][r][2] = x[2], rs[i][r][3] = x[3];
                } else {
#pragma unroll
                    for (int u = 0; u < 4; u++) rs[i][r][u] = ok && 4 * wq + u < W ? p[u] : 0u;
                }
            }
        }
    };
    uint32_t as[APT];
    auto load_R = [&](int c, int part) {
        if constexpr (PRE) load_R_c(c, part);
        else load_R_t(c, part);
    };
    // words of L: row a / (KC/32) of the tile, word a % (KC/32) of the chunk
    auto load_L = [&](int c) {
        const int rows_c = nct - KC * c < KC ? nct - KC * c : KC;
#pragma unroll
        for (int i = 0; i < APT; i++) {
            const int a = tid + i * THREADS, r = a / (KC / 32), wq = a % (KC / 32);
            const bool ok = r < TM && row_base + r < nct && 32 * wq < rows_c;
            as[i] = ok ? Lp[(size_t)(row_base + r) * W + (KC / 32) * c + wq] : 0u;
        }
    };
    auto stage_R_c = [&](int c, int part) {
        uint8_t* dst = Bs + (c & 1) * bsz;
#pragma unroll
        for (int i = 0; i < SPT_C; i++) {
            if (part >= 0 && i % NP != part) continue;
            const int u = tid + i * THREADS;
            if (16 * u < bsz) *reinterpret_cast<u32x4*>(dst + 16 * u) = rc[i];
        }
    };
    auto stage_R_t = [&](int c, int part) {
        const int rows_c = nct - KC * c < KC ? nct - KC * c : KC;
        uint8_t* dst = Bs + (c & 1) * bsz;
#pragma unroll
        for (int i = 0; i < SPT_T; i++) {
            if (part >= 0 && i % NP != part) continue;
            int jq, wq;
            block_of(i, jq, wq);
            if (4 * wq < W && 4 * jq < rows_c) {
#pragma unroll
                for (int u = 0; u < 4; u++) {
                    const uint32_t blk[4] = {rs[i][0][u], rs[i][1][u], rs[i][2][u], rs[i][3][u]};
                    uint32_t col[4];
                    transpose4x4(blk, col);
#pragma unroll
                    for (int cc = 0; cc < 4; cc++) {
                        const int n = 16 * wq + 4 * u + cc;
                        // columns past the row (a partial last unit) are never read
                        *reinterpret_cast<uint32_t*>(dst + n * BP + 16 * ((jq >> 2) ^ mfma_swz(n)) + 4 * (jq & 3)) =
                            col[cc] ^ 0x80808080u;
                    }
                }
            }
        }
    };
    auto stage_R = [&](int c, int part) {
        if constexpr (PRE) stage_R_c(c, part);
        else stage_R_t(c, part);
    };
    // the chunk's bits of L as bytes: word s of row r gives units 2 s and
    // 2 s + 1 (its two halves) of the row, XOR-swizzled by row like the
    // columns of R; the staging thread also counts the bits
    uint32_t pcs[APT];
#pragma unroll
    for (int i = 0; i < APT; i++) pcs[i] = 0u;
    auto stage_L = [&](int c) {
        uint8_t* ad = As + (c & 1) * TM * KC;
#pragma unroll
        for (int i = 0; i < APT; i++) {
            const int a = tid + i * THREADS, r = a / (KC / 32), wq = a % (KC / 32);
            if (a < TM * (KC / 32)) {
                pcs[i] += __builtin_popcount(as[i]);
#pragma unroll
                for (int h = 0; h < 2; h++)
                    *reinterpret_cast<i32x4*>(ad + r * KC + 16 * ((2 * wq + h) ^ mfma_swz(r))) =
                        spread_bits(as[i] >> (16 * h));
            }
        }
    };

    i32x16 acc[2][CF];
#pragma unroll
    for (int f = 0; f < 2; f++)
#pragma unroll
        for (int q = 0; q < CF; q++)
#pragma unroll
            for (int r = 0; r < 16; r++) acc[f][q][r] = 0;
    // B fragments of this lane: column 32 fi + lane % 32 (fragments past the
    // row read the last one; their sums are never used), units 2 s + half
    int bcol[CF], bswz[CF];
#pragma unroll
    for (int q = 0; q < CF; q++) {
        const int fi = wc * CF + q < NF ? wc * CF + q : NF - 1;
        const int n = 32 * fi + (lane & 31);
        bcol[q] = n * BP;
        bswz[q] = mfma_swz(n);
    }

    if constexpr (PRE) {
        // Chunks of R (already in chunk layout) and of the bits of L go from
        // global memory straight into LDS, three chunks deep: chunk c + 2 is
        // requested while chunk c is multiplied, and each wave waits only for
        // its own requests of chunk c before the barrier that opens it.
        // Every wave issues DR + DL requests per chunk (units past the chunk
        // repeat its last unit, rows past the product its last row, words
        // past the row its last word: all in bounds), so that the wait is a
        // constant count.  Bits of L past the product (the last chunk's
        // missing rows of R) are cleared before they are spread.
        constexpr int NW = RG * CG;
        constexpr int DR = (4 * CG * CF + NW - 1) / NW;  // 1 KB units of R per wave per chunk
        constexpr int DL = 4 / CG;                        // 256-byte row groups of L per wave per chunk
        static_assert(4 % CG == 0, "row groups of L split evenly over the waves");
        const int units = 4 * NF;
        uint8_t* Rb = reinterpret_cast<uint8_t*>(lds);  // 3 chunks of R
        uint8_t* Lb = Rb + 3 * bsz;                      // 3 chunks of L: 16 bytes (128 bits) per tile row
        const uint8_t* rsrc = sg.rt + (size_t)yl * rt_item_bytes(g);
        const uint8_t* Lbytes = (const uint8_t*)Lp;
        auto request = [&](int c) {
            const int buf = c % 3;
            const uint8_t* src = rsrc + (size_t)c * bsz;
            uint8_t* dst = Rb + buf * bsz;
#pragma unroll
            for (int t = 0; t < DR; t++) {
                const int u = wave + NW * t < units ? wave + NW * t : units - 1;
                load_to_lds<16>(src + (size_t)u * 1024 + lane * 16, dst + u * 1024);
            }
#pragma unroll
            for (int t = 0; t < DL; t++) {
                const int j = wave * DL + t;  // rows 16 j .. 16 j + 15 of the tile
                int row = row_base + 16 * j + (lane >> 2);
                row = row < nct ? row : nct - 1;
                int word = 4 * c + (lane & 3);
                word = word < W ? word : W - 1;
                load_to_lds<4>(Lbytes + ((size_t)row * W + word) * 4, Lb + buf * TM * 16 + j * 256);
            }
        };
        // this lane's rows of A: 64 wr + 32 f + lane % 32, 16 bytes each per chunk
        int arow16[2];
#pragma unroll
        for (int f = 0; f < 2; f++) arow16[f] = (64 * wr + 32 * f + (lane & 31)) * 16;
        uint32_t pc[2] = {0u, 0u};

        request(0);
        if (1 < nchunks) request(1);
        for (int c = 0; c < nchunks; c++) {
            if (c + 1 < nchunks) wait_vmcnt<DR + DL>();
            else wait_vmcnt<0>();
            barrier_only();
            if (c + 2 < nchunks) request(c + 2);
            const uint8_t* Bc = Rb + (c % 3) * bsz;
            const uint8_t* Lc = Lb + (c % 3) * TM * 16;
            const int rows_c = nct - KC * c < KC ? nct - KC * c : KC;
            u32x4 lw[2];
#pragma unroll
            for (int f = 0; f < 2; f++) lw[f] = *reinterpret_cast<const u32x4*>(Lc + arow16[f]);
            i32x4 Bx[2][CF];
#pragma unroll
            for (int q = 0; q < CF; q++)
                Bx[0][q] = *reinterpret_cast<const i32x4*>(Bc + bcol[q] + 16 * (half ^ bswz[q]));
#pragma unroll
            for (int st = 0; st < KC / 32; st++) {
                if (st + 1 < KC / 32) {
#pragma unroll
                    for (int q = 0; q < CF; q++)
                        Bx[(st + 1) & 1][q] =
                            *reinterpret_cast<const i32x4*>(Bc + bcol[q] + 16 * ((2 * (st + 1) + half) ^ bswz[q]));
                }
                i32x4 Af[2];
#pragma unroll
                for (int f = 0; f < 2; f++) {
                    const uint32_t w = 32 * st < rows_c ? lw[f][st] : 0u;
                    const uint32_t b16 = (w >> (16 * half)) & 0xFFFFu;
                    pc[f] += __builtin_popcount(b16);
                    Af[f] = spread_bits(b16);
                }
#pragma unroll
                for (int q = 0; q < CF; q++) {
                    acc[0][q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Af[0], Bx[st & 1][q], acc[0][q], 0, 0, 0);
                    acc[1][q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Af[1], Bx[st & 1][q], acc[1][q], 0, 0, 0);
                }
            }
        }
        // every wave done with the chunk buffers before the epilogue reuses
        // them; the popcount of a row is the sum over its two half-lanes
        __syncthreads();
#pragma unroll
        for (int f = 0; f < 2; f++) {
            const uint32_t tot = pc[f] + __shfl_xor(pc[f], 32);
            if (wc == 0 && half == 0) Pc[64 * wr + 32 * f + (lane & 31)] = (int32_t)tot;
        }
    } else {
    // this lane's rows of A: 64 wr + 32 f + lane % 32
        int arow[2];
    #pragma unroll
        for (int f = 0; f < 2; f++) {
            const int r = 64 * wr + 32 * f + (lane & 31);
            arow[f] = r * KC;
            (void)r;
        }
        int aswz[2];
    #pragma unroll
        for (int f = 0; f < 2; f++) aswz[f] = mfma_swz(64 * wr + 32 * f + (lane & 31));
    
        load_R(0, -1);
        load_L(0);
        stage_R(0, -1);
        stage_L(0);
        if (1 < nchunks) {
            load_R(1, -1);
            load_L(1);
        }
        __syncthreads();
        for (int c = 0; c < nchunks; c++) {
            const uint8_t* Bc = Bs + (c & 1) * bsz;
            const uint8_t* Ac = As + (c & 1) * TM * KC;
            const int rows_c = nct - KC * c < KC ? nct - KC * c : KC;
            const bool next = c + 1 < nchunks, next2 = c + 2 < nchunks;
            // fragments of step s + 1 are read from LDS before the products of step s
            i32x4 B[CF], A[2];
            auto read_frags = [&](int s) {
    #pragma unroll
                for (int q = 0; q < CF; q++)
                    B[q] = *reinterpret_cast<const i32x4*>(Bc + bcol[q] + 16 * ((2 * s + half) ^ bswz[q]));
    #pragma unroll
                for (int f = 0; f < 2; f++)
                    A[f] = *reinterpret_cast<const i32x4*>(Ac + arow[f] + 16 * ((2 * s + half) ^ aswz[f]));
            };
            read_frags(0);
    #pragma unroll
            for (int s = 0; s < KC / 32; s++) {
                if (32 * s < rows_c) {
                    i32x4 Bq[CF], Af[2];
    #pragma unroll
                    for (int q = 0; q < CF; q++) Bq[q] = B[q];
                    Af[0] = A[0], Af[1] = A[1];
                    if (s + 1 < KC / 32 && 32 * (s + 1) < rows_c) read_frags(s + 1);
    #pragma unroll
                    for (int q = 0; q < CF; q++) {
                        acc[0][q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Af[0], Bq[q], acc[0][q], 0, 0, 0);
                        acc[1][q] = __builtin_amdgcn_mfma_i32_32x32x32_i8(Af[1], Bq[q], acc[1][q], 0, 0, 0);
                    }
                }
                // staging parts that fall after this step
    #pragma unroll
                for (int p = 0; p < NP; p++) {
                    if ((p + 1) * (KC / 32) / NP - 1 != s) continue;
                    if (next) stage_R(c + 1, p);
                    if (next2) load_R(c + 2, p);
                }
            }
            if (next) stage_L(c + 1);
            if (next2) load_L(c + 2);
            __syncthreads();
        }
    
        // popcount of each row: the sum over the KC/32 staging threads of the
        // row (consecutive lanes)
    #pragma unroll
        for (int i = 0; i < APT; i++) {
            pcs[i] += __shfl_xor(pcs[i], 1);
            pcs[i] += __shfl_xor(pcs[i], 2);
            const int a = tid + i * THREADS;
            if (a < TM * (KC / 32) && (a & 3) == 0) Pc[a >> 2] = (int32_t)pcs[i];
        }
    }

    // Epilogue, in passes of one slab of 32 rows (slab 2 wr + f is fragment f
    // of row group wr; Nct is a multiple of 32, so every pass is whole).  The
    // 32 W words of a pass (row-major, flat) go to the threads as quads of 4
    // consecutive words.  The pass's words of L, R and of the item's extra
    // operands come from global memory straight into LDS, one pass ahead.
    //  1. The waves holding the pass's rows store their column sums in S.
    //  2. Per quad and output, each word's limb of a L + b R + c P + g G + e E
    //     (P's limb from its four byte column sums) is rippled through the
    //     quad from carry 0, restarting at the first limb of every element;
    //     the carry out of the quad goes to Cq (0 where the quad ends an
    //     element).  The limb is A + 2^16 B with A and B sums of small
    //     coefficients times 16-bit halves and byte sums (24-bit products).
    //  3. Each quad takes the carry out of the quad before it (unless it
    //     starts an element) and ripples it through its words; repeated while
    //     any carry leaves a quad.  Carries never cross an element: the sums
    //     are mod 2^k per element.
    //  4. The outputs are written with 16-byte stores.
    // The item's coefficients and operands are the same for the whole
    // workgroup.
    const int nout = __builtin_amdgcn_readfirstlane(it.nout);
    int cLo[kMaxOut], cRo[kMaxOut], cPo[kMaxOut], cGo[kMaxOut], cEo[kMaxOut], eso[kMaxOut];
    gword* Do[kMaxOut];
    // operand slots: 0 = L, 1 = R, then the distinct extra operands
    const gword* opsrc[2 + kMaxE] = {Lp, Rp};
    int32_t eref[kMaxE];
    int nops = 2;
#pragma unroll
    for (int o = 0; o < kMaxOut; o++) {
        cLo[o] = __builtin_amdgcn_readfirstlane((int)it.cL[o]);
        cRo[o] = __builtin_amdgcn_readfirstlane((int)it.cR[o]);
        cPo[o] = __builtin_amdgcn_readfirstlane((int)it.cP[o]);
        cGo[o] = __builtin_amdgcn_readfirstlane((int)it.cG[o]);
        cEo[o] = __builtin_amdgcn_readfirstlane((int)it.cE[o]);
        const int32_t er = __builtin_amdgcn_readfirstlane(it.E[o]);
        const int32_t dr = __builtin_amdgcn_readfirstlane(it.dst[o]);
        Do[o] = o < nout ? ctp(bufs, dr) : nullptr;
        eso[o] = -1;
        if (o < nout && er >= 0) {
#pragma unroll
            for (int q = 0; q < kMaxE; q++)
                if (q + 2 < nops && eref[q] == er) eso[o] = q;
            if (eso[o] < 0 && nops < 2 + kMaxE) {  // (the plan keeps at most kMaxE per item)
                eref[nops - 2] = er;
                opsrc[nops] = ctp(bufs, er);
                eso[o] = nops - 2;
                ++nops;
            }
        }
    }
    const int kw = g.kw, kb = g.k;
    const int QP = 8 * W;  // quads of a pass
    int32_t* S = reinterpret_cast<int32_t*>(lds);
    int32_t* Cq = S + 32 * SP;
    uint8_t* OPS = reinterpret_cast<uint8_t*>(Cq + kMaxOut * QP);  // 2 buffers x (2 + kMaxE) operands
    const int OPB = mfma_op_bytes(W);
    int32_t* more = Pc + TM;  // the last round in which a carry left a quad
    int round = 0;
    if (tid == 0) *more = 0;  // (read only after the barriers below)
    // the pass's words of every operand into buffer b: 16-byte units, 64
    // consecutive units per wave instruction (the last block's lanes past
    // the pass re-read its last unit and land in the block's padding)
    auto stage_ops = [&](int p0, int b) {
        const size_t pbase = (size_t)(row_base + 32 * p0) * W;
        for (int blk = __builtin_amdgcn_readfirstlane(wave); 64 * blk < QP; blk += RG * CG) {
            const int u = 64 * blk + lane < QP ? 64 * blk + lane : QP - 1;
#pragma unroll
            for (int s = 0; s < 2 + kMaxE; s++)
                if (s < nops)
                    load_to_lds<16>((const uint8_t*)(opsrc[s] + pbase + 4 * u), OPS + (b * (2 + kMaxE) + s) * OPB + 1024 * blk);
        }
    };
    stage_ops(0, 0);
    for (int p0 = 0; p0 < 2 * RG; p0++) {
        const int prow = row_base + 32 * p0;  // first row of the pass
        if (prow >= nct) break;               // (the same for every thread)
        const int b = p0 & 1;
        // this pass's operands in LDS (each wave waits for its own loads, and
        // its stores of the pass before); the pass before is done with S,
        // Cq and the other buffer
        wait_vmcnt<0>();
        lds_barrier();
        if (p0 + 1 < 2 * RG && prow + 32 < nct) stage_ops(p0 + 1, b ^ 1);
        // 1. column sums: column c of row rl at word c / 4 (16-byte units
        // permuted as mfma_sum_unit), byte c % 4
#pragma unroll
        for (int f = 0; f < 2; f++) {
            if (2 * wr + f != p0) continue;
#pragma unroll
            for (int q = 0; q < CF; q++) {
                const int fi = wc * CF + q;
                if (fi < NF) {
                    const int col = 32 * fi + (lane & 31);
                    const int cu = 4 * mfma_sum_unit(col >> 2) + (col & 3);
#pragma unroll
                    for (int r = 0; r < 16; r++) S[(8 * (r >> 2) + 4 * half + (r & 3)) * SP + cu] = acc[f][q][r];
                }
            }
        }
        lds_barrier();
        // 2. limbs of every output, rippled within the quad
        const uint8_t* ob = OPS + b * (2 + kMaxE) * OPB;
        u32x4 oq[EPT][kMaxOut];
        // per quad: bit u (0..3) = word u starts an element, bit 4 = a quad
        // of the pass, bit 5 = its last word ends an element
        int qv[EPT];
#pragma unroll
        for (int i = 0; i < EPT; i++) {
            const int j = tid + i * THREADS, fw = 4 * j;
            qv[i] = 0;
#pragma unroll
            for (int o = 0; o < kMaxOut; o++) oq[i][o] = u32x4{0u, 0u, 0u, 0u};
            if (j >= QP) continue;
            int rl = fw / W, w = fw - rl * W;
            int e = w / kw, l = w - e * kw;
            int row = prow + rl;
            int br = row / kb, tr = row - br * kb;
            int cpc = 128 * Pc[32 * p0 + rl];  // each byte sum misses 128 per set bit of the row of L
            const u32x4 lv = *reinterpret_cast<const u32x4*>(ob + 16 * j);
            const u32x4 rv = *reinterpret_cast<const u32x4*>(ob + OPB + 16 * j);
            u32x4 ev[kMaxE];
#pragma unroll
            for (int q = 0; q < kMaxE; q++)
                ev[q] = q + 2 < nops ? *reinterpret_cast<const u32x4*>(ob + (2 + q) * OPB + 16 * j)
                                     : u32x4{0u, 0u, 0u, 0u};
            int64_t cy[kMaxOut];
#pragma unroll
            for (int o = 0; o < kMaxOut; o++) cy[o] = 0;
            int qm = 1 << 4;
#pragma unroll
            for (int u = 0; u < 4; u++) {
                if (u > 0) {
                    ++w, ++l;
                    if (l == kw) l = 0, ++e;
                    if (w == W) {
                        w = 0, e = 0, l = 0, ++rl, ++row, ++tr;
                        if (tr == kb) tr = 0, ++br;
                        cpc = 128 * Pc[32 * p0 + rl];
                    }
                }
                if (l == 0) {
                    qm |= 1 << u;
#pragma unroll
                    for (int o = 0; o < kMaxOut; o++) cy[o] = 0;
                }
                const i32x4 s4 = *reinterpret_cast<const i32x4*>(S + rl * SP + 4 * mfma_sum_unit(w));
                const int s0 = s4[0] + cpc, s1 = s4[1] + cpc, s2 = s4[2] + cpc, s3 = s4[3] + cpc;
                const uint32_t Gv = (e == br && l == (tr >> 5)) ? (1u << (tr & 31)) : 0u;
                const int Ll = lv[u] & 0xFFFF, Lh = lv[u] >> 16, Rl = rv[u] & 0xFFFF, Rh = rv[u] >> 16;
                const int Gl = Gv & 0xFFFF, Gh = Gv >> 16;
#pragma unroll
                for (int o = 0; o < kMaxOut; o++) {
                    if (o < nout) {
                        // P's limb = s0 + 2^8 s1 + 2^16 (s2 + 2^8 s3) with the byte sums
                        // s below 2^20, so every partial sum stays below 2^31
                        int A = __mul24(cPo[o], s0) + (__mul24(cPo[o], s1) << 8) + __mul24(cLo[o], Ll) +
                                __mul24(cRo[o], Rl) + __mul24(cGo[o], Gl);
                        int B = __mul24(cPo[o], s2) + (__mul24(cPo[o], s3) << 8) + __mul24(cLo[o], Lh) +
                                __mul24(cRo[o], Rh) + __mul24(cGo[o], Gh);
                        if (eso[o] >= 0) {
                            const uint32_t x = eso[o] == 0 ? ev[0][u] : ev[kMaxE - 1][u];
                            A += __mul24(cEo[o], (int)(x & 0xFFFF));
                            B += __mul24(cEo[o], (int)(x >> 16));
                        }
                        const int64_t v = cy[o] + (int64_t)A + (int64_t)B * 65536;
                        oq[i][o][u] = (uint32_t)v;
                        cy[o] = v >> 32;
                    }
                }
            }
            if (l == kw - 1) qm |= 1 << 5;
            qv[i] = qm;
#pragma unroll
            for (int o = 0; o < kMaxOut; o++)
                if (o < nout) Cq[o * QP + j] = (qm >> 5) ? 0 : (int32_t)cy[o];  // |carry| < 2^15
        }
        lds_barrier();
        // 3. carries between quads, until none leaves a quad (a thread that
        // passes one on marks the round in `more`; round numbers grow over
        // the passes, so the mark needs no clearing)
        for (;;) {
            ++round;
            int32_t cin[EPT][kMaxOut];
#pragma unroll
            for (int i = 0; i < EPT; i++) {
                const int j = tid + i * THREADS;
#pragma unroll
                for (int o = 0; o < kMaxOut; o++)
                    cin[i][o] = (o < nout && qv[i] && !(qv[i] & 1)) ? Cq[o * QP + j - 1] : 0;
            }
            lds_barrier();
#pragma unroll
            for (int i = 0; i < EPT; i++) {
                if (!qv[i]) continue;
                const int j = tid + i * THREADS;
#pragma unroll
                for (int o = 0; o < kMaxOut; o++) {
                    if (o >= nout) continue;
                    int64_t c = cin[i][o];
#pragma unroll
                    for (int u = 0; u < 4; u++) {
                        if (u > 0 && (qv[i] >> u & 1)) c = 0;  // a new element: the carry stops
                        const int64_t v = (int64_t)oq[i][o][u] + c;
                        oq[i][o][u] = (uint32_t)v;
                        c = v >> 32;
                    }
                    if (qv[i] >> 5) c = 0;
                    Cq[o * QP + j] = (int32_t)c;
                    if (c != 0) *more = round;
                }
            }
            lds_barrier();
            if (*more != round) break;
        }
        // 4. outputs
        const size_t pbase = (size_t)prow * W;
#pragma unroll
        for (int i = 0; i < EPT; i++) {
            if (!qv[i]) continue;
            const int fw = 4 * (tid + i * THREADS);
#pragma unroll
            for (int o = 0; o < kMaxOut; o++)
                if (o < nout) *reinterpret_cast<gu32x4*>(Do[o] + pbase + fw) = oq[i][o];
        }
    }
}

template <int RG, int CG, int CF, bool PRE>
__global__ void __launch_bounds__(RG * CG * 64) k_product_mfma(const ProdSeg* __restrict__ segs, int nseg,
                                                               ProdSeg seg0, ProdItem one, int lds_bytes)
{
    product_mfma_block<RG, CG, CF, PRE>(segs, nseg, seg0, one, lds_bytes, xcd_order(blockIdx.x, gridDim.x));
}

// ---------------------------------------------------------------------------
// The matrix-core product with 256 threads and little LDS, so that two
// workgroups share a CU and one's epilogue (carry chains: VALU, LDS and
// memory latency) runs while the other's matrix cores are busy.
//
// A product's rows go in tiles of 128, and its row of n + 1 elements in
// column splits of mfma2_eps(g, CF) whole elements (one split, the whole row,
// where it fits 64 CF byte columns); a workgroup owns one tile of one split.
// The carry chains run within an element, so the splits are independent.
// Waves: 2 x 2; wave (wr, wc) owns rows 64 wr .. 64 wr + 63 of the tile (two
// 32-row A fragments) and the split's 32-column fragments wc CF .. wc CF +
// CF - 1.  R comes in the 64-row chunk layout of k_rtrans<64> (a column's 64
// bytes contiguous, its 16-byte units permuted by swz64), the split's 1 KB
// units of it straight from global memory into LDS three chunks deep, with
// the chunk's 64 bits of each tile row of L; one barrier per chunk.  The
// epilogue is that of k_product_mfma in passes of PR = 16 PM rows (PM > 1
// where a row is so short that the four waves' lanes hold more than 16 rows'
// quads at once: fewer, fuller passes).  DIRECT (small products, where the
// latency of a level matters more than its rate): the workgroup reads R's
// rows itself and transposes them into every chunk of the layout above, all
// chunks held in LDS at once, so that no transposition pass runs before the
// launch and the main loop waits on nothing.
template <int CF, int PM, bool DIRECT>
__global__ void __launch_bounds__(256, 2) k_product_mfma2(const ProdSeg* __restrict__ segs, int nseg, ProdSeg seg0,
                                                           ProdItem one, int lds_bytes)
{
#define SFFT_MFMA2_TILE xcd_order(blockIdx.x, gridDim.x)
#include "mfma2_body.inc"
#undef SFFT_MFMA2_TILE
}

// The same body for tile `tile` of a segment (the persistent plan kernel).
template <int CF, int PM, bool DIRECT>
__device__ __forceinline__ void product_mfma2_block(const ProdSeg* __restrict__ segs, int nseg, ProdSeg seg0,
                                                    ProdItem one, int lds_bytes, uint32_t tile)
{
#define SFFT_MFMA2_TILE tile
#include "mfma2_body.inc"
#undef SFFT_MFMA2_TILE
}


// One (row, element) of one linear item: dst = cX X + cY Y + cG G, limb by
// limb with the carry.
__device__ __forceinline__ void linear_task(const LinItem& it, const Bufs& bufs, const Geo& g, int task)
{
    const int row = task / g.n1, e = task % g.n1;
    const int br = row / g.k, tr = row % g.k;
    gword* dst = ctp(bufs, it.dst);
    const gword* X = it.X >= 0 ? ctp(bufs, it.X) : nullptr;
    const gword* Y = it.Y >= 0 ? ctp(bufs, it.Y) : nullptr;
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

__global__ void __launch_bounds__(kThreads) k_linear(const LinSeg* __restrict__ segs, int nseg, LinSeg seg0,
                                                     LinItem one, uint32_t ybase)
{
    const uint32_t y = blockIdx.y + ybase;
    LinSeg sg = seg0;
    if (nseg > 1) sg = segs[find_segment(segs, nseg, y, [](const LinSeg& q) { return q.first; })];
    const Geo g = sg.geo;
    const int task = blockIdx.x * kThreads + threadIdx.x;
    if (task >= g.nct * g.n1) return;
    const LinItem it = sg.items ? load_global(sg.items + (y - sg.first)) : one;
    linear_task(it, sg.bufs, g, task);
}

template <int THREADS, int LPR, int DPL, int RPL, int PD, int CG, bool ENC>
hipError_t launch_t(const ProdCfg& cfg, const ProdSeg* d_segs, int nseg, const ProdSeg& seg0, const ProdItem& one,
                    int64_t blocks, uint64_t seed, uint64_t first_id, const MuBits* mu, hipStream_t s)
{
    // the LDS cap, once per instantiation (thread-safe static initialisation)
    static const hipError_t attr =
        hipFuncSetAttribute((const void*)k_product<THREADS, LPR, DPL, RPL, PD, CG, ENC>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr != hipSuccess) return attr;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    const KCfg kc{1u};
    MuBits none{};
    hipLaunchKernelGGL((k_product<THREADS, LPR, DPL, RPL, PD, CG, ENC>), dim3((unsigned)blocks), dim3(THREADS),
                       cfg.lds_bytes, s, kc, d_segs, nseg, seg0, one, seed, first_id, mu ? *mu : none);
    return hipGetLastError();
}

template <int RG, int CG, int CF, bool PRE>
hipError_t launch_mfma_t(const ProdCfg& cfg, const ProdSeg* d_segs, int nseg, const ProdSeg& seg0,
                         const ProdItem& one, int64_t blocks, hipStream_t s)
{
    // the LDS cap, once per instantiation (thread-safe static initialisation)
    static const hipError_t attr =
        hipFuncSetAttribute((const void*)k_product_mfma<RG, CG, CF, PRE>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr != hipSuccess) return attr;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_product_mfma<RG, CG, CF, PRE>), dim3((unsigned)blocks), dim3(RG * CG * 64), cfg.lds_bytes, s,
                       d_segs, nseg, seg0, one, cfg.lds_bytes);
    return hipGetLastError();
}

template <int CF, int PM, bool DIRECT>
hipError_t launch_mfma2_pm(const ProdCfg& cfg, const ProdSeg* d_segs, int nseg, const ProdSeg& seg0,
                           const ProdItem& one, int64_t blocks, hipStream_t s)
{
    static const hipError_t attr = hipFuncSetAttribute((const void*)k_product_mfma2<CF, PM, DIRECT>,
                                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr != hipSuccess) return attr;
    if (blocks <= 0) return hipSuccess;
    if (blocks > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_product_mfma2<CF, PM, DIRECT>), dim3((unsigned)blocks), dim3(256), cfg.lds_bytes, s, d_segs,
                       nseg, seg0, one, cfg.lds_bytes);
    return hipGetLastError();
}

template <int CF, bool DIRECT>
hipError_t launch_mfma2_t(const ProdCfg& cfg, const ProdSeg* d_segs, int nseg, const ProdSeg& seg0,
                          const ProdItem& one, int64_t blocks, hipStream_t s)
{
    switch (cfg.pm) {
    case 1: return launch_mfma2_pm<CF, 1, DIRECT>(cfg, d_segs, nseg, seg0, one, blocks, s);
    case 2: return launch_mfma2_pm<CF, 2, DIRECT>(cfg, d_segs, nseg, seg0, one, blocks, s);
    case 4: return launch_mfma2_pm<CF, 4, DIRECT>(cfg, d_segs, nseg, seg0, one, blocks, s);
    default: return hipErrorInvalidValue;
    }
}

// Tilings: (threads, lanes per row, digit slots per lane, rows per lane,
// lookup pipeline depth, 4-bit groups per chunk).  The first kDefaultTilings
// are the defaults, one per width class; the rest are alternatives the tuner
// may pick for a geometry.
struct Tiling {
    int threads, lpr, dpl, rpl, pd, cg;
};
constexpr Tiling kTilings[] = {
    {256, 4, 4, 8, 2, 8},    // rows of <= 16 digits
    {256, 8, 4, 12, 1, 8},   // <= 32
    {256, 8, 8, 7, 2, 8},    // <= 64
    {512, 8, 12, 5, 2, 8},   // <= 96
    {512, 8, 16, 4, 1, 4},   // <= 128
    // alternatives
    {512, 8, 4, 12, 1, 8},   // <= 32, 8 waves
    {512, 8, 8, 7, 2, 8},    // <= 64, 8 waves
    {256, 8, 8, 8, 2, 4},    // <= 64, 16-row chunks
    {512, 8, 12, 5, 1, 8},   // <= 96, pipeline depth 1
    {256, 8, 12, 5, 2, 4},   // <= 96, 4 waves, 16-row chunks
    {256, 4, 12, 4, 2, 8},   // <= 48, 4 lanes per row
    {512, 4, 20, 2, 1, 8},   // <= 80, 4 lanes per row
};
constexpr int kNumLookupTilings = (int)(sizeof(kTilings) / sizeof(kTilings[0]));
constexpr int kDefaultTilings = 5;

// Matrix-core tilings: (row groups, column groups, 32-column fragments per
// wave).  They follow the lookup tilings in the tiling numbering; a tiling
// serves a geometry whose NF = ceil(4 W / 32) fragments give each column
// group CF of them (the last fewer).
struct MfmaTiling {
    int rg, cgw, cf;
    // right operands transposed by k_rtrans before the launch: 0 no, 1 into
    // 128-row chunks (k_product_mfma), 2 into 64-row chunks (the 256-thread
    // k_product_mfma2, two workgroups per CU)
    int pre;
};
constexpr MfmaTiling kMfmaTilings[] = {
    {2, 4, 1, false}, {2, 4, 2, false}, {2, 4, 3, false},  // 512 threads, 128-row tiles
    {2, 2, 1, false}, {2, 2, 2, false}, {2, 2, 3, false},  // 256 threads, 128-row tiles
    {2, 2, 4, false}, {2, 2, 5, false}, {2, 2, 6, false},
    {4, 2, 2, false}, {4, 2, 3, false}, {4, 2, 4, false},  // 512 threads, 256-row tiles
    {2, 4, 1, true},  {2, 4, 2, true},  {2, 4, 3, true},   // the same with a transposition pass
    {4, 2, 2, true},  {4, 2, 3, true},  {4, 2, 4, true},
    {2, 2, 1, 2},     {2, 2, 2, 2},     {2, 2, 3, 2},      // 256 threads, 64-row chunks, <= 80 KB of LDS
    {2, 2, 4, 2},
    {2, 2, 1, 3},     {2, 2, 2, 3},                        // the same, R transposed in the workgroup, all chunks in LDS
};
constexpr int kNumMfmaTilings = (int)(sizeof(kMfmaTilings) / sizeof(kMfmaTilings[0]));
constexpr int kNumTilings = kNumLookupTilings + kNumMfmaTilings;

hipError_t dispatch_mfma(const ProdCfg& cfg, const ProdSeg* d_segs, int nseg, const ProdSeg& seg0, const ProdItem& one,
                         int64_t blocks, hipStream_t s)
{
#define MCASE(I)                                                                                         \
    if (cfg.tiling == kNumLookupTilings + I)                                                             \
        return launch_mfma_t<kMfmaTilings[I].rg, kMfmaTilings[I].cgw, kMfmaTilings[I].cf,                 \
                             kMfmaTilings[I].pre == 1>(cfg, d_segs, nseg, seg0, one, blocks, s);
#define MCASE2(I)                                                                                        \
    if (cfg.tiling == kNumLookupTilings + I)                                                             \
        return launch_mfma2_t<kMfmaTilings[I].cf, kMfmaTilings[I].pre == 3>(cfg, d_segs, nseg, seg0, one, blocks, s);
    MCASE(0)
    MCASE(1)
    MCASE(2)
    MCASE(3)
    MCASE(4)
    MCASE(5)
    MCASE(6)
    MCASE(7)
    MCASE(8)
    MCASE(9)
    MCASE(10)
    MCASE(11)
    MCASE(12)
    MCASE(13)
    MCASE(14)
    MCASE(15)
    MCASE(16)
    MCASE(17)
    MCASE2(18)
    MCASE2(19)
    MCASE2(20)
    MCASE2(21)
    MCASE2(22)
    MCASE2(23)
#undef MCASE
#undef MCASE2
    static_assert(kNumMfmaTilings == 24, "one MCASE per matrix-core tiling");
    return hipErrorInvalidValue;
}

template <bool ENC>
hipError_t dispatch(const ProdCfg& cfg, const ProdSeg* d_segs, int nseg, const ProdSeg& seg0, const ProdItem& one,
                    int64_t blocks, uint64_t seed, uint64_t first_id, const MuBits* mu, hipStream_t s)
{
    if (cfg.mfma) {
        if (ENC) return hipErrorInvalidValue;  // encryption draws its bits of L inside the lookup kernel
        return dispatch_mfma(cfg, d_segs, nseg, seg0, one, blocks, s);
    }
#define CASE(I)                                                                                              \
    if (cfg.tiling == I)                                                                                     \
        return launch_t<kTilings[I].threads, kTilings[I].lpr, kTilings[I].dpl, kTilings[I].rpl, kTilings[I].pd, \
                        kTilings[I].cg, ENC>(cfg, d_segs, nseg, seg0, one, blocks, seed, first_id, mu, s);
    CASE(0)
    CASE(1)
    CASE(2)
    CASE(3)
    CASE(4)
    CASE(5)
    CASE(6)
    CASE(7)
    CASE(8)
    CASE(9)
    CASE(10)
    CASE(11)
#undef CASE
    static_assert(kNumLookupTilings == 12, "one CASE per tiling");
    return hipErrorInvalidValue;
}

ProdSeg single_segment(const Bufs& b, const Geo& g, const ProdCfg& cfg)
{
    ProdSeg sg{};
    sg.bufs = b;
    sg.geo = g;
    sg.nd = cfg.nd;
    sg.wd = cfg.wd;
    return sg;
}

}  // namespace

int tiling_count() { return kNumTilings; }

void tiling_fields(int ti, int* f)
{
    if (ti >= kNumLookupTilings) {
        const MfmaTiling& t = kMfmaTilings[ti - kNumLookupTilings];
        f[0] = t.rg * t.cgw * 64, f[1] = t.rg, f[2] = t.cgw, f[3] = t.cf, f[4] = t.pre, f[5] = 0, f[6] = 1;
        return;
    }
    const Tiling& t = kTilings[ti];
    f[0] = t.threads, f[1] = t.lpr, f[2] = t.dpl, f[3] = t.rpl, f[4] = t.pd, f[5] = t.cg, f[6] = 0;
}

namespace {
bool mfma_config(const Geo& g, int ti, ProdCfg* cfg)
{
    const MfmaTiling& t = kMfmaTilings[ti - kNumLookupTilings];
    const int nf = (4 * g.W + 31) / 32;
    if (t.pre < 2 && (nf + t.cgw - 1) / t.cgw != t.cf) return false;
    // the staging blocks of a chunk (32 row quads x ceil(W/4) word quads,
    // 8 x 8 per wave) fit the threads' blocks
    const int threads = t.rg * t.cgw * 64;
    const int spt = (kMfmaChunk / 4 * 2 * t.cgw * t.cf + threads - 1) / threads;
    if (t.pre < 2 && 4 * ((g.W + 31) / 32) > spt * threads / 64) return false;
    *cfg = ProdCfg{};
    cfg->tiling = ti;
    cfg->mfma = true;
    cfg->threads = t.rg * t.cgw * 64;
    cfg->rg = t.rg;
    cfg->cgw = t.cgw;
    cfg->cf = t.cf;
    cfg->pre = t.pre;
    cfg->max_nct = g.nct;
    cfg->tr = 64 * t.rg;
    cfg->nd = (g.k + kDigitBits - 1) / kDigitBits;
    cfg->wd = g.n1 * cfg->nd;
    // LDS: the main loop's chunks, or the epilogue's slab of 32 rows of
    // column sums and its carries between quads, and a popcount per tile row
    // (the transposition-pass tilings keep three chunks of R and of the bits
    // of L in flight, the others two chunks of R and of L as bytes)
    // (the 256-thread kernel: three 64-row chunks of R and of the bits of L,
    // or its epilogue's passes of 16 rows)
    const int tail = cfg->tr * 4 + 16;  // popcounts, a flag
    if (t.pre >= 2) {
        // column splits of whole elements (mfma2_eps), each filling more than
        // 2 (CF - 1) of the tile's 2 CF fragments
        const int eps = mfma2_eps(g, t.cf);
        if (eps == 0 || nf > 12) return false;
        const int cs = (g.n1 + eps - 1) / eps;
        const int bytes = cs == 1 ? 4 * g.W : eps * g.k / 8;
        if ((bytes + 31) / 32 <= 2 * (t.cf - 1)) return false;
        const int ww = cs == 1 ? g.W : eps * g.kw;  // words of a split row
        // split rows in whole quads, at most 16; whole rows (W <= 64) of any
        // number of words, in groups of rows that are whole quads
        if (cs > 1 && (ww % 4 != 0 || ww / 4 > 16)) return false;
        cfg->cs = cs;
        // epilogue passes of 16 pm rows: as many (up to 64) as the four
        // waves' lanes take at once (groups of rpg rows, qg quads each), as
        // long as the LDS stays within two workgroups per CU or what 16 rows
        // need
        const int rpg = cs > 1 || ww % 4 == 0 ? 1 : (ww & 1) ? 4 : 2;
        const int qg = rpg * ww / 4;
        const int sweep = 4 * (64 / qg) * rpg;
        // (pre 3: every 64-row chunk of R and of the bits of L at once)
        const int main_bytes =
            t.pre == 3 ? (g.nct + 63) / 64 * (4 * t.cf * 1024 + cfg->tr * 8) : mfma2_main_bytes(t.cf);
        auto lds_for = [&](int pm) {
            return std::max(main_bytes, mfma2_epi_bytes(t.cf, 16 * pm * ww / 4, pm)) + tail;
        };
        const int lim = std::max(lds_for(1), 80 * 1024);
        cfg->pm = sweep >= 64 ? 4 : sweep >= 32 ? 2 : 1;
        while (cfg->pm > 1 && lds_for(cfg->pm) > lim) cfg->pm /= 2;
        cfg->lds_bytes = lds_for(cfg->pm);
        return cfg->lds_bytes <= 160 * 1024;
    }
    const int chunks = t.pre ? 3 * nf * 32 * kMfmaPitch + 3 * cfg->tr * 16
                             : 2 * nf * 32 * kMfmaPitch + 2 * cfg->tr * kMfmaChunk;
    cfg->lds_bytes = std::max(chunks, mfma_epi_bytes(nf, g.W)) + tail;
    return cfg->lds_bytes <= 160 * 1024;
}
}  // namespace

bool tiling_config(const Geo& g, int ti, ProdCfg* cfg)
{
    if (ti < 0 || ti >= kNumTilings) return false;
    if (g.nct % 32 != 0 || g.W * 32 != g.nct || g.W > kMaxRowWords) return false;
    if (ti >= kNumLookupTilings) return mfma_config(g, ti, cfg);
    const Tiling& t = kTilings[ti];
    const int nd = (g.k + kDigitBits - 1) / kDigitBits;
    const int wd = g.n1 * nd;
    if (t.lpr * t.dpl < wd) return false;
    *cfg = ProdCfg{};
    cfg->tiling = ti;
    cfg->threads = t.threads;
    cfg->cg = t.cg;
    cfg->nd = nd;
    cfg->wd = wd;
    cfg->lpr = t.lpr;
    cfg->dpl = t.dpl;
    cfg->st = t.lpr * t.dpl;
    cfg->rpw = 64 / t.lpr;
    const int per_iter = (t.threads / 64) * cfg->rpw;
    cfg->rpl = t.rpl;
    cfg->tr = per_iter * t.rpl;
    // LDS: two chunks of rows of R, three chunks of bits of L, two table
    // sets; the epilogue reuses it for one pass of 64-bit digit sums
    const int pi = pass_iters(t.threads, cfg->rpw, cfg->st, t.rpl);
    const int main_words = 2 * 4 * t.cg * g.W + 3 * cfg->tr + 2 * t.cg * 16 * cfg->st;
    const int epi_words = 2 * per_iter * pi * cfg->st;
    cfg->lds_bytes = 4 * (main_words > epi_words ? main_words : epi_words);
    return cfg->lds_bytes <= 160 * 1024;
}

namespace {
std::mutex g_tuned_mu;
std::map<std::pair<int, int>, int> g_tuned;  // (k, n+1) -> tiling
}  // namespace

void set_tuned_tiling(const Geo& g, int ti)
{
    std::lock_guard<std::mutex> lock(g_tuned_mu);
    if (ti < 0) g_tuned.erase({g.k, g.n1});
    else g_tuned[{g.k, g.n1}] = ti;
}

bool product_config(const Geo& g, ProdCfg* cfg)
{
    {
        std::lock_guard<std::mutex> lock(g_tuned_mu);
        auto it = g_tuned.find({g.k, g.n1});
        if (it != g_tuned.end() && tiling_config(g, it->second, cfg)) return true;
    }
    // matrix cores first: products of at most 512 rows (levels too small to
    // fill the GPU, bound by a workgroup's latency) on the 256-thread kernel
    // that transposes R in the workgroup; else the 256-thread kernel with
    // two workgroups per CU where it serves the row (whole quads of words per
    // split row), then rows of up to 2 fragments on 256 threads, 3..8 on
    // 256-row tiles with the transposition pass, 9..12 on four column groups
    // transposing in-kernel
    if (g.nct <= 512 && tiling_config(g, kNumLookupTilings + 22, cfg)) return true;
    static const int order[] = {18, 19, 20, 21, 3, 15, 16, 17, 4, 0, 1, 2};
    for (int i : order)
        if (tiling_config(g, kNumLookupTilings + i, cfg)) return true;
    return lookup_config(g, cfg);
}

bool lookup_config(const Geo& g, ProdCfg* cfg)
{
    for (int i = 0; i < kDefaultTilings; i++)
        if (tiling_config(g, i, cfg)) return true;
    return false;
}

namespace {
// the transposition of a launch's right operands (matrix-core tilings)
template <int KC>
hipError_t launch_rtrans_t(const ProdCfg& cfg, const ProdSeg* d_segs, int nseg, const ProdSeg& seg0,
                           const ProdItem& one, int64_t items, hipStream_t s)
{
    constexpr int kMaxChunkBytes = 12 * 32 * KC;  // rows of up to 12 fragments
    // once (thread-safe static initialisation)
    static const hipError_t attr =
        hipFuncSetAttribute((const void*)k_rtrans<KC>, hipFuncAttributeMaxDynamicSharedMemorySize, kMaxChunkBytes);
    if (attr != hipSuccess) return attr;
    if (items <= 0) return hipSuccess;
    if (items > 0x7FFFFFFF) return hipErrorInvalidValue;
    // chunks of the launch's largest Nct, else of the widest row the tiling
    // serves: Nct = 32 W <= 256 CG CF, or, split into whole elements, rows
    // of up to 12 fragments (W <= 96)
    const int max_nct = cfg.max_nct > 0 ? cfg.max_nct : cfg.pre == 2 ? 32 * 96 : 256 * cfg.cgw * cfg.cf;
    const unsigned chunks = (unsigned)((max_nct + KC - 1) / KC);
    hipLaunchKernelGGL(k_rtrans<KC>, dim3((unsigned)items, chunks), dim3(kRtransThreads), kMaxChunkBytes, s, d_segs,
                       nseg, seg0, one);
    return hipGetLastError();
}

hipError_t launch_rtrans(const ProdCfg& cfg, const ProdSeg* d_segs, int nseg, const ProdSeg& seg0,
                         const ProdItem& one, int64_t items, hipStream_t s)
{
    return cfg.pre == 2 ? launch_rtrans_t<64>(cfg, d_segs, nseg, seg0, one, items, s)
                        : launch_rtrans_t<kMfmaChunk>(cfg, d_segs, nseg, seg0, one, items, s);
}
}  // namespace

hipError_t launch_products(const ProdCfg& cfg, const ProdSeg* d_segs, int nseg, const ProdSeg& seg0,
                           int64_t blocks, int64_t items, hipStream_t s, hipEvent_t mark)
{
    ProdItem none{};
    if (cfg.mfma && (cfg.pre == 1 || cfg.pre == 2)) {
        hipError_t e = launch_rtrans(cfg, d_segs, nseg, seg0, none, blocks > 0 ? items : 0, s);
        if (e != hipSuccess) return e;
    }
    if (mark) {
        hipError_t e = hipEventRecord(mark, s);
        if (e != hipSuccess) return e;
    }
    return dispatch<false>(cfg, d_segs, nseg, seg0, none, blocks, 0, 0, nullptr, s);
}

bool inkernel_twin(const Geo& g, ProdCfg* cfg)
{
    if (!cfg->mfma || cfg->pre == 0 || cfg->pre == 3) return true;
    for (int i = 0; i < kNumMfmaTilings; i++) {
        const MfmaTiling& t = kMfmaTilings[i];
        if (!t.pre && t.rg == cfg->rg && t.cgw == cfg->cgw && t.cf == cfg->cf)
            return tiling_config(g, kNumLookupTilings + i, cfg);
    }
    return false;
}

hipError_t launch_product_one(const Bufs& b, const Geo& g, const ProdCfg& cfg, const ProdItem& item, uint8_t* rt,
                              hipStream_t s)
{
    ProdSeg seg = single_segment(b, g, cfg);
    seg.rt = rt;
    if (cfg.mfma && (cfg.pre == 1 || cfg.pre == 2)) {
        hipError_t e = launch_rtrans(cfg, nullptr, 1, seg, item, 1, s);
        if (e != hipSuccess) return e;
    }
    return dispatch<false>(cfg, nullptr, 1, seg, item, product_tiles(g, cfg), 0, 0, nullptr, s);
}

hipError_t launch_linear(int64_t max_elems, const LinSeg* d_segs, int nseg, const LinSeg& seg0, int64_t total,
                         hipStream_t s)
{
    LinItem none{};
    const int blocks = (int)((max_elems + kThreads - 1) / kThreads);
    for (int64_t b0 = 0; b0 < total; b0 += 65535) {
        const int64_t n = total - b0 < 65535 ? total - b0 : 65535;
        hipLaunchKernelGGL(k_linear, dim3(blocks, (unsigned)n), dim3(kThreads), 0, s, d_segs, nseg, seg0, none,
                           (uint32_t)b0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// Whole-plan persistent execution (small plans): one cooperative launch runs
// every level, the workgroups looping over the level's product tiles and
// linear tasks, with a grid-wide barrier where a kernel boundary was.  The
// barrier: each workgroup releases its writes to the device (agent-scope
// fence: the XCDs' L2s are written back), adds one to a counter, and waits
// until the counter reaches its generation times the grid size, then
// acquires (its caches invalidated).  Every wait is bounded: past the limit
// the workgroup sets an error flag and goes on, so the kernel always ends.
namespace {
constexpr uint32_t kBarrierSpins = 1u << 22;  // s_sleep rounds (about 0.1 s)

__device__ __forceinline__ void grid_barrier(uint32_t* bar, uint32_t target)
{
    __syncthreads();  // every wave's stores done (they are in this XCD's L2)
    if (threadIdx.x == 0) {
        // one release for the workgroup (L2 written back), a relaxed count,
        // a relaxed poll (each poll would otherwise invalidate the L2), one
        // acquire (the caches invalidated) for the workgroup
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(bar, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t spins = 0;
        while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (++spins == kBarrierSpins) {
                __hip_atomic_fetch_or(bar + 1, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

__global__ void k_zero_words(uint32_t* p, int n)
{
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// The level loop of a persistent plan: each level's product tiles (tile(seg,
// v) runs tile v of the level's items), then its linear passes, with a grid
// barrier after each; the output forms last.
template <int THREADS, typename Tile>
__device__ __forceinline__ void plan_persistent(const PersistArgs& a, Tile tile)
{
    const uint32_t nb = gridDim.x;
    const int64_t per = (int64_t)a.geo.nct * a.geo.n1;  // linear tasks per item
    const int64_t t0 = (int64_t)blockIdx.x * THREADS + threadIdx.x, tstep = (int64_t)nb * THREADS;
    uint32_t gen = 0;
    for (int L = 0; L < a.nlevels; L++) {
        const int64_t pb = a.lv[4 * L], pc = a.lv[4 * L + 1], p0 = a.lv[4 * L + 2], np = a.lv[4 * L + 3];
        if (pc > 0) {
            const ProdSeg seg{a.prods + pb, a.bufs, a.geo, a.nd, a.wd, 0, 0, nullptr};
            const uint32_t blocks = (uint32_t)pc * a.tiles;
            for (uint32_t v = blockIdx.x; v < blocks; v += nb) {
                tile(seg, v);
                __syncthreads();  // the next tile reuses the LDS
            }
            grid_barrier(a.bar, ++gen * nb);
        }
        for (int64_t q = 0; q < np; q++) {
            const int64_t lb = a.pass[2 * (p0 + q)], tasks = a.pass[2 * (p0 + q) + 1] * per;
            for (int64_t t = t0; t < tasks; t += tstep) linear_task(a.lins[lb + t / per], a.bufs, a.geo, (int)(t % per));
            grid_barrier(a.bar, ++gen * nb);
        }
    }
    const int64_t tasks = a.nfinal * per;
    for (int64_t t = t0; t < tasks; t += tstep) linear_task(a.finals[t / per], a.bufs, a.geo, (int)(t % per));
}

// products on the 512-thread body with in-kernel transposition
template <int RG, int CG, int CF>
__global__ void __launch_bounds__(RG * CG * 64) k_plan_persistent(PersistArgs a, int lds_bytes)
{
    const ProdItem none{};
    plan_persistent<RG * CG * 64>(a, [&](const ProdSeg& seg, uint32_t v) {
        product_mfma_block<RG, CG, CF, false>(nullptr, 1, seg, none, lds_bytes, v);
    });
}

// products on the 256-thread body that transposes R in the workgroup
template <int CF, int PM>
__global__ void __launch_bounds__(256, 2) k_plan_persistent2(PersistArgs a, int lds_bytes)
{
    const ProdItem none{};
    plan_persistent<256>(a, [&](const ProdSeg& seg, uint32_t v) {
        product_mfma2_block<CF, PM, true>(nullptr, 1, seg, none, lds_bytes, v);
    });
}

// One cooperative launch of fn (threads per workgroup) with as many
// workgroups as are resident at once, at most max_blocks.
hipError_t launch_cooperative(const void* fn, int threads, const PersistArgs& a, const ProdCfg& cfg,
                              int64_t max_blocks, hipStream_t s)
{
    int dev = 0, cus = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, cfg.lds_bytes);
    if (e != hipSuccess) return e;
    // every workgroup resident at once (the barriers wait for all of them)
    const int64_t resident = (int64_t)cus * per_cu;
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(resident, max_blocks));
    if (resident < 1) return hipErrorCooperativeLaunchTooLarge;
    hipLaunchKernelGGL(k_zero_words, dim3(1), dim3(64), 0, s, a.bar, 2);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    PersistArgs args = a;
    int lds = cfg.lds_bytes;
    void* params[] = {(void*)&args, (void*)&lds};
    return hipLaunchCooperativeKernel(fn, dim3((unsigned)grid), dim3(threads), params, (unsigned)cfg.lds_bytes, s);
}

template <int CF>
hipError_t launch_persistent_t(const PersistArgs& a, const ProdCfg& cfg, int64_t max_blocks, hipStream_t s)
{
    const void* fn = (const void*)k_plan_persistent<2, 4, CF>;
    static const hipError_t attr = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr != hipSuccess) return attr;
    return launch_cooperative(fn, 512, a, cfg, max_blocks, s);
}

template <int CF, int PM>
hipError_t launch_persistent2_t(const PersistArgs& a, const ProdCfg& cfg, int64_t max_blocks, hipStream_t s)
{
    const void* fn = (const void*)k_plan_persistent2<CF, PM>;
    static const hipError_t attr = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (attr != hipSuccess) return attr;
    return launch_cooperative(fn, 256, a, cfg, max_blocks, s);
}
}  // namespace

bool persistent_config(const Geo& g, ProdCfg* cfg)
{
    // the 256-thread kernel that transposes R in the workgroup (every chunk
    // in LDS), 1 or 2 fragments per wave; else the 512-thread kernel with
    // in-kernel transposition, 2 x 4 waves of 1 or 2 fragments: rows of up to
    // 8 fragments
    for (int i = 0; i < kNumMfmaTilings; i++) {
        const MfmaTiling& t = kMfmaTilings[i];
        if (t.pre == 3 && tiling_config(g, kNumLookupTilings + i, cfg)) return true;
    }
    for (int i = 0; i < kNumMfmaTilings; i++) {
        const MfmaTiling& t = kMfmaTilings[i];
        if (t.pre == 0 && t.rg == 2 && t.cgw == 4 && t.cf <= 2 && tiling_config(g, kNumLookupTilings + i, cfg))
            return true;
    }
    return false;
}

hipError_t launch_plan_persistent(const PersistArgs& a, const ProdCfg& cfg, int64_t max_blocks, hipStream_t s)
{
    if (cfg.pre == 3) {
        const int k = 4 * (cfg.cf - 1) + (cfg.pm == 4 ? 2 : cfg.pm == 2 ? 1 : 0);
        switch (k) {
        case 0: return launch_persistent2_t<1, 1>(a, cfg, max_blocks, s);
        case 1: return launch_persistent2_t<1, 2>(a, cfg, max_blocks, s);
        case 2: return launch_persistent2_t<1, 4>(a, cfg, max_blocks, s);
        case 4: return launch_persistent2_t<2, 1>(a, cfg, max_blocks, s);
        case 5: return launch_persistent2_t<2, 2>(a, cfg, max_blocks, s);
        case 6: return launch_persistent2_t<2, 4>(a, cfg, max_blocks, s);
        default: return hipErrorInvalidValue;
        }
    }
    return cfg.cf == 1 ? launch_persistent_t<1>(a, cfg, max_blocks, s) : launch_persistent_t<2>(a, cfg, max_blocks, s);
}

// Words [row_off, row_off + W) of each of n ciphertexts of cw words (the
// row that decryption reads) packed into dst, n x W words.
__global__ void k_gather_rows(const uint32_t* __restrict__ ct, int64_t cw, int64_t row_off, int W, int64_t n,
                              uint32_t* __restrict__ dst)
{
    const int64_t total = n * W, step = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += step) {
        const int64_t c = i / W;
        dst[i] = ct[c * cw + row_off + (i - c * W)];
    }
}

hipError_t launch_gather_rows(const uint32_t* ct, int64_t cw, int64_t row_off, int W, int64_t n, uint32_t* dst,
                              hipStream_t s)
{
    if (n <= 0 || W <= 0) return hipSuccess;
    const int64_t total = n * W;
    const int64_t want = (total + kThreads - 1) / kThreads;
    hipLaunchKernelGGL(k_gather_rows, dim3((unsigned)(want < 8192 ? want : 8192)), dim3(kThreads), 0, s, ct, cw,
                       row_off, W, n, dst);
    return hipGetLastError();
}

hipError_t launch_linear_one(const Bufs& b, const Geo& g, const LinItem& item, hipStream_t s)
{
    const int blocks = (g.nct * g.n1 + kThreads - 1) / kThreads;
    LinSeg seg0{};
    seg0.bufs = b;
    seg0.geo = g;
    hipLaunchKernelGGL(k_linear, dim3(blocks, 1), dim3(kThreads), 0, s, (const LinSeg*)nullptr, 1, seg0, item, 0u);
    return hipGetLastError();
}

hipError_t launch_encrypt(const Bufs& b, const Geo& g, const ProdCfg& cfg, const uint32_t* bits, int n_ct,
                          uint64_t seed, uint64_t first_id, hipStream_t s)
{
    if (n_ct <= 0) return hipSuccess;
    if (n_ct > kMaxEncPerLaunch) return hipErrorInvalidValue;
    ProdCfg lk = cfg;
    if (cfg.mfma && !lookup_config(g, &lk)) return hipErrorInvalidValue;
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
    return dispatch<true>(lk, nullptr, 1, single_segment(b, g, lk), one, (int64_t)n_ct * product_tiles(g, lk), seed,
                          first_id, &mu, s);
}

}  // namespace sfft
