// Host-side declarations of the gfx950 kernels' launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "schedule.hpp"

namespace sfft {

// Device buffers a ciphertext reference can point into.
struct Bufs {
    uint32_t* in;
    uint32_t* out;
    uint32_t* ws;
    uint32_t* aux;
    int64_t ct_words;  // uint32 words per ciphertext = Nct * (n+1) * k/32
};

// Ciphertext geometry: Nct rows of n1 = n+1 elements of kw = k/32 limbs.
struct Geo {
    int32_t nct, n1, kw, W, k;
};

// Per-geometry choice of the product kernel's tiling.
struct ProdCfg {
    int tiling;  // index into the kernel's tiling table
    int threads; // threads per workgroup
    int cg;      // 4-bit groups (4 rows of R each) per chunk
    int nd;    // 30-bit digits per element (ceil(k/30))
    int wd;    // digits per row (n1 * nd)
    int lpr;   // lanes per output row
    int dpl;   // digit slots per lane
    int st;    // digit slots per row (lpr * dpl >= wd)
    int rpw;   // rows per wave per row-iteration (64 / lpr)
    int rpl;   // row-iterations per lane
    int tr;    // rows per workgroup
    int lds_bytes;
    // matrix-core tilings (mfma): row groups, column groups, 32-column
    // fragments per wave
    bool mfma;
    int rg, cgw, cf;
    int pre;   // right operands transposed into rt by a pass before the launch (1: 128-row chunks, 2: 64-row)
    int cs;    // workgroups per row tile: column splits of whole elements (the 256-thread kernel), else 1
    int pm = 1;  // the 256-thread kernel's epilogue passes: 16 pm rows (1, 2 or 4)
    // rows of the transposition pass's grid: the largest Nct among a
    // launch's segments (0: the largest the tiling serves)
    int max_nct = 0;
};

// Passed to the kernel by value.
struct KCfg {
    // always 1: a run-time multiplier makes acc = digit * one + acc compile to
    // v_mad_u64_u32, which takes the 32-bit digit as is (no zero-extended pair)
    uint32_t one;
};

// The kernels' tilings: how many, and the 7 fields of one: for the lookup
// kernel (threads, lanes per row, digit slots per lane, rows per lane,
// pipeline depth, groups per chunk, 0), for the matrix-core kernel (threads,
// row groups, column groups, fragments per wave, transposition pass, 0, 1).
int tiling_count();
void tiling_fields(int ti, int* fields7);
// cfg for tiling ti on geometry g; false if ti cannot serve g (too few digit
// slots or fragments per row, or more LDS than a CU has).
bool tiling_config(const Geo& g, int ti, ProdCfg* cfg);
// The tiling a plan of geometry g uses: the one recorded for g by the tuner
// (set_tuned_tiling, process-wide; ti < 0 clears), else the matrix-core
// default for g's row width, else the lookup default of g's width class.
bool product_config(const Geo& g, ProdCfg* cfg);
// The lookup default of g's width class (encryption draws its bits of L
// inside the lookup kernel, so it always runs there).
bool lookup_config(const Geo& g, ProdCfg* cfg);
void set_tuned_tiling(const Geo& g, int ti);

// A run of work items sharing one set of buffers and one ciphertext
// geometry (one request).  A launch covers the concatenation of its
// segments; `first` is the index of the segment's first item within the
// launch.  Segments of one product launch may differ in geometry but share
// the kernel tiling (ProdCfg::tiling); nd and wd are the segment's digits per
// element and per row.  A product item takes product_tiles() workgroups (row
// tiles); first_block is the segment's first workgroup within the launch.
struct ProdSeg {
    const ProdItem* items;
    Bufs bufs;
    Geo geo;
    int32_t nd, wd;
    uint32_t first;
    uint32_t first_block;
    // matrix-core tilings: scratch for the segment's right operands in chunk
    // layout, rt_item_bytes(geo) per item (item i at rt + i * rt_item_bytes)
    uint8_t* rt;
};

// Bytes of one right operand in the matrix-core kernel's chunk layout:
// ceil(Nct/128) chunks of NF = ceil(4 W / 32) fragments x 32 columns x 128
// rows, one byte each.  0 where no matrix-core tiling serves the geometry
// (rows of more than 12 fragments).
__host__ __device__ inline int64_t rt_item_bytes(const Geo& g)
{
    const int64_t nf = (4 * (int64_t)g.W + 31) / 32;
    if (nf > 12) return 0;
    return ((int64_t)g.nct + 127) / 128 * nf * 32 * 128;
}
struct LinSeg {
    const LinItem* items;
    Bufs bufs;
    Geo geo;
    uint32_t first;
    uint32_t pad;
};

// Workgroups per product item of geometry g: row tiles times column splits.
inline int product_tiles(const Geo& g, const ProdCfg& cfg)
{
    return (g.nct + cfg.tr - 1) / cfg.tr * (cfg.cs > 1 ? cfg.cs : 1);
}

// Elements per column split of the 256-thread matrix-core kernel with cf
// fragments per wave (a tile spans 64 cf byte columns): all n + 1 where the
// row fits; else the most whole elements that fit and start every split on
// a multiple of 4 words (rows of a multiple of 4 words); 0 if none.
__host__ __device__ inline int mfma2_eps(const Geo& g, int cf)
{
    if (4 * g.W <= 64 * cf) return g.n1;
    if (g.W % 4 != 0) return 0;
    for (int e = g.n1 - 1; e >= 1; e--)
        if (e * g.k / 8 <= 64 * cf && (e * g.kw) % 4 == 0) return e;
    return 0;
}

// One launch over `blocks` workgroups (the sum over the segments of items x
// product_tiles) in nseg segments of `items` items in all: d_segs in device
// memory when nseg > 1, else seg0 (by value).  cfg is the tiling shared by
// the segments with lds_bytes the largest any of them needs.  Under a
// matrix-core tiling a transposition launch first fills each segment's rt.
// A non-null mark is recorded on s just before the product kernel itself.
hipError_t launch_products(const ProdCfg& cfg, const ProdSeg* d_segs, int nseg, const ProdSeg& seg0,
                           int64_t blocks, int64_t items, hipStream_t s, hipEvent_t mark = nullptr);
// One product item passed by value (single gates); rt as in ProdSeg (one
// item's worth, used under a matrix-core tiling).
hipError_t launch_product_one(const Bufs& b, const Geo& g, const ProdCfg& cfg, const ProdItem& item, uint8_t* rt,
                              hipStream_t s);
// Replace a transposition-pass tiling by its twin that transposes inside
// the product kernel (same tile shape, same results, no rt scratch); false
// if the twin cannot serve g.  Other tilings are left as they are.
bool inkernel_twin(const Geo& g, ProdCfg* cfg);
// Linear items; max_elems = the largest Nct * (n+1) among the segments.
hipError_t launch_linear(int64_t max_elems, const LinSeg* d_segs, int nseg, const LinSeg& seg0, int64_t total,
                         hipStream_t s);
hipError_t launch_linear_one(const Bufs& b, const Geo& g, const LinItem& item, hipStream_t s);
// row_off..row_off+W of each of n ciphertexts (cw words apart) packed into
// dst (n x W words, device)
hipError_t launch_gather_rows(const uint32_t* ct, int64_t cw, int64_t row_off, int W, int64_t n, uint32_t* dst,
                              hipStream_t s);

// A whole plan in one persistent launch (device tables of the schedule).
struct PersistArgs {
    const ProdItem* prods;
    const LinItem* lins;
    const LinItem* finals;
    const int64_t* lv;    // per level: first product item, items, first pass, passes
    const int64_t* pass;  // per linear pass: first item, items
    int32_t nlevels;
    int32_t nfinal;
    Bufs bufs;
    Geo geo;
    int32_t nd, wd;
    uint32_t tiles;  // workgroups per product item
    uint32_t* bar;   // barrier counter, time-out flag (cleared by the launch)
};
// The tiling the persistent kernel uses for a geometry; false if none serves it.
bool persistent_config(const Geo& g, ProdCfg* cfg);
// Clears the barrier words, then one cooperative launch of at most
// max_blocks workgroups, all resident at once.
hipError_t launch_plan_persistent(const PersistArgs& a, const ProdCfg& cfg, int64_t max_blocks, hipStream_t s);

// Encryption of n_ct bits: out[i] = mu_i G + R_i A with R_i drawn from
// SplitMix64 domain 4 (ciphertext id first_id + i).  bits: one bit per
// ciphertext, packed LSB first, at most kMaxEncPerLaunch per call.
constexpr int kMaxEncPerLaunch = 16384;
hipError_t launch_encrypt(const Bufs& b, const Geo& g, const ProdCfg& cfg, const uint32_t* bits, int n_ct,
                          uint64_t seed, uint64_t first_id, hipStream_t s);

}  // namespace sfft
