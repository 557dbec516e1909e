// Tiling autotuner: times every kernel tiling that can serve a ciphertext
// geometry on a synthetic level of products of that geometry and records
// the fastest for the plans created afterwards.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <vector>

#include "../../include/sfft.h"
#include "device.hpp"
#include "plan_internal.hpp"
#include "schedule.hpp"

using namespace sfft;

namespace {

Geo geometry(const sfft_params* p)
{
    Geo g;
    g.k = p->k;
    g.kw = p->k / 32;
    g.n1 = p->n_lwe + 1;
    g.nct = g.n1 * p->k;
    g.W = g.n1 * g.kw;
    return g;
}

bool params_valid(const sfft_params* p)
{
    return p && p->n_lwe >= 1 && p->n_lwe <= 64 && p->k > 0 && p->k % 32 == 0 && p->k <= 8192 &&
           p->m == (p->n_lwe + 1) * p->k;
}

uint64_t splitmix(uint64_t& s)
{
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

struct DevBuf {
    void* p = nullptr;
    ~DevBuf()
    {
        if (p) (void)hipFree(p);
    }
};

}  // namespace

extern "C" {

int sfft_tiling_count(void) { return tiling_count(); }

int sfft_tiling_describe(int32_t tiling, int32_t* fields)
{
    if (tiling < 0 || tiling >= tiling_count() || !fields) return sfft_fail(SFFT_EINVAL, "no such tiling");
    int f[7];
    tiling_fields(tiling, f);
    for (int i = 0; i < 7; i++) fields[i] = f[i];
    return SFFT_OK;
}

int sfft_set_tiling(const sfft_params* params, int32_t tiling)
{
    if (!params_valid(params)) return sfft_fail(SFFT_EINVAL, "bad params");
    const Geo g = geometry(params);
    ProdCfg cfg;
    if (tiling >= 0 && !tiling_config(g, tiling, &cfg)) return sfft_fail(SFFT_EINVAL, "tiling cannot serve this geometry");
    set_tuned_tiling(g, tiling);
    return SFFT_OK;
}

int sfft_tune(const sfft_params* params, int32_t reps, int32_t* best_tiling, double* rates, void* hip_stream)
{
    if (!params_valid(params) || !best_tiling || reps < 1) return sfft_fail(SFFT_EINVAL, "bad arguments");
    const Geo g = geometry(params);
    hipStream_t s = (hipStream_t)hip_stream;
    const int nt = tiling_count();
    ProdCfg def;
    if (!product_config(g, &def)) return sfft_fail(SFFT_EUNSUPPORTED, "no kernel configuration for this geometry");

    // A level of products on random operands: a pool of 16 operands, each
    // product writing an AND and an XOR output of its own (the two outputs
    // of a half adder), enough products for several waves of workgroups.
    const int64_t words = (int64_t)g.nct * g.W;
    const size_t ct_bytes = (size_t)words * 4;
    const int pool = 16;
    int64_t items = (8 * 512 + product_tiles(g, def) - 1) / product_tiles(g, def);
    if (items < 16) items = 16;
    while (items > 16 && (size_t)(2 * items) * ct_bytes > ((size_t)3 << 30)) items /= 2;
    DevBuf d_pool, d_out, d_items, d_rt;
    hipError_t e = hipMalloc(&d_pool.p, pool * ct_bytes);
    if (e == hipSuccess) e = hipMalloc(&d_out.p, 2 * items * ct_bytes);
    if (e == hipSuccess) e = hipMalloc(&d_items.p, items * sizeof(ProdItem));
    if (e == hipSuccess && rt_item_bytes(g) > 0) e = hipMalloc(&d_rt.p, (size_t)items * rt_item_bytes(g));
    if (e != hipSuccess) return sfft_hip_fail(e, "tuner buffers");
    {
        std::vector<uint32_t> host((size_t)pool * words);
        uint64_t st = 0x5EED5EEDull + (uint64_t)g.k * 131 + g.n1;
        for (auto& w : host) w = (uint32_t)splitmix(st);
        e = hipMemcpy(d_pool.p, host.data(), host.size() * 4, hipMemcpyHostToDevice);
        if (e != hipSuccess) return sfft_hip_fail(e, "tuner upload");
    }
    std::vector<ProdItem> it(items);
    for (int64_t i = 0; i < items; i++) {
        ProdItem& x = it[i];
        std::memset(&x, 0, sizeof x);
        x.L = ct_ref(B_IN, (int32_t)(i % pool));
        x.R = ct_ref(B_IN, (int32_t)((i * 5 + 1) % pool));
        x.nout = 2;
        x.dst[0] = ct_ref(B_OUT, (int32_t)(2 * i));
        x.cP[0] = 1;
        x.dst[1] = ct_ref(B_OUT, (int32_t)(2 * i + 1));
        x.cL[1] = 1, x.cR[1] = 1, x.cP[1] = -2;
        for (int o = 0; o < kMaxOut; o++) x.E[o] = -1;
        for (int o = 2; o < kMaxOut; o++) x.dst[o] = -1;
    }
    e = hipMemcpy(d_items.p, it.data(), it.size() * sizeof(ProdItem), hipMemcpyHostToDevice);
    if (e != hipSuccess) return sfft_hip_fail(e, "tuner upload");
    const Bufs b{(uint32_t*)d_pool.p, (uint32_t*)d_out.p, nullptr, nullptr, words};

    hipEvent_t t0, t1;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess)
        return sfft_fail(SFFT_EDEVICE, "tuner events");
    int best = -1;
    double best_rate = 0;
    for (int ti = 0; ti < nt; ti++) {
        if (rates) rates[ti] = 0;
        ProdCfg cfg;
        if (!tiling_config(g, ti, &cfg)) continue;
        const ProdSeg seg{(const ProdItem*)d_items.p, b, g, cfg.nd, cfg.wd, 0, 0, (uint8_t*)d_rt.p};
        const int64_t blocks = items * product_tiles(g, cfg);
        e = launch_products(cfg, nullptr, 1, seg, blocks, items, s);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(t0, s);
        for (int r = 0; r < reps && e == hipSuccess; r++) e = launch_products(cfg, nullptr, 1, seg, blocks, items, s);
        if (e == hipSuccess) e = hipEventRecord(t1, s);
        if (e == hipSuccess) e = hipEventSynchronize(t1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
        if (e != hipSuccess) {
            (void)hipEventDestroy(t0);
            (void)hipEventDestroy(t1);
            return sfft_hip_fail(e, "tuner launch");
        }
        const double rate = (double)items * reps * std::pow((double)g.nct, 3) / (ms * 1e-3);
        if (rates) rates[ti] = rate;
        if (rate > best_rate) best_rate = rate, best = ti;
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (best < 0) return sfft_fail(SFFT_EUNSUPPORTED, "no tiling serves this geometry");
    set_tuned_tiling(g, best);
    *best_tiling = best;
    return SFFT_OK;
}

int sfft_plan_tune(sfft_plan* plan, const uint32_t* ct_in_dev, uint32_t* ct_out_dev, void* ws_dev, int64_t ws_bytes,
                   int32_t reps, int32_t* best_tiling, double* rates, void* hip_stream)
{
    if (!plan || !best_tiling || reps < 1) return sfft_fail(SFFT_EINVAL, "bad arguments");
    // the tuner is the one caller that changes a plan's launch configuration
    PlanCore* pc = const_cast<PlanCore*>(plan_core_of(plan));
    const Schedule& S = pc->sched;
    const Geo g = pc->geo;
    hipStream_t s = (hipStream_t)hip_stream;
    const int nt = tiling_count();
    if (rates)
        for (int ti = 0; ti < nt; ti++) rates[ti] = 0;
    int lv = -1;
    int64_t most = 0;
    for (size_t i = 0; i < S.levels.size(); i++)
        if (S.levels[i].prod_count > most) most = S.levels[i].prod_count, lv = (int)i;
    *best_tiling = pc->cfg.tiling;
    if (lv < 0) return SFFT_OK;
    // the plan's steps up to its widest level, so that the level's inputs
    // exist; re-running the level rewrites the same outputs (its inputs stay
    // live through it, so no output slot aliases one)
    int rc = sfft_execute_steps(plan, 0, lv + 1, ct_in_dev, ct_out_dev, ws_dev, ws_bytes, hip_stream);
    if (rc != SFFT_OK) return rc;
    const Bufs b{const_cast<uint32_t*>(ct_in_dev), ct_out_dev, (uint32_t*)ws_dev, nullptr, (int64_t)g.nct * g.W};
    hipEvent_t t0, t1;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess)
        return sfft_fail(SFFT_EDEVICE, "tuner events");
    int best = -1;
    double best_rate = 0;
    ProdCfg best_cfg{};
    for (int ti = 0; ti < nt; ti++) {
        ProdCfg cfg;
        if (!tiling_config(g, ti, &cfg)) continue;
        const ProdSeg seg{pc->d_prods + S.levels[lv].prod_begin, b, g, cfg.nd, cfg.wd, 0, 0,
                          (uint8_t*)ws_dev + pc->slot_bytes()};
        const int64_t blocks = most * product_tiles(g, cfg);
        hipError_t e = launch_products(cfg, nullptr, 1, seg, blocks, most, s);  // warm-up
        if (e == hipSuccess) e = hipEventRecord(t0, s);
        for (int r = 0; r < reps && e == hipSuccess; r++) e = launch_products(cfg, nullptr, 1, seg, blocks, most, s);
        if (e == hipSuccess) e = hipEventRecord(t1, s);
        if (e == hipSuccess) e = hipEventSynchronize(t1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
        if (e != hipSuccess) {
            (void)hipEventDestroy(t0);
            (void)hipEventDestroy(t1);
            return sfft_hip_fail(e, "plan tuner launch");
        }
        const double rate = (double)most * reps * std::pow((double)g.nct, 3) / (ms * 1e-3);
        if (rates) rates[ti] = rate;
        if (rate > best_rate) best_rate = rate, best = ti, best_cfg = cfg;
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (best < 0) return sfft_fail(SFFT_EUNSUPPORTED, "no tiling serves this geometry");
    pc->cfg = best_cfg;
    for (size_t st = 0; st < pc->step_blocks.size(); st++) {
        const int64_t prods = st < S.levels.size() ? S.levels[st].prod_count : 0;
        pc->step_blocks[st] = prods * product_tiles(g, best_cfg);
    }
    set_tuned_tiling(g, best);
    *best_tiling = best;
    return SFFT_OK;
}

}  // extern "C"
