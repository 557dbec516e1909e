// Fixed batches: a set of requests known in advance (compiled plans with
// their input, output and workspace buffers) merged level by level, as the
// request loop merges them, but compiled once.  Global step s advances every
// request that still has a step s: the product items of all of them whose
// kernel tiling and LDS occupancy class match go into one launch (one
// segment per request, each with its own geometry), then the linear passes,
// one launch per sub-pass.  Every step's segment lists are uploaded once, at
// creation, into one device table, so an execution is the launch sequence
// alone: no host work between launches and nothing to wait for.  The whole
// sequence can be captured once into a HIP graph and replayed with one
// graph launch (the buffers are fixed, so the graph stays valid).  The
// butterflies of a stage are independent (paper, section "FFT in FHE") and
// requests are independent altogether, so each request's ciphertexts equal
// those of its plan run alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "../../include/sfft.h"
#include "device.hpp"
#include "plan_internal.hpp"
#include "schedule.hpp"

using namespace sfft;

namespace {

constexpr int64_t kAlign = 256;
int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct BatchLaunch {
    bool product;
    ProdCfg cfg;          // products: the group's tiling, largest LDS of its members
    int64_t table_off;    // byte offset of the segment list in the device table
    int32_t nseg;
    ProdSeg pseg0;        // the first segment by value (used when nseg == 1)
    LinSeg lseg0;
    int64_t blocks, items;  // products: workgroups and items; linear: items
    int64_t max_elems;      // linear: the largest geometry's Nct (n + 1)
};

}  // namespace

struct sfft_batch {
    std::vector<BatchLaunch> launches;
    uint8_t* d_table = nullptr;
    int64_t steps = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    ~sfft_batch()
    {
        if (d_table) (void)hipDeviceSynchronize();  // launches in flight read the table
        if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (d_table) (void)hipFree(d_table);
    }
};

namespace {

int batch_ws_bytes(const sfft_plan* const* plans, int32_t n, int64_t* bytes)
{
    int64_t total = 0;
    for (int32_t r = 0; r < n; r++) {
        if (!plans[r]) return sfft_fail(SFFT_EINVAL, "null plan in the batch");
        total += align_up(plan_core_of(plans[r])->ws_bytes());
    }
    *bytes = total;
    return SFFT_OK;
}

hipError_t enqueue(const sfft_batch* b, hipStream_t s)
{
    for (const BatchLaunch& L : b->launches) {
        hipError_t e;
        if (L.product) {
            e = launch_products(L.cfg, (const ProdSeg*)(b->d_table + L.table_off), L.nseg, L.pseg0, L.blocks,
                                L.items, s);
        } else {
            e = launch_linear(L.max_elems, (const LinSeg*)(b->d_table + L.table_off), L.nseg, L.lseg0, L.items, s);
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

extern "C" {

int sfft_batch_workspace_bytes(const sfft_plan* const* plans, int32_t n, int64_t* bytes)
{
    if (!plans || !bytes || n < 0) return sfft_fail(SFFT_EINVAL, "null argument");
    return batch_ws_bytes(plans, n, bytes);
}

int sfft_batch_create(const sfft_plan* const* plans, const uint32_t* const* ct_in_dev, uint32_t* const* ct_out_dev,
                      int32_t n, void* ws_dev, int64_t ws_bytes, sfft_batch** out)
{
    if (!out) return sfft_fail(SFFT_EINVAL, "null batch pointer");
    *out = nullptr;
    if (!plans || !ct_in_dev || !ct_out_dev || n < 1) return sfft_fail(SFFT_EINVAL, "empty batch");
    int64_t need = 0;
    int rc = batch_ws_bytes(plans, n, &need);
    if (rc != SFFT_OK) return rc;
    if (ws_bytes < need) return sfft_fail(SFFT_EINVAL, "workspace too small: need " + std::to_string(need) + " bytes");
    if (need > 0 && !ws_dev) return sfft_fail(SFFT_EINVAL, "null workspace");
    std::vector<const PlanCore*> pcs(n);
    std::vector<Bufs> bufs(n);
    int64_t max_steps = 0, ws_off = 0;
    for (int32_t r = 0; r < n; r++) {
        const PlanCore* pc = plan_core_of(plans[r]);
        if (!ct_out_dev[r] || (pc->info.n_inputs > 0 && !ct_in_dev[r])) return sfft_fail(SFFT_EINVAL, "null buffer");
        pcs[r] = pc;
        bufs[r] = Bufs{const_cast<uint32_t*>(ct_in_dev[r]), ct_out_dev[r], (uint32_t*)((uint8_t*)ws_dev + ws_off),
                       nullptr, pc->ct_words()};
        ws_off += align_up(pc->ws_bytes());
        max_steps = std::max<int64_t>(max_steps, (int64_t)pc->sched.levels.size() + 1);
    }

    sfft_batch* bt = new (std::nothrow) sfft_batch();
    if (!bt) return sfft_fail(SFFT_ENOMEM, "out of host memory");
    std::vector<uint8_t> table;
    auto place = [&](const void* src, size_t bytes) -> int64_t {
        const int64_t at = align_up((int64_t)table.size());
        table.resize((size_t)at + bytes);
        std::memcpy(table.data() + at, src, bytes);
        return at;
    };
    struct ProdGroup {
        ProdCfg cfg;
        std::vector<ProdSeg> segs;
    };
    struct LinGroup {
        std::vector<LinSeg> segs;
        int64_t n = 0, max_elems = 0;
    };
    for (int64_t st = 0; st < max_steps; st++) {
        std::map<std::pair<int, int>, ProdGroup> pgroups;  // (8 tiling + epilogue pass rows / 16, workgroups per CU by LDS)
        std::vector<LinGroup> lgroups;
        auto add_lin = [&](size_t q, const LinItem* items, const Bufs& b, const Geo& g, int64_t count) {
            if (lgroups.size() <= q) lgroups.resize(q + 1);
            LinGroup& G = lgroups[q];
            G.segs.push_back(LinSeg{items, b, g, (uint32_t)G.n, 0});
            G.n += count;
            G.max_elems = std::max<int64_t>(G.max_elems, (int64_t)g.nct * g.n1);
        };
        for (int32_t r = 0; r < n; r++) {
            const PlanCore& pc = *pcs[r];
            const Schedule& S = pc.sched;
            if (st >= (int64_t)S.levels.size() + 1) continue;
            const Bufs& b = bufs[r];
            if (st < (int64_t)S.levels.size()) {
                const LevelWork& lw = S.levels[st];
                if (lw.prod_count) {
                    ProdGroup& G = pgroups[{8 * pc.cfg.tiling + pc.cfg.pm, 160 * 1024 / std::max(pc.cfg.lds_bytes, 1)}];
                    if (G.segs.empty()) G.cfg = pc.cfg;
                    G.cfg.lds_bytes = std::max(G.cfg.lds_bytes, pc.cfg.lds_bytes);
                    G.cfg.max_nct = std::max(G.cfg.max_nct, pc.geo.nct);
                    // first / first_block hold the item and tile counts until numbered below
                    G.segs.push_back(ProdSeg{pc.d_prods + lw.prod_begin, b, pc.geo, pc.cfg.nd, pc.cfg.wd,
                                             (uint32_t)lw.prod_count, (uint32_t)product_tiles(pc.geo, pc.cfg),
                                             (uint8_t*)b.ws + pc.slot_bytes()});
                }
                for (size_t q = 0; q < lw.lin.size(); q++)
                    add_lin(q, pc.d_lins + lw.lin[q].first, b, pc.geo, lw.lin[q].second);
            } else if (!S.final_lins.empty()) {
                add_lin(0, pc.d_final, b, pc.geo, (int64_t)S.final_lins.size());
            }
        }
        for (auto& kv : pgroups) {
            ProdGroup& G = kv.second;
            // longer workgroups (larger Nct) first, so the launch ends on short ones
            std::stable_sort(G.segs.begin(), G.segs.end(),
                             [](const ProdSeg& a, const ProdSeg& c) { return a.geo.nct > c.geo.nct; });
            int64_t items = 0, blocks = 0;
            for (ProdSeg& q : G.segs) {
                const int64_t it = q.first, tiles = q.first_block;
                q.first = (uint32_t)items;
                q.first_block = (uint32_t)blocks;
                items += it;
                blocks += it * tiles;
            }
            if (blocks > 0x7FFFFFFF) {
                delete bt;
                return sfft_fail(SFFT_EUNSUPPORTED, "a merged level exceeds one launch's workgroups");
            }
            BatchLaunch L{};
            L.product = true;
            L.cfg = G.cfg;
            L.nseg = (int32_t)G.segs.size();
            L.pseg0 = G.segs[0];
            L.blocks = blocks;
            L.items = items;
            L.table_off = place(G.segs.data(), G.segs.size() * sizeof(ProdSeg));
            bt->launches.push_back(L);
        }
        for (LinGroup& G : lgroups) {
            if (!G.n) continue;
            BatchLaunch L{};
            L.product = false;
            L.nseg = (int32_t)G.segs.size();
            L.lseg0 = G.segs[0];
            L.items = G.n;
            L.max_elems = G.max_elems;
            L.table_off = place(G.segs.data(), G.segs.size() * sizeof(LinSeg));
            bt->launches.push_back(L);
        }
    }
    bt->steps = max_steps;
    if (!table.empty()) {
        hipError_t e = hipMalloc((void**)&bt->d_table, table.size());
        if (e == hipSuccess) e = hipMemcpy(bt->d_table, table.data(), table.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            delete bt;
            return sfft_hip_fail(e, "batch table upload");
        }
    }
    *out = bt;
    return SFFT_OK;
}

int sfft_batch_info(const sfft_batch* b, int64_t* steps, int64_t* launches)
{
    if (!b || !steps || !launches) return sfft_fail(SFFT_EINVAL, "null argument");
    *steps = b->steps;
    *launches = (int64_t)b->launches.size();
    return SFFT_OK;
}

int sfft_batch_execute(const sfft_batch* b, void* hip_stream)
{
    if (!b) return sfft_fail(SFFT_EINVAL, "null batch");
    const hipError_t e = enqueue(b, (hipStream_t)hip_stream);
    return e == hipSuccess ? SFFT_OK : sfft_hip_fail(e, "batch launch");
}

int sfft_batch_execute_graph(sfft_batch* b, void* hip_stream)
{
    if (!b) return sfft_fail(SFFT_EINVAL, "null batch");
    if (!hip_stream) return sfft_fail(SFFT_EINVAL, "graph capture needs a stream other than the null stream");
    hipStream_t s = (hipStream_t)hip_stream;
    if (!b->graph_exec) {
        // the kernels' LDS caps are set once per kernel outside any capture
        // (a launch of no workgroups sets them and launches nothing)
        for (const BatchLaunch& L : b->launches) {
            if (!L.product) continue;
            const ProdSeg none{};
            const hipError_t e = launch_products(L.cfg, nullptr, 1, none, 0, 0, s);
            if (e != hipSuccess) return sfft_hip_fail(e, "batch kernel set-up");
        }
        hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return sfft_hip_fail(e, "batch capture begin");
        const hipError_t el = enqueue(b, s);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(s, &g);
        if (el != hipSuccess || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return sfft_hip_fail(el != hipSuccess ? el : e, "batch capture");
        }
        hipGraphExec_t x = nullptr;
        e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return sfft_hip_fail(e, "batch graph instantiation");
        }
        b->graph = g;
        b->graph_exec = x;
    }
    const hipError_t e = hipGraphLaunch(b->graph_exec, s);
    return e == hipSuccess ? SFFT_OK : sfft_hip_fail(e, "batch graph launch");
}

void sfft_batch_destroy(sfft_batch* b) { delete b; }

}  // extern "C"
