// Request loop: continuous batching of encrypted FFTs of different shapes.
//
// Every request runs its own compiled plan (a sequence of steps: product
// levels and the linear passes after them).  A global step advances every
// admitted request by one of its own steps; the product items of all
// requests whose kernel tiling matches go into one launch (one segment per
// request, each with its own ciphertext geometry), then the linear passes.
// Launches of different tilings within a step run concurrently on the
// server's own streams, joined before the step's linear passes.  Steps are
// enqueued without waiting for the device: a ring of segment buffers, each
// with an event, lets the host run a few steps ahead, and a request is
// retired (its workspace freed, its result reported) when the event
// recorded after its last step has completed.  Requests are admitted in
// arrival order while a workspace for their plan fits the device memory
// budget and the number of requests in flight is below the limit, so
// requests that arrive while others run join at their step 0 and overlap
// with them on the device.  The paper's FFT evaluates butterflies
// independently within each stage (section "FFT in FHE"); requests are
// independent altogether, which is what makes the interleaving exact: each
// request's ciphertexts are bit-identical alone and in the mix.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/sfft.h"
#include "device.hpp"
#include "netlist.hpp"
#include "plan_internal.hpp"
#include "schedule.hpp"

using namespace sfft;

namespace {

double now_s()
{
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over one device arena (offsets in bytes, 256-aligned).
class Arena {
public:
    void reset(int64_t size)
    {
        size_ = size;
        free_.clear();
        if (size > 0) free_[0] = size;
        used_ = peak_ = 0;
    }
    int64_t alloc(int64_t bytes)
    {
        bytes = (bytes + 255) / 256 * 256;
        if (bytes == 0) bytes = 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                const int64_t off = it->first, rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                sizes_[off] = bytes;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return off;
            }
        }
        return -1;
    }
    void release(int64_t off)
    {
        auto s = sizes_.find(off);
        if (s == sizes_.end()) return;
        int64_t bytes = s->second;
        sizes_.erase(s);
        used_ -= bytes;
        int64_t start = off;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && next->first == off + bytes) {
            bytes += next->second;
            free_.erase(next);
        }
        auto prev = free_.lower_bound(off);
        if (prev != free_.begin()) {
            --prev;
            if (prev->first + prev->second == off) {
                start = prev->first;
                bytes += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = bytes;
    }
    int64_t size() const { return size_; }
    int64_t peak() const { return peak_; }

private:
    int64_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<int64_t, int64_t> free_, sizes_;
};

struct Request {
    uint64_t ticket;
    std::shared_ptr<PlanCore> plan;
    const uint32_t* in;
    uint32_t* out;
    int64_t ws_off = -1;
    int32_t step = 0;
    int32_t waited = 0;               // steps in a row the fill policy left it out
    hipEvent_t fin = nullptr;         // recorded after its last step
    double arrival = 0, done_at = -1;
};

// A marker per request event (admitted, done), for marker traces.
void mark_request(const Request& r, const char* what)
{
    char label[96];
    std::snprintf(label, sizeof label, "sfft request %llu %s: %dD len %d F %d", (unsigned long long)r.ticket, what,
                  r.plan->shape.dims, r.plan->shape.len, r.plan->shape.F);
    roctxMarkA(label);
}

// Steps a request may be left out by the fill policy before it runs anyway.
constexpr int kMaxWait = 8;
// Segment buffers in flight (the host runs at most this many steps ahead of
// the device) and streams of a step's concurrent launches beside the caller's.
constexpr int kRing = 4;
constexpr int kAux = 3;

struct StepSlot {
    void* host = nullptr;  // pinned
    void* dev = nullptr;
    hipEvent_t done = nullptr;  // recorded after the step that used the slot
    bool busy = false;
};

}  // namespace

struct sfft_server {
    sfft_server_cfg cfg;
    bool dry = false;
    double vclock = 0;  // modelled time (dry-run)
    uint8_t* arena_dev = nullptr;
    Arena arena;
    std::map<std::string, std::shared_ptr<PlanCore>> plans;
    std::deque<std::unique_ptr<Request>> queue;
    std::vector<std::unique_ptr<Request>> active;
    std::vector<std::unique_ptr<Request>> finishing;  // every step enqueued, device not done yet
    std::map<uint64_t, std::unique_ptr<Request>> done;
    uint64_t next_ticket = 1;
    // segment staging (host pinned + device), a ring of step slots
    StepSlot ring[kRing];
    int64_t ring_next = 0;
    size_t seg_cap = 0;
    hipStream_t aux[kAux] = {};
    hipEvent_t fork = nullptr, join[kAux] = {};
    sfft_server_stats st{};
};

static std::string plan_key(const sfft_shape* s, const sfft_params* p)
{
    char buf[160];
    std::snprintf(buf, sizeof(buf), "%d/%d/%d/%d/%d/%d|%d/%d/%d/%d", s->dims, s->len, s->F, s->f, s->is_complex,
                  s->nand_only, p->n_lwe,
                  p->k, p->m, p->eta);
    return buf;
}

static double now_of(const sfft_server* sv) { return sv->dry ? sv->vclock : now_s(); }

extern "C" {

int sfft_server_create(const sfft_server_cfg* cfg, sfft_server** out)
{
    if (!cfg || !out) return sfft_fail(SFFT_EINVAL, "null argument");
    *out = nullptr;
    if (cfg->mem_budget_bytes <= 0 || cfg->max_active < 0) return sfft_fail(SFFT_EINVAL, "bad server configuration");
    auto* sv = new (std::nothrow) sfft_server();
    if (!sv) return sfft_fail(SFFT_ENOMEM, "out of host memory");
    sv->cfg = *cfg;
    sv->dry = (cfg->flags & SFFT_SERVER_DRYRUN) != 0;
    sv->arena.reset(cfg->mem_budget_bytes);
    if (!sv->dry) {
        hipError_t e = hipMalloc((void**)&sv->arena_dev, (size_t)cfg->mem_budget_bytes);
        if (e != hipSuccess) {
            delete sv;
            return sfft_fail(SFFT_ENOMEM, "cannot allocate the server's device memory budget");
        }
        sv->seg_cap = 1 << 20;  // bytes of segment lists per step
        for (StepSlot& sl : sv->ring) {
            if (e == hipSuccess) e = hipHostMalloc(&sl.host, sv->seg_cap, hipHostMallocDefault);
            if (e == hipSuccess) e = hipMalloc(&sl.dev, sv->seg_cap);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        }
        // default-priority streams that do not synchronise with the null stream
        for (int a = 0; a < kAux && e == hipSuccess; a++) {
            e = hipStreamCreateWithFlags(&sv->aux[a], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&sv->join[a], hipEventDisableTiming);
        }
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sv->fork, hipEventDisableTiming);
        if (e != hipSuccess) {
            sfft_server_destroy(sv);
            return sfft_fail(SFFT_ENOMEM, "cannot allocate segment staging, streams or events");
        }
    }
    *out = sv;
    return SFFT_OK;
}

int sfft_server_submit(sfft_server* sv, const sfft_shape* shape, const sfft_params* params,
                       const uint32_t* ct_in_dev, uint32_t* ct_out_dev, uint64_t* ticket)
{
    if (!sv || !shape || !params || !ticket) return sfft_fail(SFFT_EINVAL, "null argument");
    if (!sv->dry && (!ct_in_dev || !ct_out_dev)) return sfft_fail(SFFT_EINVAL, "null ciphertext buffer");
    const std::string key = plan_key(shape, params);
    std::shared_ptr<PlanCore> pc;
    auto it = sv->plans.find(key);
    if (it != sv->plans.end()) {
        pc = it->second;
    } else {
        pc = std::make_shared<PlanCore>();
        const int rc = plan_core_build(shape, params, !sv->dry, pc.get());
        if (rc != SFFT_OK) return rc;
        sv->plans[key] = pc;
    }
    if (pc->ws_bytes() > sv->arena.size())
        return sfft_fail(SFFT_ENOMEM, "request workspace exceeds the server's memory budget");
    auto r = std::make_unique<Request>();
    r->ticket = sv->next_ticket++;
    r->plan = pc;
    r->in = ct_in_dev;
    r->out = ct_out_dev;
    r->arrival = now_of(sv);
    *ticket = r->ticket;
    sv->queue.push_back(std::move(r));
    sv->st.submitted++;
    return SFFT_OK;
}

int sfft_server_submit_plan(sfft_server* sv, const sfft_plan* plan, const uint32_t* ct_in_dev, uint32_t* ct_out_dev,
                            uint64_t* ticket)
{
    if (!sv || !plan || !ticket) return sfft_fail(SFFT_EINVAL, "null argument");
    if (sv->dry) return sfft_fail(SFFT_EINVAL, "a dry-run server compiles its own plans (sfft_server_submit)");
    if (!ct_in_dev || !ct_out_dev) return sfft_fail(SFFT_EINVAL, "null ciphertext buffer");
    // shared with the caller, who keeps it alive: no-op deleter
    std::shared_ptr<PlanCore> pc(const_cast<PlanCore*>(plan_core_of(plan)), [](PlanCore*) {});
    if (pc->ws_bytes() > sv->arena.size())
        return sfft_fail(SFFT_ENOMEM, "request workspace exceeds the server's memory budget");
    auto r = std::make_unique<Request>();
    r->ticket = sv->next_ticket++;
    r->plan = pc;
    r->in = ct_in_dev;
    r->out = ct_out_dev;
    r->arrival = now_of(sv);
    *ticket = r->ticket;
    sv->queue.push_back(std::move(r));
    sv->st.submitted++;
    return SFFT_OK;
}

// Requests whose last step the device has finished (every one, with `all`
// after the caller's stream was synchronised): workspace back to the arena,
// results reported.
static int retire(sfft_server* sv, bool all)
{
    const double t = now_of(sv);
    std::vector<std::unique_ptr<Request>> still;
    for (auto& rp : sv->finishing) {
        bool fin = all || sv->dry || !rp->fin;
        if (!fin) {
            const hipError_t q = hipEventQuery(rp->fin);
            if (q == hipSuccess) fin = true;
            else if (q != hipErrorNotReady) return sfft_hip_fail(q, "server request completion");
        }
        if (!fin) {
            still.push_back(std::move(rp));
            continue;
        }
        if (rp->fin) (void)hipEventDestroy(rp->fin), rp->fin = nullptr;
        rp->done_at = t;
        sv->arena.release(rp->ws_off);
        rp->ws_off = -1;
        sv->st.completed++;
        sv->st.gates += rp->plan->info.gates;
        sv->st.fft_points += rp->plan->points;
        mark_request(*rp, "done");
        sv->done[rp->ticket] = std::move(rp);
    }
    sv->finishing.swap(still);
    return SFFT_OK;
}

int sfft_server_step(sfft_server* sv, void* hip_stream, int32_t* pending)
{
    if (!sv) return sfft_fail(SFFT_EINVAL, "null server");
    hipStream_t s = (hipStream_t)hip_stream;
    int rc = retire(sv, false);
    if (rc != SFFT_OK) return rc;
    // admission by workspace footprint and slot limit, in arrival order; with
    // the fill policy a request whose workspace does not fit yet lets later
    // ones that fit pass (no head-of-line blocking), lockstep keeps strict order
    for (auto it = sv->queue.begin(); it != sv->queue.end();) {
        if (sv->cfg.max_active > 0 && (int)(sv->active.size() + sv->finishing.size()) >= sv->cfg.max_active) break;
        Request* r = it->get();
        const int64_t off = sv->arena.alloc(std::max<int64_t>(r->plan->ws_bytes(), 1));
        if (off < 0) {
            if (sv->cfg.fill_blocks > 0) {
                ++it;
                continue;
            }
            break;
        }
        r->ws_off = off;
        mark_request(*r, "admitted");
        sv->active.push_back(std::move(*it));
        it = sv->queue.erase(it);
        sv->st.admitted++;
    }
    sv->st.max_active = std::max<int64_t>(sv->st.max_active, (int64_t)sv->active.size());
    sv->st.peak_ws_bytes = std::max<int64_t>(sv->st.peak_ws_bytes, sv->arena.peak());
    if (sv->active.empty()) {
        if (pending) *pending = (int32_t)(sv->queue.size() + sv->finishing.size());
        return SFFT_OK;
    }

    // This step's work: the product items of every request whose kernel
    // tiling matches go into one launch (segments may differ in k and n+1),
    // split further by how many workgroups of the launch fit a CU's 160 KB
    // of LDS (the launch allocates its largest member's LDS for every
    // workgroup, so one large member must not halve the others' occupancy);
    // the linear passes of all requests go by sub-pass index.
    struct ProdGroup {
        ProdCfg cfg;  // the shared tiling; lds_bytes = the largest any member needs
        std::vector<ProdSeg> segs;
        int64_t n = 0, blocks = 0;
    };
    struct LinGroup {
        std::vector<LinSeg> segs;
        int64_t n = 0, max_elems = 0;
    };
    std::map<std::pair<int, int>, ProdGroup> pgroups;  // (8 tiling + epilogue pass rows / 16, workgroups per CU by LDS)
    std::vector<LinGroup> lgroups;
    double model_s = 0;
    // which requests advance this step (all, or least remaining work first
    // up to fill_blocks workgroups; one left out kMaxWait steps in a row
    // runs first, so that a steady stream of small requests cannot starve it)
    std::vector<Request*> run;
    for (auto& rp : sv->active) run.push_back(rp.get());
    if (sv->cfg.fill_blocks > 0) {
        std::stable_sort(run.begin(), run.end(), [](const Request* a, const Request* b) {
            const bool wa = a->waited >= kMaxWait, wb = b->waited >= kMaxWait;
            if (wa != wb) return wa;
            return a->plan->work_from[a->step] < b->plan->work_from[b->step];
        });
        // the first request always runs; others join while the step is below
        // the target, except one whose level alone exceeds the target (it
        // would set the step's pace for all the small ones: it waits)
        std::vector<Request*> pick;
        int64_t blocks = 0;
        for (Request* q : run) {
            const int64_t qb = q->plan->step_blocks[q->step];
            if (!pick.empty() && q->waited < kMaxWait && (blocks >= sv->cfg.fill_blocks || qb > sv->cfg.fill_blocks)) {
                q->waited++;
                continue;
            }
            q->waited = 0;
            pick.push_back(q);
            blocks += qb;
        }
        run.swap(pick);
    }
    auto add_lin = [&](size_t q, const LinItem* items, const Bufs& b, const Geo& g, int64_t count) {
        if (lgroups.size() <= q) lgroups.resize(q + 1);
        LinGroup& G = lgroups[q];
        G.segs.push_back(LinSeg{items, b, g, (uint32_t)G.n, 0});
        G.n += count;
        G.max_elems = std::max<int64_t>(G.max_elems, (int64_t)g.nct * g.n1);
    };
    for (Request* r : run) {
        const PlanCore& pc = *r->plan;
        const Schedule& S = pc.sched;
        Bufs b{const_cast<uint32_t*>(r->in), r->out,
               sv->dry ? nullptr : (uint32_t*)(sv->arena_dev + r->ws_off), nullptr, pc.ct_words()};
        const int32_t st = r->step;
        if (st < (int32_t)S.levels.size()) {
            const LevelWork& lw = S.levels[st];
            if (lw.prod_count) {
                ProdGroup& G = pgroups[{8 * pc.cfg.tiling + pc.cfg.pm, 160 * 1024 / std::max(pc.cfg.lds_bytes, 1)}];
                if (G.segs.empty()) G.cfg = pc.cfg;
                G.cfg.lds_bytes = std::max(G.cfg.lds_bytes, pc.cfg.lds_bytes);
                G.cfg.max_nct = std::max(G.cfg.max_nct, pc.geo.nct);
                G.segs.push_back(ProdSeg{pc.d_prods + lw.prod_begin, b, pc.geo, pc.cfg.nd, pc.cfg.wd,
                                         (uint32_t)lw.prod_count, (uint32_t)product_tiles(pc.geo, pc.cfg),
                                         sv->dry ? nullptr : sv->arena_dev + r->ws_off + pc.slot_bytes()});
                sv->st.products += lw.prod_count;
                model_s += (double)lw.prod_count * (double)pc.geo.nct * pc.geo.nct * pc.geo.nct;
            }
            for (size_t q = 0; q < lw.lin.size(); q++) add_lin(q, pc.d_lins + lw.lin[q].first, b, pc.geo, lw.lin[q].second);
        } else if (!S.final_lins.empty()) {
            add_lin(0, pc.d_final, b, pc.geo, (int64_t)S.final_lins.size());
        }
    }

    // Within a launch, workgroups of larger Nct walk more chunks of R and run
    // longer: dispatch them first, so that the launch ends on short ones.
    // (first / first_block hold the item and tile counts until here.)
    for (auto& kv : pgroups) {
        ProdGroup& G = kv.second;
        std::stable_sort(G.segs.begin(), G.segs.end(),
                         [](const ProdSeg& a, const ProdSeg& b) { return a.geo.nct > b.geo.nct; });
        for (ProdSeg& q : G.segs) {
            const int64_t items = q.first, tiles = q.first_block;
            q.first = (uint32_t)G.n;
            q.first_block = (uint32_t)G.blocks;
            G.n += items;
            G.blocks += items * tiles;
        }
    }

    if (!sv->dry) {
        // a free slot of the ring: the step that used it last is done
        StepSlot& sl = sv->ring[sv->ring_next % kRing];
        sv->ring_next++;
        hipError_t e = hipSuccess;
        if (sl.busy) {
            e = hipEventSynchronize(sl.done);
            if (e != hipSuccess) return sfft_hip_fail(e, "server step slot");
            sl.busy = false;
        }
        // stage every segment list in one host->device copy
        size_t off = 0;
        auto place = [&](const void* src, size_t bytes) -> size_t {
            off = (off + 63) / 64 * 64;
            const size_t at = off;
            if (at + bytes > sv->seg_cap) return (size_t)-1;
            std::memcpy((uint8_t*)sl.host + at, src, bytes);
            off += bytes;
            return at;
        };
        std::vector<size_t> p_at, l_at;
        for (auto& kv : pgroups) {
            p_at.push_back(place(kv.second.segs.data(), kv.second.segs.size() * sizeof(ProdSeg)));
            if (p_at.back() == (size_t)-1) return sfft_fail(SFFT_ENOMEM, "segment staging full");
        }
        for (auto& G : lgroups) {
            l_at.push_back(place(G.segs.data(), G.segs.size() * sizeof(LinSeg)));
            if (l_at.back() == (size_t)-1) return sfft_fail(SFFT_ENOMEM, "segment staging full");
        }
        e = hipMemcpyAsync(sl.dev, sl.host, off, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return sfft_hip_fail(e, "segment upload");
        // products: the first tiling group on the caller's stream, the others
        // on the server's streams (forked after the upload, joined back
        // before the linear passes), so that their launches overlap
        // (SFFT_SERVER_SERIAL: every group on the caller's stream, in turn)
        const bool serial = (sv->cfg.flags & SFFT_SERVER_SERIAL) != 0;
        const int ng = serial ? 1 : (int)pgroups.size();
        if (ng > 1) {
            e = hipEventRecord(sv->fork, s);
            if (e != hipSuccess) return sfft_hip_fail(e, "server fork");
        }
        size_t gi = 0;
        for (auto& kv : pgroups) {
            const ProdGroup& G = kv.second;
            const int a = gi == 0 || serial ? -1 : (int)((gi - 1) % kAux);
            hipStream_t gs = a < 0 ? s : sv->aux[a];
            if (a >= 0 && gi <= (size_t)kAux) {
                e = hipStreamWaitEvent(gs, sv->fork, 0);
                if (e != hipSuccess) return sfft_hip_fail(e, "server fork wait");
            }
            e = launch_products(G.cfg, (const ProdSeg*)((uint8_t*)sl.dev + p_at[gi]), (int)G.segs.size(), G.segs[0],
                                G.blocks, G.n, gs);
            if (e != hipSuccess) return sfft_hip_fail(e, "server product launch");
            sv->st.launches++;
            gi++;
        }
        for (int a = 0; a < kAux && a + 1 < ng; a++) {
            e = hipEventRecord(sv->join[a], sv->aux[a]);
            if (e == hipSuccess) e = hipStreamWaitEvent(s, sv->join[a], 0);
            if (e != hipSuccess) return sfft_hip_fail(e, "server join");
        }
        for (size_t q = 0; q < lgroups.size(); q++) {
            const LinGroup& G = lgroups[q];
            if (!G.n) continue;
            e = launch_linear(G.max_elems, (const LinSeg*)((uint8_t*)sl.dev + l_at[q]), (int)G.segs.size(),
                              G.segs[0], G.n, s);
            if (e != hipSuccess) return sfft_hip_fail(e, "server linear launch");
            sv->st.launches++;
        }
        e = hipEventRecord(sl.done, s);
        if (e != hipSuccess) return sfft_hip_fail(e, "server step event");
        sl.busy = true;
    } else {
        const double rate = sv->cfg.dry_bitmac_per_s > 0 ? sv->cfg.dry_bitmac_per_s : 1e15;
        sv->vclock += model_s / rate + 1e-5;
    }
    sv->st.steps++;

    // advance the requests that ran; those past their last step finish when
    // the device is done with this step
    for (Request* r : run) r->step++;
    std::vector<std::unique_ptr<Request>> still;
    for (auto& rp : sv->active) {
        if (rp->step >= (int32_t)rp->plan->sched.levels.size() + 1) {
            if (!sv->dry) {
                hipError_t e = hipEventCreateWithFlags(&rp->fin, hipEventDisableTiming);
                if (e == hipSuccess) e = hipEventRecord(rp->fin, s);
                if (e != hipSuccess) return sfft_hip_fail(e, "server request event");
            }
            sv->finishing.push_back(std::move(rp));
        } else {
            still.push_back(std::move(rp));
        }
    }
    sv->active.swap(still);
    rc = retire(sv, false);
    if (rc != SFFT_OK) return rc;
    if (pending) *pending = (int32_t)(sv->active.size() + sv->queue.size() + sv->finishing.size());
    return SFFT_OK;
}

int sfft_server_poll(sfft_server* sv, uint64_t ticket, int32_t* done, double* latency_s)
{
    if (!sv || !done) return sfft_fail(SFFT_EINVAL, "null argument");
    int rc = retire(sv, false);
    if (rc != SFFT_OK) return rc;
    auto it = sv->done.find(ticket);
    if (it == sv->done.end()) {
        *done = 0;
        if (latency_s) *latency_s = -1;
        for (auto& r : sv->active)
            if (r->ticket == ticket) return SFFT_OK;
        for (auto& r : sv->finishing)
            if (r->ticket == ticket) return SFFT_OK;
        for (auto& r : sv->queue)
            if (r->ticket == ticket) return SFFT_OK;
        return sfft_fail(SFFT_EINVAL, "unknown ticket");
    }
    *done = 1;
    if (latency_s) *latency_s = it->second->done_at - it->second->arrival;
    return SFFT_OK;
}

int sfft_server_drain(sfft_server* sv, void* hip_stream)
{
    if (!sv) return sfft_fail(SFFT_EINVAL, "null server");
    int32_t pending = 1;
    while (pending > 0) {
        const size_t before = sv->active.size() + sv->queue.size() + sv->finishing.size();
        if (sv->active.empty() && sv->queue.empty()) {
            // every step enqueued: wait for the device, then retire
            if (!sv->dry) {
                const hipError_t e = hipStreamSynchronize((hipStream_t)hip_stream);
                if (e != hipSuccess) return sfft_hip_fail(e, "server drain");
            }
            return retire(sv, true);
        }
        if (sv->active.empty() && !sv->finishing.empty() && !sv->dry) {
            // nothing runs until a finishing request frees its workspace
            const hipError_t e = hipEventSynchronize(sv->finishing.front()->fin);
            if (e != hipSuccess) return sfft_hip_fail(e, "server drain");
        }
        const int rc = sfft_server_step(sv, hip_stream, &pending);
        if (rc != SFFT_OK) return rc;
        if (sv->active.empty() && sv->finishing.empty() && pending > 0 && before == (size_t)pending)
            return sfft_fail(SFFT_ENOMEM, "queued request cannot be admitted");
    }
    return SFFT_OK;
}

int sfft_server_stats_get(const sfft_server* sv, sfft_server_stats* out)
{
    if (!sv || !out) return sfft_fail(SFFT_EINVAL, "null argument");
    *out = sv->st;
    out->queued = (int64_t)sv->queue.size();
    out->active = (int64_t)(sv->active.size() + sv->finishing.size());
    out->clock_s = sv->dry ? sv->vclock : now_s();
    return SFFT_OK;
}

void sfft_server_destroy(sfft_server* sv)
{
    if (!sv) return;
    if (sv->arena_dev) (void)hipDeviceSynchronize();  // enqueued steps may still use the arena
    for (auto& rp : sv->finishing)
        if (rp->fin) (void)hipEventDestroy(rp->fin);
    for (StepSlot& sl : sv->ring) {
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.dev) (void)hipFree(sl.dev);
        if (sl.host) (void)hipHostFree(sl.host);
    }
    for (int a = 0; a < kAux; a++) {
        if (sv->join[a]) (void)hipEventDestroy(sv->join[a]);
        if (sv->aux[a]) (void)hipStreamDestroy(sv->aux[a]);
    }
    if (sv->fork) (void)hipEventDestroy(sv->fork);
    if (sv->arena_dev) (void)hipFree(sv->arena_dev);
    delete sv;
}

}  // extern "C"
