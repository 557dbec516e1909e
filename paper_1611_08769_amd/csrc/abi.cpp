// C ABI of libsfft: keys, encryption, plans, execution, decryption, gates.
#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdio>
#include <cstring>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/sfft.h"
#include "device.hpp"
#include "netlist.hpp"
#include "plan_internal.hpp"
#include "schedule.hpp"

using namespace sfft;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* where)
{
    return fail(SFFT_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

}  // namespace

int sfft_fail(int code, const std::string& msg) { return fail(code, msg); }
int sfft_hip_fail(hipError_t e, const char* where) { return hip_fail(e, where); }

namespace {

bool params_ok(const sfft_params* p, std::string* why)
{
    if (!p) { *why = "null params"; return false; }
    if (p->n_lwe < 1 || p->n_lwe > 64) { *why = "n_lwe must be in [1, 64]"; return false; }
    if (p->k <= 0 || p->k % 32 || p->k > 8192) { *why = "k must be a multiple of 32 in [32, 8192]"; return false; }
    if (p->m != (p->n_lwe + 1) * p->k) { *why = "m must equal (n_lwe+1)*k"; return false; }
    return true;
}

Geo geo_of(const sfft_params* p)
{
    Geo g;
    g.k = p->k;
    g.kw = p->k / 32;
    g.n1 = p->n_lwe + 1;
    g.nct = g.n1 * p->k;
    g.W = g.n1 * g.kw;
    return g;
}

int64_t ct_words(const Geo& g) { return (int64_t)g.nct * g.W; }

bool shape_ok(const sfft_shape* s, std::string* why)
{
    if (!s) { *why = "null shape"; return false; }
    if (s->dims != 1 && s->dims != 2) { *why = "dims must be 1 or 2"; return false; }
    if (s->len < 2 || s->len > 4096 || (s->len & (s->len - 1))) { *why = "len must be a power of two in [2, 4096]"; return false; }
    if (s->F < 1 || s->F > 32 || s->f < 0 || s->f > s->F) { *why = "need 1 <= F <= 32 and 0 <= f <= F"; return false; }
    if (s->is_complex != 0 && s->is_complex != 1) { *why = "is_complex must be 0 or 1"; return false; }
    if (s->nand_only != 0 && s->nand_only != 1) { *why = "nand_only must be 0 or 1"; return false; }
    return true;
}

Shape to_shape(const sfft_shape* s)
{
    Shape r{s->dims, s->len, s->F, s->f, s->is_complex != 0};
    r.nand_only = s->nand_only != 0;
    return r;
}

// ---- host SplitMix64 (domains: 1 t, 2 B, 3 e, 4 encryption masks) ----------
uint64_t mix64(uint64_t z)
{
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
uint64_t word64(uint64_t seed, uint64_t dom, uint64_t i) { return mix64(mix64(seed + dom * kGamma) + (i + 1) * kGamma); }

// uniform element of Z_{2^k}: ceil(k/64) words, little-endian, top word masked
void zq_element(uint64_t seed, uint64_t dom, uint64_t e, int k, uint32_t* out)
{
    const int L = (k + 63) / 64, kw = k / 32;
    for (int w = 0; w < L; w++) {
        uint64_t v = word64(seed, dom, e * (uint64_t)L + (uint64_t)w);
        const int bits = (w == L - 1) ? k - 64 * (L - 1) : 64;
        if (bits < 64) v &= (1ull << bits) - 1;
        if (2 * w < kw) out[2 * w] = (uint32_t)v;
        if (2 * w + 1 < kw) out[2 * w + 1] = (uint32_t)(v >> 32);
    }
}

int ternary(uint64_t seed, uint64_t j)
{
    const uint64_t wd = word64(seed, 3, (2 * j) / 64);
    const int s = (int)((2 * j) % 64);
    return (int)((wd >> s) & 1) - (int)((wd >> (s + 1)) & 1);
}

// r = a * b mod 2^(32 kw)
void mul_mod(const uint32_t* a, const uint32_t* b, int kw, uint32_t* r)
{
    std::vector<uint32_t> t(kw, 0);
    for (int i = 0; i < kw; i++) {
        uint64_t carry = 0;
        for (int j = 0; i + j < kw; j++) {
            const uint64_t v = (uint64_t)t[i + j] + (uint64_t)a[i] * b[j] + carry;
            t[i + j] = (uint32_t)v;
            carry = v >> 32;
        }
    }
    std::memcpy(r, t.data(), sizeof(uint32_t) * kw);
}

// r += a mod 2^(32 kw)
void add_mod(uint32_t* r, const uint32_t* a, int kw)
{
    uint64_t carry = 0;
    for (int i = 0; i < kw; i++) {
        const uint64_t v = (uint64_t)r[i] + a[i] + carry;
        r[i] = (uint32_t)v;
        carry = v >> 32;
    }
}

// r = -a mod 2^(32 kw)
void neg_mod(const uint32_t* a, int kw, uint32_t* r)
{
    uint64_t carry = 1;
    for (int i = 0; i < kw; i++) {
        const uint64_t v = (uint64_t)(~a[i]) + carry;
        r[i] = (uint32_t)v;
        carry = v >> 32;
    }
}

// decrypted bit of one ciphertext's row k-1 (n1 elements of kw limbs)
int decrypt_row(const uint32_t* row, const uint32_t* sk, int n1, int kw, int k)
{
    std::vector<uint32_t> x(kw, 0), t(kw);
    for (int b = 0; b < n1; b++) {
        mul_mod(row + b * kw, sk + b * kw, kw, t.data());
        add_mod(x.data(), t.data(), kw);
    }
    // add q/4 = 2^(k-2) and take bit k-1
    std::vector<uint32_t> quarter(kw, 0);
    quarter[(k - 2) / 32] = 1u << ((k - 2) % 32);
    add_mod(x.data(), quarter.data(), kw);
    return (int)((x[(k - 1) / 32] >> ((k - 1) % 32)) & 1u);
}

}  // namespace

// The shape checks and conversion, for the ring executor.
bool sfft_shape_check(const sfft_shape* s, std::string* why) { return shape_ok(s, why); }
Shape sfft_shape_of(const sfft_shape* s) { return to_shape(s); }

struct sfft_plan : PlanCore {};

const PlanCore* plan_core_of(const sfft_plan* plan) { return plan; }

namespace {
// Compile the circuit of a shape for params: netlist, noise check, sharing,
// lowering.  Host only.
// The plan's workspace: its slots, then one level's right operands in the
// transposition layout.
int64_t plan_ws_bytes(const Schedule& S, const Geo& g)
{
    return S.n_slots * ct_words(g) * 4 + S.max_level_products * rt_item_bytes(g);
}

// Levels within a workspace bound.  One level's transposition scratch takes
// at most an eighth of it (and at most 8192 items, plenty to fill the GPU).
// The products may run at most `window` ahead of the first one not yet run,
// in order of first appearance (for an image: a few rows, then a few
// columns, in lockstep); the widest window whose schedule fits is found by
// halving from the whole circuit, then refined by bisection.  No slot bound
// is set at first: under one, the list scheduler runs a single product per
// level whenever the live set sits at the bound; it is the last resort.
int schedule_within(const Compact& sc, const Geo& g, int64_t ws_limit, Schedule* sched)
{
    const int64_t rt = std::max<int64_t>(rt_item_bytes(g), 1);
    LiveLimit lim;
    lim.max_level_products = std::max<int64_t>(1, std::min<int64_t>(ws_limit / 8 / rt, 8192));
    int64_t products = 0;
    for (size_t v = 0; v < sc.size(); v++) products += is_product_type(sc.t[v]);
    auto fits = [&](int64_t window, Schedule* out) {
        lim.max_window = window;
        *out = lower(sc, lim);
        return plan_ws_bytes(*out, g) <= ws_limit;
    };
    int64_t hi = std::max<int64_t>(products, 1);  // the widest window tried
    if (fits(hi, sched)) return SFFT_OK;
    int64_t lo = 0;  // the widest window known to fit (0: none yet)
    Schedule best;
    while (hi > 1) {
        const int64_t w = hi / 2;
        if (fits(w, &best)) {
            lo = w;
            break;
        }
        hi = w;
    }
    if (lo == 0) {
        // no window fits: a bound on the live slots themselves (levels of
        // a single product wherever the live set sits at the bound)
        lim.max_window = 0;
        lim.max_slots = (ws_limit - lim.max_level_products * rt) / (ct_words(g) * 4);
        if (lim.max_slots > 0) {
            *sched = lower(sc, lim);
            if (plan_ws_bytes(*sched, g) <= ws_limit) return SFFT_OK;
        }
        return fail(SFFT_ENOMEM, "the circuit cannot be scheduled within a workspace of " +
                                     std::to_string(ws_limit) + " bytes");
    }
    // the widest fitting window lies in [lo, 2 lo): a few bisection steps
    for (int step = 0; step < 3 && hi - lo > 1; step++) {
        const int64_t w = lo + (hi - lo) / 2;
        Schedule s;
        if (fits(w, &s)) {
            lo = w;
            best = std::move(s);
        } else {
            hi = w;
        }
    }
    *sched = std::move(best);
    return SFFT_OK;
}

int compile_plan(const sfft_shape* shape, const sfft_params* params, Schedule* sched, sfft_plan_info* info,
                 int64_t ws_limit = 0)
{
    if (ws_limit < 0) return fail(SFFT_EINVAL, "negative workspace bound");
    std::string why;
    if (!shape_ok(shape, &why)) return fail(SFFT_EINVAL, why);
    if (!params_ok(params, &why)) return fail(SFFT_EINVAL, why);
    if (params->eta != 1) return fail(SFFT_EUNSUPPORTED, "only eta = 1 is implemented");
    try {
        const Geo geo = geo_of(params);
        const Compact c = compact(build_fft_netlist(to_shape(shape)));
        const int need = noise_bits(c, (int64_t)geo.nct);
        if (need > params->k)
            return fail(SFFT_ENOISE, "k = " + std::to_string(params->k) +
                                         " is below the circuit's noise bound (needs " + std::to_string(need) +
                                         " bits at this Nct)");
        const NetStats st = netlist_stats(c);
        if (ws_limit > 0) {
            const int rc = schedule_within(share(c), geo, ws_limit, sched);
            if (rc != SFFT_OK) return rc;
        } else {
            *sched = lower(share(c));
        }
        sfft_plan_info& in = *info;
        std::memset(&in, 0, sizeof(in));
        in.nodes = st.nodes;
        in.gates = st.gates;
        in.products = st.products;
        in.exec_products = sched->n_products;
        in.levels = (int64_t)sched->levels.size() - 1;
        in.max_level_products = sched->max_level_products;
        in.n_inputs = c.n_inputs;
        in.n_outputs = (int64_t)c.outputs.size();
        in.ws_cts = sched->n_slots;
        in.ws_bytes = plan_ws_bytes(*sched, geo);
        in.noise_bound_bits = need - 3;
        in.exec_steps = (int64_t)sched->levels.size() + 1;
        in.k_required = choose_k(c, params->n_lwe);
        for (const ProdItem& it : sched->prods) {
            in.prod_ct_reads += 2;
            for (int o = 0; o < it.nout; o++) {
                in.prod_ct_writes += 1;
                bool seen = it.E[o] < 0;
                for (int q = 0; q < o && !seen; q++) seen = it.E[q] == it.E[o];
                if (!seen) in.prod_ct_reads += 1;
            }
        }
        const std::string h = netlist_hash(c);
        std::memcpy(in.netlist_sha256, h.c_str(), 64);
        in.netlist_sha256[64] = 0;
        return SFFT_OK;
    } catch (const std::bad_alloc&) {
        return fail(SFFT_ENOMEM, "out of host memory compiling the plan");
    } catch (const std::exception& e) {
        return fail(SFFT_EINVAL, e.what());
    }
}
}  // namespace

namespace sfft {

PlanCore::~PlanCore()
{
    // work enqueued with this plan may still read its tables
    if (d_prods || d_lins || d_final || d_persist || !prod_events.empty()) (void)hipDeviceSynchronize();
    for (auto& pr : prod_events) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    if (graph_exec) (void)hipGraphExecDestroy(graph_exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (d_persist) (void)hipFree(d_persist);
    if (d_bar) (void)hipFree(d_bar);
    if (d_prods) (void)hipFree(d_prods);
    if (d_lins) (void)hipFree(d_lins);
    if (d_final) (void)hipFree(d_final);
}

int plan_core_build(const sfft_shape* shape, const sfft_params* params, bool upload, PlanCore* pl, int64_t ws_limit)
{
    const int rc = compile_plan(shape, params, &pl->sched, &pl->info, ws_limit);
    if (rc != SFFT_OK) return rc;
    pl->shape = *shape;
    pl->params = *params;
    pl->geo = geo_of(params);
    pl->points = shape->dims == 1 ? shape->len : (int64_t)shape->len * shape->len;
    if (!product_config(pl->geo, &pl->cfg)) return fail(SFFT_EUNSUPPORTED, "no kernel configuration for this geometry");
    const size_t nsteps = pl->sched.levels.size() + 1;
    pl->step_blocks.assign(nsteps, 0);
    pl->work_from.assign(nsteps + 1, 0.0);
    const double per_product = (double)pl->geo.nct * pl->geo.nct * pl->geo.nct;
    for (size_t st = nsteps; st-- > 0;) {
        const int64_t prods = st < pl->sched.levels.size() ? pl->sched.levels[st].prod_count : 0;
        pl->step_blocks[st] = prods * product_tiles(pl->geo, pl->cfg);
        pl->work_from[st] = pl->work_from[st + 1] + (double)prods * per_product;
    }
    if (!upload) return SFFT_OK;
    auto put = [&](const void* src, size_t bytes, void** dst) -> hipError_t {
        *dst = nullptr;
        if (!bytes) return hipSuccess;
        hipError_t e = hipMalloc(dst, bytes);
        if (e != hipSuccess) return e;
        return hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
    };
    hipError_t e = put(pl->sched.prods.data(), pl->sched.prods.size() * sizeof(ProdItem), (void**)&pl->d_prods);
    if (e == hipSuccess) e = put(pl->sched.lins.data(), pl->sched.lins.size() * sizeof(LinItem), (void**)&pl->d_lins);
    if (e == hipSuccess)
        e = put(pl->sched.final_lins.data(), pl->sched.final_lins.size() * sizeof(LinItem), (void**)&pl->d_final);
    if (e != hipSuccess) return hip_fail(e, "plan upload");
    return SFFT_OK;
}

}  // namespace sfft

extern "C" {

const char* sfft_last_error(void) { return g_err.c_str(); }

int sfft_size_params(const sfft_shape* shape, int32_t n_lwe, sfft_params* out)
{
    std::string why;
    if (!shape_ok(shape, &why)) return fail(SFFT_EINVAL, why);
    if (!out || n_lwe < 1 || n_lwe > 64) return fail(SFFT_EINVAL, "n_lwe must be in [1, 64]");
    try {
        const Compact c = compact(build_fft_netlist(to_shape(shape)));
        const int k = choose_k(c, n_lwe);
        if (k < 0) return fail(SFFT_ENOISE, "no k <= 8192 satisfies the noise rule");
        out->n_lwe = n_lwe;
        out->k = k;
        out->m = (n_lwe + 1) * k;
        out->eta = 1;
        return SFFT_OK;
    } catch (const std::bad_alloc&) {
        return fail(SFFT_ENOMEM, "out of host memory building the netlist");
    } catch (const std::exception& e) {
        return fail(SFFT_EINVAL, e.what());
    }
}

int64_t sfft_ct_bytes(const sfft_params* params)
{
    std::string why;
    if (!params_ok(params, &why)) return fail(SFFT_EINVAL, why);
    const int64_t nct = (int64_t)(params->n_lwe + 1) * params->k;
    return nct * nct / 8;
}

int sfft_keygen(const sfft_params* p, uint64_t seed, uint32_t* pk_host, uint32_t* sk_host)
{
    std::string why;
    if (!params_ok(p, &why)) return fail(SFFT_EINVAL, why);
    if (p->eta != 1) return fail(SFFT_EUNSUPPORTED, "only eta = 1 is implemented");
    if (!pk_host || !sk_host) return fail(SFFT_EINVAL, "null key buffer");
    const Geo g = geo_of(p);
    const int n = p->n_lwe, kw = g.kw, k = p->k, m = p->m;
    std::vector<uint32_t> t((size_t)n * kw);
    for (int i = 0; i < n; i++) zq_element(seed, 1, (uint64_t)i, k, &t[(size_t)i * kw]);
    // s = (1, -t)
    std::memset(sk_host, 0, sizeof(uint32_t) * (size_t)g.n1 * kw);
    sk_host[0] = 1;
    for (int i = 0; i < n; i++) neg_mod(&t[(size_t)i * kw], kw, sk_host + (size_t)(i + 1) * kw);
    // A = [B t + e | B], row-major m x (n+1)
    std::vector<uint32_t> prod(kw), minus1(kw, 0xFFFFFFFFu), one(kw, 0);
    one[0] = 1;
    for (int j = 0; j < m; j++) {
        uint32_t* row = pk_host + (size_t)j * g.n1 * kw;
        std::memset(row, 0, sizeof(uint32_t) * kw);
        for (int i = 0; i < n; i++) {
            uint32_t* Bji = row + (size_t)(i + 1) * kw;
            zq_element(seed, 2, (uint64_t)j * n + i, k, Bji);
            mul_mod(Bji, &t[(size_t)i * kw], kw, prod.data());
            add_mod(row, prod.data(), kw);
        }
        const int e = ternary(seed, (uint64_t)j);
        if (e == 1) add_mod(row, one.data(), kw);
        if (e == -1) add_mod(row, minus1.data(), kw);
    }
    return SFFT_OK;
}

int sfft_encrypt(const sfft_params* p, const uint32_t* pk_dev, const int32_t* fixed_host, int64_t n_values,
                 int32_t F, uint64_t seed, uint64_t first_ct_id, uint32_t* ct_dev, void* hip_stream)
{
    std::string why;
    if (!params_ok(p, &why)) return fail(SFFT_EINVAL, why);
    if (p->eta != 1) return fail(SFFT_EUNSUPPORTED, "only eta = 1 is implemented");
    if (F < 1 || F > 32 || n_values < 0) return fail(SFFT_EINVAL, "bad F or n_values");
    if (n_values > 0 && (!pk_dev || !fixed_host || !ct_dev)) return fail(SFFT_EINVAL, "null buffer");
    const Geo g = geo_of(p);
    ProdCfg cfg;
    if (!product_config(g, &cfg)) return fail(SFFT_EUNSUPPORTED, "no kernel configuration for this geometry");
    const int64_t n_ct = n_values * F;
    std::vector<uint32_t> bits(kMaxEncPerLaunch / 32);
    Bufs b{nullptr, nullptr, nullptr, const_cast<uint32_t*>(pk_dev), ct_words(g)};
    for (int64_t c0 = 0; c0 < n_ct; c0 += kMaxEncPerLaunch) {
        const int64_t cnt = std::min<int64_t>(kMaxEncPerLaunch, n_ct - c0);
        std::fill(bits.begin(), bits.end(), 0u);
        for (int64_t i = 0; i < cnt; i++) {
            const int64_t c = c0 + i;
            const uint32_t u = (uint32_t)fixed_host[c / F];
            if ((u >> (c % F)) & 1u) bits[i / 32] |= 1u << (i % 32);
        }
        b.out = ct_dev + c0 * ct_words(g);
        hipError_t e = launch_encrypt(b, g, cfg, bits.data(), (int)cnt, seed, first_ct_id + (uint64_t)c0,
                                      (hipStream_t)hip_stream);
        if (e != hipSuccess) return hip_fail(e, "encrypt launch");
    }
    return SFFT_OK;
}


int sfft_analyze(const sfft_shape* shape, const sfft_params* params, sfft_plan_info* info)
{
    if (!info) return fail(SFFT_EINVAL, "null info");
    Schedule sched;
    return compile_plan(shape, params, &sched, info);
}

int sfft_analyze_bounded(const sfft_shape* shape, const sfft_params* params, int64_t ws_limit_bytes,
                         sfft_plan_info* info)
{
    if (!info) return fail(SFFT_EINVAL, "null info");
    Schedule sched;
    return compile_plan(shape, params, &sched, info, ws_limit_bytes);
}

int sfft_plan_create(const sfft_shape* shape, const sfft_params* params, sfft_plan** out)
{
    return sfft_plan_create_bounded(shape, params, 0, out);
}

int sfft_plan_create_bounded(const sfft_shape* shape, const sfft_params* params, int64_t ws_limit_bytes,
                             sfft_plan** out)
{
    if (!out) return fail(SFFT_EINVAL, "null plan pointer");
    *out = nullptr;
    sfft_plan* pl = new (std::nothrow) sfft_plan();
    if (!pl) return fail(SFFT_ENOMEM, "out of host memory");
    const int rc = plan_core_build(shape, params, true, pl, ws_limit_bytes);
    if (rc != SFFT_OK) {
        delete pl;
        return rc;
    }
    *out = pl;
    return SFFT_OK;
}

int sfft_plan_info_get(const sfft_plan* plan, sfft_plan_info* info)
{
    if (!plan || !info) return fail(SFFT_EINVAL, "null argument");
    *info = plan->info;
    info->tiling = plan->cfg.tiling;
    return SFFT_OK;
}

int sfft_plan_workspace_bytes(const sfft_plan* plan, int64_t* bytes)
{
    if (!plan || !bytes) return fail(SFFT_EINVAL, "null argument");
    *bytes = plan->ws_bytes();
    return SFFT_OK;
}

void sfft_plan_destroy(sfft_plan* plan) { delete plan; }

int sfft_execute_steps(const sfft_plan* plan, int32_t first, int32_t count, const uint32_t* ct_in_dev,
                       uint32_t* ct_out_dev, void* ws_dev, int64_t ws_bytes, void* hip_stream)
{
    if (!plan) return fail(SFFT_EINVAL, "null plan");
    const Schedule& S = plan->sched;
    const int32_t nsteps = (int32_t)S.levels.size() + 1;
    if (first < 0 || count < 0 || first + count > nsteps) return fail(SFFT_EINVAL, "step range out of bounds");
    int64_t need = 0;
    sfft_plan_workspace_bytes(plan, &need);
    if (ws_bytes < need) return fail(SFFT_EINVAL, "workspace too small: need " + std::to_string(need) + " bytes");
    if (!ct_out_dev || (plan->info.n_inputs > 0 && !ct_in_dev) || (need > 0 && !ws_dev))
        return fail(SFFT_EINVAL, "null buffer");
    const Geo& g = plan->geo;
    Bufs b{const_cast<uint32_t*>(ct_in_dev), ct_out_dev, (uint32_t*)ws_dev, nullptr, ct_words(g)};
    hipStream_t s = (hipStream_t)hip_stream;
    for (int32_t st = first; st < first + count; st++) {
        // a host range per step (its launches being enqueued), for marker traces
        char label[64];
        std::snprintf(label, sizeof label, "sfft level %d: %lld products", st,
                      st < (int32_t)S.levels.size() ? (long long)S.levels[st].prod_count : 0ll);
        roctxRangePushA(label);
        struct PopRange {
            ~PopRange() { roctxRangePop(); }
        } pop_range;
        if (st < (int32_t)S.levels.size()) {
            const LevelWork& lw = S.levels[st];
            if (lw.prod_count) {
                const ProdSeg seg{plan->d_prods + lw.prod_begin, b, g, plan->cfg.nd, plan->cfg.wd, 0, 0,
                                  (uint8_t*)ws_dev + plan->slot_bytes()};
                std::pair<hipEvent_t, hipEvent_t> ev{nullptr, nullptr};
                if (plan->time_products) {
                    hipError_t e = hipEventCreate(&ev.first);
                    if (e == hipSuccess) e = hipEventCreate(&ev.second);
                    if (e != hipSuccess) {
                        if (ev.first) (void)hipEventDestroy(ev.first);
                        return hip_fail(e, "timing events");
                    }
                    plan->prod_events.push_back(ev);
                }
                hipError_t e = launch_products(plan->cfg, nullptr, 1, seg,
                                               (int64_t)lw.prod_count * product_tiles(g, plan->cfg), lw.prod_count, s,
                                               ev.first);
                if (e != hipSuccess) return hip_fail(e, "product launch");
                if (ev.second && (e = hipEventRecord(ev.second, s)) != hipSuccess) return hip_fail(e, "timing event");
            }
            for (const auto& pass : lw.lin) {
                const LinSeg seg{plan->d_lins + pass.first, b, g, 0, 0};
                hipError_t e = launch_linear((int64_t)g.nct * g.n1, nullptr, 1, seg, pass.second, s);
                if (e != hipSuccess) return hip_fail(e, "linear launch");
            }
        } else if (!S.final_lins.empty()) {
            const LinSeg seg{plan->d_final, b, g, 0, 0};
            hipError_t e = launch_linear((int64_t)g.nct * g.n1, nullptr, 1, seg, (int64_t)S.final_lins.size(), s);
            if (e != hipSuccess) return hip_fail(e, "output launch");
        }
    }
    return SFFT_OK;
}

int sfft_execute(const sfft_plan* plan, const uint32_t* ct_in_dev, uint32_t* ct_out_dev, void* ws_dev,
                 int64_t ws_bytes, void* hip_stream)
{
    if (!plan) return fail(SFFT_EINVAL, "null plan");
    return sfft_execute_steps(plan, 0, (int32_t)plan->sched.levels.size() + 1, ct_in_dev, ct_out_dev, ws_dev,
                              ws_bytes, hip_stream);
}

int sfft_execute_graph(sfft_plan* plan, const uint32_t* ct_in_dev, uint32_t* ct_out_dev, void* ws_dev,
                       int64_t ws_bytes, void* hip_stream)
{
    if (!plan) return fail(SFFT_EINVAL, "null plan");
    if (!hip_stream) return fail(SFFT_EINVAL, "graph capture needs a stream other than the null stream");
    hipStream_t s = (hipStream_t)hip_stream;
    if (!plan->graph_exec || plan->graph_in != ct_in_dev || plan->graph_out != ct_out_dev || plan->graph_ws != ws_dev) {
        if (plan->graph_exec) (void)hipGraphExecDestroy(plan->graph_exec);
        if (plan->graph) (void)hipGraphDestroy(plan->graph);
        plan->graph_exec = nullptr;
        plan->graph = nullptr;
        // set the kernel's LDS attribute outside the capture (a launch of
        // no workgroups does only that)
        const ProdSeg none{nullptr, Bufs{}, plan->geo, plan->cfg.nd, plan->cfg.wd, 0, 0, nullptr};
        hipError_t e = launch_products(plan->cfg, nullptr, 1, none, 0, 0, s);
        if (e != hipSuccess) return hip_fail(e, "graph preparation");
        e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "graph capture");
        const int rc = sfft_execute(plan, ct_in_dev, ct_out_dev, ws_dev, ws_bytes, hip_stream);
        hipGraph_t g = nullptr;
        e = hipStreamEndCapture(s, &g);
        if (rc != SFFT_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return hip_fail(e, "graph capture");
        e = hipGraphInstantiate(&plan->graph_exec, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(g);
            return hip_fail(e, "graph instantiation");
        }
        plan->graph = g;
        plan->graph_in = ct_in_dev;
        plan->graph_out = ct_out_dev;
        plan->graph_ws = ws_dev;
    }
    hipError_t e = hipGraphLaunch(plan->graph_exec, s);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return SFFT_OK;
}

int sfft_execute_persistent(sfft_plan* plan, const uint32_t* ct_in_dev, uint32_t* ct_out_dev, void* ws_dev,
                            int64_t ws_bytes, void* hip_stream)
{
    if (!plan) return fail(SFFT_EINVAL, "null plan");
    int64_t need = 0;
    sfft_plan_workspace_bytes(plan, &need);
    if (ws_bytes < need) return fail(SFFT_EINVAL, "workspace too small: need " + std::to_string(need) + " bytes");
    if (!ct_out_dev || (plan->info.n_inputs > 0 && !ct_in_dev) || (need > 0 && !ws_dev))
        return fail(SFFT_EINVAL, "null buffer");
    const Geo& g = plan->geo;
    ProdCfg cfg{};
    if (!persistent_config(g, &cfg))
        return fail(SFFT_EUNSUPPORTED, "no persistent kernel for this geometry (rows of more than 8 fragments)");
    const Schedule& S = plan->sched;
    const int64_t nl = (int64_t)S.levels.size();
    if (!plan->d_persist) {
        std::vector<int64_t> t(4 * nl);
        std::vector<int64_t> passes;
        for (int64_t L = 0; L < nl; L++) {
            const LevelWork& lw = S.levels[L];
            t[4 * L] = lw.prod_begin;
            t[4 * L + 1] = lw.prod_count;
            t[4 * L + 2] = (int64_t)passes.size() / 2;
            t[4 * L + 3] = (int64_t)lw.lin.size();
            for (const auto& pr : lw.lin) {
                passes.push_back(pr.first);
                passes.push_back(pr.second);
            }
        }
        t.insert(t.end(), passes.begin(), passes.end());
        int64_t* d = nullptr;
        uint32_t* bar = nullptr;
        hipError_t e = hipMalloc((void**)&d, sizeof(int64_t) * std::max<size_t>(t.size(), 1));
        if (e == hipSuccess && !t.empty()) e = hipMemcpy(d, t.data(), sizeof(int64_t) * t.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMalloc((void**)&bar, 2 * sizeof(uint32_t));
        if (e != hipSuccess) {
            if (d) (void)hipFree(d);
            return hip_fail(e, "persistent tables");
        }
        plan->d_persist = d;
        plan->d_bar = bar;
    }
    PersistArgs a{};
    a.prods = plan->d_prods;
    a.lins = plan->d_lins;
    a.finals = plan->d_final;
    a.lv = plan->d_persist;
    a.pass = plan->d_persist + 4 * nl;
    a.nlevels = (int32_t)nl;
    a.nfinal = (int32_t)S.final_lins.size();
    a.bufs = Bufs{const_cast<uint32_t*>(ct_in_dev), ct_out_dev, (uint32_t*)ws_dev, nullptr, ct_words(g)};
    a.geo = g;
    a.nd = cfg.nd;
    a.wd = cfg.wd;
    a.tiles = (uint32_t)product_tiles(g, cfg);
    a.bar = plan->d_bar;
    // enough workgroups for the widest level's tiles and its linear tasks
    int64_t widest = 1;
    for (const LevelWork& lw : S.levels) {
        widest = std::max<int64_t>(widest, lw.prod_count * a.tiles);
        for (const auto& pr : lw.lin)
            widest = std::max<int64_t>(widest, (pr.second * g.nct * g.n1 + cfg.threads - 1) / cfg.threads);
    }
    widest = std::max<int64_t>(widest, ((int64_t)S.final_lins.size() * g.nct * g.n1 + cfg.threads - 1) / cfg.threads);
    const hipError_t e = launch_plan_persistent(a, cfg, widest, (hipStream_t)hip_stream);
    return e == hipSuccess ? SFFT_OK : hip_fail(e, "persistent launch");
}

int sfft_plan_persistent_timeouts(sfft_plan* plan, int32_t* flag)
{
    if (!plan || !flag) return fail(SFFT_EINVAL, "null argument");
    *flag = 0;
    if (!plan->d_bar) return SFFT_OK;
    uint32_t w[2] = {0, 0};
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(w, plan->d_bar, sizeof w, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(e, "persistent status");
    *flag = (int32_t)w[1];
    return SFFT_OK;
}

int sfft_plan_time_products(sfft_plan* plan, int32_t enable)
{
    if (!plan) return fail(SFFT_EINVAL, "null plan");
    plan->time_products = enable != 0;
    return SFFT_OK;
}

int sfft_plan_product_time(sfft_plan* plan, double* total_ms, int64_t* launches)
{
    if (!plan || !total_ms || !launches) return fail(SFFT_EINVAL, "null argument");
    double sum = 0.0;
    hipError_t err = hipSuccess;
    for (auto& pr : plan->prod_events) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(pr.second);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, pr.first, pr.second);
        if (e != hipSuccess && err == hipSuccess) err = e;
        sum += ms;
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
    }
    *launches = (int64_t)plan->prod_events.size();
    *total_ms = sum;
    plan->prod_events.clear();
    if (err != hipSuccess) return hip_fail(err, "product timing");
    return SFFT_OK;
}

int sfft_plan_step_products(const sfft_plan* plan, int64_t* counts, int32_t n)
{
    if (!plan || (n > 0 && !counts)) return fail(SFFT_EINVAL, "null argument");
    const Schedule& S = plan->sched;
    const int32_t nsteps = (int32_t)S.levels.size() + 1;
    if (n != nsteps) return fail(SFFT_EINVAL, "need exactly exec_steps entries");
    for (int32_t st = 0; st < nsteps; st++) counts[st] = st < (int32_t)S.levels.size() ? S.levels[st].prod_count : 0;
    return SFFT_OK;
}

}  // extern "C"

namespace {
// Bits of n_ct ciphertexts (host, or device: row k-1 of each copied to the
// host, on the null stream or, with on_stream, on hip_stream alone).
int decrypt_bits_impl(const sfft_params* p, const uint32_t* sk_host, const uint32_t* ct, int64_t n_ct,
                      int ct_on_device, bool on_stream, void* hip_stream, int32_t* bits_out)
{
    std::string why;
    if (!params_ok(p, &why)) return fail(SFFT_EINVAL, why);
    if (n_ct < 0 || (n_ct > 0 && (!sk_host || !ct || !bits_out))) return fail(SFFT_EINVAL, "bad buffers");
    const Geo g = geo_of(p);
    const int64_t cw = ct_words(g);
    const size_t row_off = (size_t)(p->k - 1) * g.W;
    std::vector<uint32_t> rows;
    const uint32_t* src = ct;
    int64_t stride = cw;
    if (ct_on_device && n_ct > 0) {
        rows.resize((size_t)n_ct * g.W);
        // the rows gathered on the device into a stream-ordered buffer, then
        // one linear copy to the host and a wait for the stream (the null
        // stream unless one is given).  A strided 2D copy to pageable memory
        // on the null stream returned wrong words under a kernel-tracing
        // profiler while the device data was right; this form does not
        // depend on the runtime's 2D copy.
        const hipStream_t s = on_stream ? (hipStream_t)hip_stream : nullptr;
        const size_t bytes = sizeof(uint32_t) * rows.size();
        uint32_t* d_rows = nullptr;
        hipError_t e = hipMallocAsync((void**)&d_rows, bytes, s);
        if (e == hipSuccess) e = launch_gather_rows(ct, cw, (int64_t)row_off, g.W, n_ct, d_rows, s);
        if (e == hipSuccess) e = hipMemcpyAsync(rows.data(), d_rows, bytes, hipMemcpyDeviceToHost, s);
        if (d_rows) {
            const hipError_t ef = hipFreeAsync(d_rows, s);
            if (e == hipSuccess) e = ef;
        }
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "decrypt copy");
        src = rows.data();
        stride = g.W;
    } else {
        src = ct + row_off;
    }
    for (int64_t i = 0; i < n_ct; i++) bits_out[i] = decrypt_row(src + i * stride, sk_host, g.n1, g.kw, p->k);
    return SFFT_OK;
}

int decrypt_impl(const sfft_params* p, const uint32_t* sk_host, const uint32_t* ct, int64_t n_values, int32_t F,
                 int ct_on_device, bool on_stream, void* hip_stream, int32_t* fixed_out)
{
    if (F < 1 || F > 32 || n_values < 0) return fail(SFFT_EINVAL, "bad F or n_values");
    if (n_values > 0 && !fixed_out) return fail(SFFT_EINVAL, "null output");
    std::vector<int32_t> bits((size_t)(n_values * F));
    const int rc = decrypt_bits_impl(p, sk_host, ct, n_values * F, ct_on_device, on_stream, hip_stream, bits.data());
    if (rc != SFFT_OK) return rc;
    for (int64_t v = 0; v < n_values; v++) {
        uint32_t u = 0;
        for (int i = 0; i < F; i++) u |= (uint32_t)(bits[(size_t)(v * F + i)] & 1) << i;
        if (F < 32 && (u >> (F - 1)) & 1u) u |= ~0u << F;  // sign-extend
        fixed_out[v] = (int32_t)u;
    }
    return SFFT_OK;
}
}  // namespace

extern "C" {

int sfft_decrypt_bits(const sfft_params* p, const uint32_t* sk_host, const uint32_t* ct, int64_t n_ct,
                      int ct_on_device, int32_t* bits_out)
{
    return decrypt_bits_impl(p, sk_host, ct, n_ct, ct_on_device, false, nullptr, bits_out);
}

int sfft_decrypt(const sfft_params* p, const uint32_t* sk_host, const uint32_t* ct, int64_t n_values, int32_t F,
                 int ct_on_device, int32_t* fixed_out)
{
    return decrypt_impl(p, sk_host, ct, n_values, F, ct_on_device, false, nullptr, fixed_out);
}

int sfft_decrypt_stream(const sfft_params* p, const uint32_t* sk_host, const uint32_t* ct_dev, int64_t n_values,
                        int32_t F, void* hip_stream, int32_t* fixed_out)
{
    return decrypt_impl(p, sk_host, ct_dev, n_values, F, 1, true, hip_stream, fixed_out);
}

int sfft_noise_bits(const sfft_params* p, const uint32_t* sk_host, const uint32_t* ct_dev, int64_t n_ct,
                    const int32_t* mu_bits, void* hip_stream, int32_t* max_bits)
{
    std::string why;
    if (!params_ok(p, &why)) return fail(SFFT_EINVAL, why);
    if (!max_bits || n_ct < 0 || (n_ct > 0 && (!sk_host || !ct_dev || !mu_bits))) return fail(SFFT_EINVAL, "bad buffers");
    const Geo g = geo_of(p);
    const int kw = g.kw, n1 = g.n1;
    const int64_t cw = ct_words(g);
    std::vector<uint32_t> ct((size_t)cw), x(kw), t(kw), e(kw);
    const hipStream_t s = (hipStream_t)hip_stream;
    int worst = 0;
    for (int64_t c = 0; c < n_ct; c++) {
        hipError_t err = hipMemcpyAsync(ct.data(), ct_dev + c * cw, sizeof(uint32_t) * cw, hipMemcpyDeviceToHost, s);
        if (err == hipSuccess) err = hipStreamSynchronize(s);
        if (err != hipSuccess) return hip_fail(err, "noise copy");
        for (int r = 0; r < g.nct; r++) {
            const uint32_t* row = ct.data() + (size_t)r * g.W;
            std::fill(x.begin(), x.end(), 0u);
            for (int b = 0; b < n1; b++) {
                mul_mod(row + b * kw, sk_host + b * kw, kw, t.data());
                add_mod(x.data(), t.data(), kw);
            }
            if (mu_bits[c] & 1) {
                // - 2^t s_b: s_b shifted left by t bits mod 2^k, negated, added
                const int b = r / p->k, sh = r % p->k, ls = sh / 32, bs = sh % 32;
                std::fill(e.begin(), e.end(), 0u);
                const uint32_t* sb = sk_host + b * kw;
                for (int i = kw - 1; i >= ls; i--) {
                    const uint64_t hi = (uint64_t)sb[i - ls] << bs;
                    const uint64_t lo = (i - ls - 1 >= 0 && bs) ? (uint64_t)sb[i - ls - 1] >> (32 - bs) : 0;
                    e[i] = (uint32_t)(hi | lo);
                }
                neg_mod(e.data(), kw, t.data());
                add_mod(x.data(), t.data(), kw);
            }
            // centred: values with the top bit set stand for x - 2^k
            if (x[kw - 1] >> 31) {
                neg_mod(x.data(), kw, t.data());
                x = t;
            }
            int bits = 0;
            for (int i = kw - 1; i >= 0 && !bits; i--)
                if (x[i]) bits = 32 * i + (32 - __builtin_clz(x[i]));
            worst = std::max(worst, bits);
        }
    }
    *max_bits = worst;
    return SFFT_OK;
}

}  // extern "C"

// One gate.  A transposition-pass tiling is replaced by its in-kernel twin,
// so no scratch is needed and nothing is allocated.
static int gate_impl(const sfft_params* p, int32_t gate, const uint32_t* x_dev, const uint32_t* y_dev,
                     uint32_t* out_dev, void* hip_stream)
{
    std::string why;
    if (!params_ok(p, &why)) return fail(SFFT_EINVAL, why);
    if (!x_dev || !out_dev || (gate != 3 && !y_dev)) return fail(SFFT_EINVAL, "null buffer");
    if (gate < 3 || gate > 9) return fail(SFFT_EINVAL, "gate must be 3..9");
    const Geo g = geo_of(p);
    Bufs b{const_cast<uint32_t*>(x_dev), out_dev, nullptr, const_cast<uint32_t*>(y_dev), ct_words(g)};
    hipStream_t s = (hipStream_t)hip_stream;
    hipError_t e;
    if (gate == 3 || gate == 7) {
        LinItem li{};
        li.dst = ct_ref(B_OUT, 0);
        li.X = ct_ref(B_IN, 0);
        if (gate == 3) {
            li.Y = -1;
            li.cX = -1;
            li.cG = 1;
        } else {
            li.Y = ct_ref(B_AUX, 0);
            li.cX = 1;
            li.cY = 1;
        }
        e = launch_linear_one(b, g, li, s);
    } else {
        ProdCfg cfg;
        if (!product_config(g, &cfg)) return fail(SFFT_EUNSUPPORTED, "no kernel configuration for this geometry");
        ProdItem it{};
        it.L = ct_ref(B_IN, 0);
        it.R = ct_ref(B_AUX, 0);
        it.nout = 1;
        it.dst[0] = ct_ref(B_OUT, 0);
        it.E[0] = -1;
        for (int i = 1; i < kMaxOut; i++) it.dst[i] = it.E[i] = -1;
        switch (gate) {
        case 4: case 9: it.cP[0] = 1; break;
        case 5: it.cL[0] = 1; it.cR[0] = 1; it.cP[0] = -2; break;
        case 6: it.cL[0] = 1; it.cR[0] = 1; it.cP[0] = -1; break;
        case 8: it.cP[0] = -1; it.cG[0] = 1; break;
        }
        if (!inkernel_twin(g, &cfg)) return fail(SFFT_EUNSUPPORTED, "no kernel configuration for this geometry");
        e = launch_product_one(b, g, cfg, it, nullptr, s);
    }
    if (e != hipSuccess) return hip_fail(e, "gate launch");
    return SFFT_OK;
}

extern "C" {

int sfft_gate(const sfft_params* p, int32_t gate, const uint32_t* x_dev, const uint32_t* y_dev, uint32_t* out_dev,
              void* hip_stream)
{
    return gate_impl(p, gate, x_dev, y_dev, out_dev, hip_stream);
}


}  // extern "C"
