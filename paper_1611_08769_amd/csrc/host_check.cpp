// Host-only self-check of the netlist builder and the lowering, meant to be
// compiled with g++ under AddressSanitizer and UndefinedBehaviorSanitizer
// (no HIP, no device): it builds the FFT netlist of several shapes, runs
// dead-code elimination, sharing, hashing, statistics and the modulus rule,
// lowers each to its schedule (as soon as possible, and under live-set
// bounds by list scheduling), and evaluates the schedules on plaintext bits
// (P = L AND R, every output form a L + b R + c P + g + e E) level by level
// with the levels' parallel semantics: a level's items all read before any
// writes.  Every output form must give 0 or 1, nothing may read a slot that
// holds no value, and the outputs must equal a direct evaluation of the
// netlist (paper, Lemma "evaluation": the circuit of gates computes the
// plaintext function).  Exit status 0 on success; with the argument "plant"
// one coefficient of the schedule is corrupted first and the status is 0
// only if the check catches it.
//
//   g++ -std=c++17 -O1 -g -fsanitize=address,undefined -fno-sanitize-recover=all \
//       host_check.cpp netlist.cpp schedule.cpp -o host_check && ./host_check
#include <cstdio>
#include <cstdlib>
#include <stdexcept>
#include <string>
#include <vector>

#include "netlist.hpp"
#include "schedule.hpp"

using namespace sfft;

namespace {

uint64_t g_state = 0x9E3779B97F4A7C15ull;
int next_bit()
{
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return (int)(g_state >> 63);
}

void check(bool ok, const std::string& what)
{
    if (!ok) throw std::runtime_error(what);
}

std::vector<int> eval_netlist(const Compact& c, const std::vector<int>& in)
{
    std::vector<int> v(c.size(), -1);
    for (size_t i = 0; i < c.size(); i++) {
        const int x = c.a[i] >= 0 && c.t[i] != T_IN ? v[c.a[i]] : 0;
        const int y = c.b[i] >= 0 ? v[c.b[i]] : 0;
        switch (c.t[i]) {
        case T_IN: v[i] = in.at(c.a[i]); break;
        case T_C0: v[i] = 0; break;
        case T_C1: v[i] = 1; break;
        case T_NOT: v[i] = 1 - x; break;
        case T_AND: v[i] = x & y; break;
        case T_XOR: v[i] = x ^ y; break;
        case T_OR: v[i] = x | y; break;
        case T_XADD: check(x + y <= 1, "XADD of two ones"); v[i] = x + y; break;
        case T_NAND: v[i] = 1 - (x & y); break;
        default: check(false, "bad node type");
        }
    }
    std::vector<int> out;
    for (int32_t o : c.outputs) out.push_back(v.at(o));
    return out;
}

struct Store {
    std::vector<int> in, out, ws;
    int& at(int32_t ref)
    {
        const uint32_t buf = (uint32_t)ref >> 29, idx = (uint32_t)ref & ((1u << 29) - 1);
        std::vector<int>* v = buf == B_IN ? &in : buf == B_OUT ? &out : buf == B_WS ? &ws : nullptr;
        check(v != nullptr && idx < v->size(), "reference out of range");
        return (*v)[idx];
    }
    int read(int32_t ref)
    {
        const int x = at(ref);
        check(x == 0 || x == 1, "read of a location that holds no bit");
        return x;
    }
};

void run_lins(Store& st, const LinItem* it, int64_t n)
{
    std::vector<std::pair<int32_t, int>> writes;
    for (int64_t i = 0; i < n; i++) {
        const LinItem& li = it[i];
        const int x = li.X >= 0 ? st.read(li.X) : 0, y = li.Y >= 0 ? st.read(li.Y) : 0;
        const int v = li.cX * x + li.cY * y + li.cG;
        check(v == 0 || v == 1, "linear form outside {0,1}");
        writes.push_back({li.dst, v});
    }
    for (auto& w : writes) st.at(w.first) = w.second;
}

std::vector<int> eval_schedule(const Schedule& S, const Compact& c, const std::vector<int>& in)
{
    Store st;
    st.in = in;
    st.out.assign(c.outputs.size(), -1);
    st.ws.assign((size_t)S.n_slots, -1);
    for (size_t lv = 0; lv < S.levels.size(); lv++) {
        const LevelWork& lw = S.levels[lv];
        check(lw.prod_begin >= 0 && lw.prod_begin + lw.prod_count <= (int64_t)S.prods.size(), "level range");
        std::vector<std::pair<int32_t, int>> writes;
        for (int64_t i = lw.prod_begin; i < lw.prod_begin + lw.prod_count; i++) {
            const ProdItem& it = S.prods[(size_t)i];
            check(it.nout >= 1 && it.nout <= kMaxOut, "product outputs");
            const int L = st.read(it.L), R = st.read(it.R), P = L & R;
            int distinct_e = 0;
            for (int o = 0; o < it.nout; o++) {
                bool seen = it.E[o] < 0;
                for (int q = 0; q < o && !seen; q++) seen = it.E[q] == it.E[o];
                distinct_e += !seen;
                const int e = it.E[o] >= 0 ? st.read(it.E[o]) : 0;
                const int v = it.cL[o] * L + it.cR[o] * R + it.cP[o] * P + it.cG[o] + it.cE[o] * e;
                check(v == 0 || v == 1, "epilogue form outside {0,1}");
                writes.push_back({it.dst[o], v});
            }
            check(distinct_e <= kMaxE, "more distinct extra operands than an item carries");
        }
        for (auto& w : writes) st.at(w.first) = w.second;
        for (const auto& pass : lw.lin) {
            check(pass.first >= 0 && pass.first + pass.second <= (int64_t)S.lins.size(), "linear pass range");
            run_lins(st, S.lins.data() + pass.first, pass.second);
        }
    }
    run_lins(st, S.final_lins.data(), (int64_t)S.final_lins.size());
    return st.out;
}

// plant: corrupt one epilogue coefficient of the lowered schedule (the
// checker's own test: the evaluation must then fail)
bool g_plant = false;

void check_shape(const Shape& s, int trials)
{
    const Compact c = compact(build_fft_netlist(s));
    const Compact sh = share(c);
    const NetStats st = netlist_stats(c);
    const std::string h = netlist_hash(c);
    check(h.size() == 64, "hash length");
    const int k = choose_k(c, 1);
    check(k > 0 && k % 32 == 0 && noise_bits(c, 2 * (int64_t)k) <= k, "modulus rule");
    Schedule S = lower(sh);
    if (g_plant) {
        // the middle product's first form with a product term: its P
        // coefficient flipped (AND becomes -AND)
        for (size_t i = S.prods.size() / 2; i < S.prods.size(); i++)
            if (S.prods[i].cP[0] != 0) {
                S.prods[i].cP[0] = (int8_t)-S.prods[i].cP[0];
                break;
            }
    }
    check(S.n_products <= st.products, "sharing added products");
    check((int32_t)c.n_inputs == s.n_inputs() && (int)c.outputs.size() == s.n_outputs(), "input/output counts");
    // schedules under live-set bounds: a slot bound, a level bound and a
    // window of a sixteenth of the products; the slots they use must not
    // exceed the unbounded schedule's
    LiveLimit lim;
    lim.max_slots = S.n_slots / 2;
    lim.max_level_products = 16;
    lim.max_window = (int64_t)S.n_products / 16 + 1;
    const Schedule Sb = lower(sh, lim);
    lim.max_slots = 0;
    const Schedule Sw = lower(sh, lim);
    check(Sb.n_products == S.n_products && Sw.n_products == S.n_products, "bounded schedule product count");
    check(Sb.max_level_products <= 16 && Sw.max_level_products <= 16, "level bound");
    check(Sw.n_slots <= S.n_slots, "windowed schedule uses more slots");
    for (int t = 0; t < trials; t++) {
        std::vector<int> in((size_t)c.n_inputs);
        for (auto& b : in) b = next_bit();
        const std::vector<int> want = eval_netlist(c, in), got = eval_schedule(S, sh, in);
        check(want == eval_netlist(sh, in), "shared netlist differs");
        check(got == want, "schedule evaluation differs from the netlist");
        check(eval_schedule(Sb, sh, in) == want, "bounded schedule evaluation differs from the netlist");
        check(eval_schedule(Sw, sh, in) == want, "windowed schedule evaluation differs from the netlist");
    }
    std::printf("dims=%d len=%d Q(%d,%d) %s%s: nodes=%lld products=%lld exec=%lld levels=%zu slots=%lld k=%d; "
                "bounded: levels %zu slots %lld, windowed: levels %zu slots %lld; ok\n",
                s.dims, s.len, s.F, s.f, s.is_complex ? "complex" : "real", s.nand_only ? " nand" : "",
                (long long)st.nodes, (long long)st.products, (long long)S.n_products, S.levels.size() - 1,
                (long long)S.n_slots, k, Sb.levels.size() - 1, (long long)Sb.n_slots, Sw.levels.size() - 1,
                (long long)Sw.n_slots);
}

}  // namespace

int main(int argc, char** argv)
{
    g_plant = argc > 1 && std::string(argv[1]) == "plant";
    try {
        const Shape shapes[] = {
            {1, 2, 4, 2, true},   {1, 8, 8, 4, false},  {1, 16, 16, 8, true}, {2, 4, 8, 4, false},
            {2, 4, 6, 3, true},   {1, 64, 16, 8, true}, {1, 4, 8, 4, true, true},
        };
        for (const Shape& s : shapes) check_shape(s, s.len >= 64 ? 2 : 8);
    } catch (const std::exception& e) {
        std::fprintf(stderr, "host check failed: %s\n", e.what());
        return g_plant ? 0 : 1;
    }
    if (g_plant) {
        std::fprintf(stderr, "planted mistake not detected\n");
        return 1;
    }
    std::printf("host check passed\n");
    return 0;
}
