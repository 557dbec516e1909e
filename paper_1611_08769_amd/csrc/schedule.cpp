#include "schedule.hpp"

#include <algorithm>
#include <functional>
#include <queue>
#include <map>
#include <stdexcept>
#include <unordered_map>

namespace sfft {
namespace {

// Linear form over one product (P and its operands L, R), the gadget G and up
// to two further ciphertexts already in memory.
struct Form {
    int32_t prod = -1;
    int cL = 0, cR = 0, cP = 0, cG = 0;
    int nt = 0;
    int32_t tn[3] = {-1, -1, -1};
    int tc[3] = {0, 0, 0};
};

Form term(int32_t v)
{
    Form f;
    f.nt = 1;
    f.tn[0] = v;
    f.tc[0] = 1;
    return f;
}

Form neg(Form f)
{
    f.cL = -f.cL; f.cR = -f.cR; f.cP = -f.cP; f.cG = -f.cG;
    for (int i = 0; i < f.nt; i++) f.tc[i] = -f.tc[i];
    return f;
}

// sum of two forms; returns false if the result needs more than 3 terms
bool add_forms(const Form& x, const Form& y, Form* out)
{
    if (x.prod >= 0 && y.prod >= 0 && x.prod != y.prod) return false;
    Form r = x;
    r.prod = x.prod >= 0 ? x.prod : y.prod;
    r.cL += y.cL; r.cR += y.cR; r.cP += y.cP; r.cG += y.cG;
    for (int i = 0; i < y.nt; i++) {
        int j = 0;
        while (j < r.nt && r.tn[j] != y.tn[i]) j++;
        if (j < r.nt) {
            r.tc[j] += y.tc[i];
        } else {
            if (r.nt == 3) return false;
            r.tn[r.nt] = y.tn[i];
            r.tc[r.nt] = y.tc[i];
            r.nt++;
        }
    }
    // drop cancelled terms
    int k = 0;
    for (int i = 0; i < r.nt; i++) {
        if (r.tc[i] == 0) continue;
        r.tn[k] = r.tn[i];
        r.tc[k] = r.tc[i];
        k++;
    }
    r.nt = k;
    *out = r;
    return true;
}

// Levels under a bound on the live set (list scheduling).  Products are
// taken in order of first appearance in the netlist (for the FFT, the
// butterflies of the first rows and stages first) once their operands are in
// memory; a level takes ready products while the workspace ciphertexts that
// would be live through it stay within lim.max_slots, the level holds at
// most lim.max_level_products and the product lies within lim.max_window of
// the first product not yet run, and always takes at least the first ready
// one.
// A product-free linear node is computed right after the level that makes
// its last term available (sub-passes as in the unbounded schedule).  A
// workspace ciphertext is live from the level that writes it to the last
// level that reads it, as the slot assignment that follows counts it.
int32_t bounded_levels(const Compact& c, const std::vector<Form>& form, const std::vector<uint8_t>& mat,
                       const std::vector<int32_t>& pl, const std::vector<int32_t>& pr,
                       const std::vector<std::vector<int32_t>>& attached, const LiveLimit& lim,
                       std::vector<int32_t>* plevel_out, std::vector<int32_t>* avail_out, std::vector<int32_t>* sub_out)
{
    const size_t n = c.size();
    const int32_t np = (int32_t)pl.size();
    std::vector<int32_t>& plevel = *plevel_out;
    std::vector<int32_t>& avail = *avail_out;
    std::vector<int32_t>& sub = *sub_out;
    std::vector<uint8_t> is_output(n, 0);
    for (int32_t o : c.outputs)
        if (o >= 2 && c.t[o] != T_IN) is_output[o] = 1;
    // slot holders: materialised nodes other than inputs and outputs
    auto holds_slot = [&](size_t v) { return mat[v] && c.t[v] != T_IN && !is_output[v]; };

    // readers of every node: products (as operands or extra terms) and
    // linear nodes; pending operand counts of both
    std::vector<std::vector<int32_t>> prod_readers(n), lin_readers(n);
    std::vector<int32_t> uses(n, 0), p_wait(np, 0), l_wait(n, 0);
    auto read_by_prod = [&](int32_t u, int32_t p) {
        prod_readers[u].push_back(p);
        uses[u]++;
        p_wait[p]++;
    };
    for (int32_t p = 0; p < np; p++) {
        if (attached[p].empty()) continue;
        read_by_prod(pl[p], p);
        read_by_prod(pr[p], p);
        for (int32_t o : attached[p])
            for (int i = 0; i < form[o].nt; i++) read_by_prod(form[o].tn[i], p);
    }
    std::vector<int32_t> lin_nodes;
    for (size_t v = 0; v < n; v++) {
        if (!mat[v] || c.t[v] == T_IN || form[v].prod >= 0) continue;
        lin_nodes.push_back((int32_t)v);
        for (int i = 0; i < form[v].nt; i++) {
            lin_readers[form[v].tn[i]].push_back((int32_t)v);
            uses[form[v].tn[i]]++;
            l_wait[v]++;
        }
    }

    std::priority_queue<int32_t, std::vector<int32_t>, std::greater<int32_t>> ready;
    std::vector<int32_t> dying;  // slot holders whose last reader ran at this level
    auto read_once = [&](int32_t u) {
        if (--uses[u] == 0 && holds_slot(u)) dying.push_back(u);
    };
    std::vector<int32_t> became;  // nodes that came into memory at the current level
    int64_t live = 0;             // slot holders in memory and still to be read

    // a node is in memory from level L on: wake its readers
    std::function<void(int32_t, int32_t)> arrive = [&](int32_t v, int32_t L) {
        avail[v] = L;
        for (int32_t p : prod_readers[v])
            if (--p_wait[p] == 0) ready.push(p);
        for (int32_t w : lin_readers[v]) {
            if (--l_wait[w] != 0) continue;
            // a linear node: computed after level L in sub-pass order
            int32_t s = 0;
            for (int i = 0; i < form[w].nt; i++) {
                const int32_t t = form[w].tn[i];
                if (c.t[t] != T_IN && form[t].prod < 0 && avail[t] == L) s = std::max(s, sub[t] + 1);
            }
            sub[w] = s;
            if (holds_slot(w)) live++;
            for (int i = 0; i < form[w].nt; i++) read_once(form[w].tn[i]);  // read at level L
            arrive(w, L);
        }
    };

    for (size_t v = 0; v < n; v++)
        if (c.t[v] == T_IN) arrive((int32_t)v, 0);
    // linear nodes with no terms (constants) are in memory from level 0
    for (int32_t v : lin_nodes)
        if (form[v].nt == 0 && avail[v] < 0) {
            sub[v] = 0;
            if (holds_slot(v)) live++;
            arrive(v, 0);
        }
    live -= (int64_t)dying.size();
    dying.clear();

    // product items of each product: a new item when kMaxOut outputs or
    // kMaxE distinct extra operands are reached (the packing below)
    std::vector<int32_t> items(np, 0);
    for (int32_t p = 0; p < np; p++) {
        int nout = 0, ne = 0;
        int32_t es[kMaxE];
        for (int32_t o : attached[p]) {
            const int32_t e = form[o].nt == 1 ? form[o].tn[0] : -1;
            bool seen = e < 0;
            for (int q = 0; q < ne && !seen; q++) seen = es[q] == e;
            if (nout == 0 || nout == kMaxOut || (!seen && ne == kMaxE)) {
                items[p]++;
                nout = 0;
                ne = 0;
                seen = e < 0;
            }
            if (!seen) es[ne++] = e;
            nout++;
        }
    }
    int32_t low = 0;  // the first product not yet scheduled
    int64_t scheduled = 0, to_schedule = 0;
    for (int32_t p = 0; p < np; p++) to_schedule += !attached[p].empty();
    int32_t L = 0;
    while (scheduled < to_schedule) {
        L++;
        if (ready.empty()) throw std::logic_error("bounded schedule: no ready product");
        std::vector<int32_t> take;
        int64_t born = 0, level_items = 0;
        while (low < np && (attached[low].empty() || plevel[low] >= 0)) low++;
        while (!ready.empty()) {
            // in order: nothing passes a product that waits
            const int32_t p = ready.top();
            if (!take.empty() && lim.max_window > 0 && p >= low + lim.max_window) break;
            int64_t b = 0;
            for (int32_t o : attached[p]) b += holds_slot(o);
            const bool fits = (lim.max_slots <= 0 || live + born + b <= lim.max_slots) &&
                              (lim.max_level_products <= 0 || level_items + items[p] <= lim.max_level_products);
            if (!take.empty() && !fits) break;
            ready.pop();
            take.push_back(p);
            born += b;
            level_items += items[p];
        }
        // the level's products read their operands and write their outputs
        for (int32_t p : take) {
            plevel[p] = L;
            read_once(pl[p]);
            read_once(pr[p]);
            for (int32_t o : attached[p])
                for (int i = 0; i < form[o].nt; i++) read_once(form[o].tn[i]);
        }
        live += born;
        for (int32_t p : take)
            for (int32_t o : attached[p]) arrive(o, L);
        scheduled += (int64_t)take.size();
        live -= (int64_t)dying.size();
        dying.clear();
    }
    for (int32_t v : lin_nodes)
        if (avail[v] < 0) throw std::logic_error("bounded schedule: linear node never computed");
    return L;
}

}  // namespace

Schedule lower(const Compact& c, const LiveLimit& lim)
{
    const size_t n = c.size();
    std::vector<Form> form(n);
    std::vector<uint8_t> mat(n, 0);
    std::vector<int32_t> pl, pr;
    std::unordered_map<uint64_t, int32_t> pid_of;

    auto product_id = [&](int32_t l, int32_t r) {
        const uint64_t key = (uint64_t)(uint32_t)l << 32 | (uint32_t)r;
        auto it = pid_of.find(key);
        if (it != pid_of.end()) return it->second;
        const int32_t id = (int32_t)pl.size();
        pl.push_back(l);
        pr.push_back(r);
        pid_of.emplace(key, id);
        return id;
    };

    // ---- forms ----------------------------------------------------------------
    for (size_t v = 0; v < n; v++) {
        const int8_t ty = c.t[v];
        Form f;
        switch (ty) {
        case T_IN: f = term((int32_t)v); mat[v] = 1; break;
        case T_C0: break;
        case T_C1: f.cG = 1; break;
        case T_AND: case T_XOR: case T_OR: case T_NAND: {
            const int32_t l = c.a[v], r = c.b[v];
            f.prod = product_id(l, r);
            mat[l] = mat[r] = 1;
            if (ty == T_AND) { f.cP = 1; }
            else if (ty == T_XOR) { f.cL = 1; f.cR = 1; f.cP = -2; }
            else if (ty == T_OR) { f.cL = 1; f.cR = 1; f.cP = -1; }
            else { f.cP = -1; f.cG = 1; }  // NAND = G - P
            break;
        }
        case T_NOT: f = neg(form[c.a[v]]); f.cG += 1; break;
        case T_XADD: {
            const int32_t x = c.a[v], y = c.b[v];
            Form fx = form[x], fy = form[y];
            if (fx.prod >= 0 && fy.prod >= 0 && fx.prod != fy.prod) {
                // keep the later product, read the earlier one from memory
                if (fx.prod < fy.prod) { mat[x] = 1; fx = term(x); }
                else { mat[y] = 1; fy = term(y); }
            }
            Form r;
            const bool ok = add_forms(fx, fy, &r);
            const int max_terms = r.prod >= 0 ? 1 : 2;
            if (!ok || r.nt > max_terms) {
                mat[x] = mat[y] = 1;
                add_forms(term(x), term(y), &r);
            }
            f = r;
            break;
        }
        default: throw std::logic_error("bad node type");
        }
        form[v] = f;
    }
    for (int32_t o : c.outputs)
        if (o >= 2) mat[o] = 1;

    // a NOT of a product-free form that has 3 terms cannot happen: the only
    // multi-term product-free forms come from the XADD fallback (2 terms)
    for (size_t v = 0; v < n; v++)
        if (mat[v] && form[v].prod < 0 && form[v].nt > 2) throw std::logic_error("linear form too wide");

    // ---- outputs attached to each product -------------------------------------
    const int32_t np = (int32_t)pl.size();
    std::vector<std::vector<int32_t>> attached(np);
    for (size_t v = 0; v < n; v++)
        if (mat[v] && c.t[v] != T_IN && form[v].prod >= 0) attached[form[v].prod].push_back((int32_t)v);

    // ---- levels ----------------------------------------------------------------
    // avail(v): level after which v is in memory (0 = inputs / level-0 linear).
    std::vector<int32_t> avail(n, -1), plevel(np, -1), sub(n, 0);
    std::vector<uint8_t> busy(n, 0), pbusy(np, 0);
    std::function<int32_t(int32_t)> avail_of;
    std::function<int32_t(int32_t)> level_of = [&](int32_t p) -> int32_t {
        if (plevel[p] >= 0) return plevel[p];
        if (pbusy[p]) throw std::logic_error("cyclic schedule");
        pbusy[p] = 1;
        int32_t L = std::max(avail_of(pl[p]), avail_of(pr[p]));
        for (int32_t o : attached[p])
            for (int i = 0; i < form[o].nt; i++) L = std::max(L, avail_of(form[o].tn[i]));
        plevel[p] = L + 1;
        return plevel[p];
    };
    avail_of = [&](int32_t v) -> int32_t {
        if (avail[v] >= 0) return avail[v];
        if (busy[v]) throw std::logic_error("cyclic schedule");
        busy[v] = 1;
        int32_t a = 0;
        if (c.t[v] == T_IN) {
            a = 0;
        } else if (form[v].prod >= 0) {
            a = level_of(form[v].prod);
        } else {
            int32_t s = 0;
            for (int i = 0; i < form[v].nt; i++) a = std::max(a, avail_of(form[v].tn[i]));
            for (int i = 0; i < form[v].nt; i++) {
                const int32_t t = form[v].tn[i];
                if (c.t[t] != T_IN && form[t].prod < 0 && avail[t] == a) s = std::max(s, sub[t] + 1);
            }
            sub[v] = s;
        }
        avail[v] = a;
        return a;
    };
    int32_t max_level = 0;
    if (lim.max_slots <= 0 && lim.max_level_products <= 0) {
        // as soon as possible: a product runs one level after its last operand
        for (int32_t p = 0; p < np; p++)
            if (!attached[p].empty()) max_level = std::max(max_level, level_of(p));
        for (size_t v = 0; v < n; v++)
            if (mat[v]) max_level = std::max(max_level, avail_of((int32_t)v));
    } else {
        max_level = bounded_levels(c, form, mat, pl, pr, attached, lim, &plevel, &avail, &sub);
    }

    // ---- homes -------------------------------------------------------------------
    std::vector<int32_t> home(n, -1);
    std::vector<uint8_t> is_out(n, 0);
    Schedule S;
    for (size_t v = 0; v < n; v++)
        if (c.t[v] == T_IN) home[v] = ct_ref(B_IN, (uint32_t)c.a[v]);
    for (size_t pos = 0; pos < c.outputs.size(); pos++) {
        const int32_t o = c.outputs[pos];
        if (o >= 2 && c.t[o] != T_IN && home[o] < 0) {
            home[o] = ct_ref(B_OUT, (uint32_t)pos);
            is_out[o] = 1;
        } else {
            LinItem li{};
            li.dst = ct_ref(B_OUT, (uint32_t)pos);
            li.X = li.Y = -1;
            if (o == kOne) li.cG = 1;
            else if (o != kZero) { li.X = o; li.cX = 1; }  // resolved to a ref below
            S.final_lins.push_back(li);
        }
    }

    // last use level of every materialised node
    std::vector<int32_t> last(n, -1);
    auto use = [&](int32_t v, int32_t L) { last[v] = std::max(last[v], L); };
    for (int32_t p = 0; p < np; p++) {
        if (attached[p].empty()) continue;
        use(pl[p], plevel[p]);
        use(pr[p], plevel[p]);
        for (int32_t o : attached[p])
            for (int i = 0; i < form[o].nt; i++) use(form[o].tn[i], plevel[p]);
    }
    for (size_t v = 0; v < n; v++)
        if (mat[v] && c.t[v] != T_IN && form[v].prod < 0)
            for (int i = 0; i < form[v].nt; i++) use(form[v].tn[i], avail[v]);

    // workspace slots: a slot freed after level L is reused from level L+1 on
    std::vector<std::vector<int32_t>> born(max_level + 2), dies(max_level + 2);
    for (size_t v = 0; v < n; v++) {
        if (!mat[v] || c.t[v] == T_IN || is_out[v]) continue;
        if (last[v] < 0) continue;  // never read (cannot happen for a needed node)
        born[avail[v]].push_back((int32_t)v);
        dies[last[v]].push_back((int32_t)v);
    }
    std::vector<int32_t> free_slots;
    int64_t nslots = 0;
    std::vector<int32_t> slot(n, -1);
    for (int32_t L = 0; L <= max_level; L++) {
        if (L > 0)
            for (int32_t v : dies[L - 1]) free_slots.push_back(slot[v]);
        for (int32_t v : born[L]) {
            if (free_slots.empty()) free_slots.push_back((int32_t)nslots++);
            slot[v] = free_slots.back();
            free_slots.pop_back();
            home[v] = ct_ref(B_WS, (uint32_t)slot[v]);
        }
    }
    S.n_slots = nslots;

    for (size_t v = 0; v < n; v++)
        if (mat[v] && home[v] < 0) throw std::logic_error("materialised node without a home");
    for (auto& li : S.final_lins)
        if (li.X >= 0) li.X = home[li.X];

    // ---- items -----------------------------------------------------------------
    // An item carries up to kMaxOut outputs of one product, whose extra
    // operands are at most kMaxE distinct ciphertexts; the outputs of a
    // product that need more take further items (the product is computed
    // again).
    std::vector<std::vector<ProdItem>> prod_at(max_level + 1);
    for (int32_t p = 0; p < np; p++) {
        if (attached[p].empty()) continue;
        const auto& outs = attached[p];
        size_t k = 0;
        while (k < outs.size()) {
            ProdItem it{};
            it.L = home[pl[p]];
            it.R = home[pr[p]];
            it.nout = 0;
            int32_t eref[kMaxE];
            int ne = 0;
            for (; k < outs.size() && it.nout < kMaxOut; k++) {
                const Form& f = form[outs[k]];
                const int32_t e = f.nt == 1 ? home[f.tn[0]] : -1;
                if (e >= 0) {
                    bool seen = false;
                    for (int q = 0; q < ne; q++) seen = seen || eref[q] == e;
                    if (!seen) {
                        if (ne == kMaxE) break;
                        eref[ne++] = e;
                    }
                }
                for (int c : {f.cL, f.cR, f.cP, f.cG, f.nt == 1 ? f.tc[0] : 0})
                    if (c < -kMaxCoef || c > kMaxCoef) throw std::logic_error("gate coefficient out of range");
                const int i = it.nout++;
                it.dst[i] = home[outs[k]];
                it.cL[i] = (int8_t)f.cL;
                it.cR[i] = (int8_t)f.cR;
                it.cP[i] = (int8_t)f.cP;
                it.cG[i] = (int8_t)f.cG;
                it.E[i] = e;
                it.cE[i] = (int8_t)(e >= 0 ? f.tc[0] : 0);
            }
            for (int i = it.nout; i < kMaxOut; i++) it.dst[i] = it.E[i] = -1;
            prod_at[plevel[p]].push_back(it);
        }
    }
    std::map<std::pair<int32_t, int32_t>, std::vector<LinItem>> lin_at;
    for (size_t v = 0; v < n; v++) {
        if (!mat[v] || c.t[v] == T_IN || form[v].prod >= 0) continue;
        const Form& f = form[v];
        LinItem li{};
        li.dst = home[v];
        li.X = f.nt > 0 ? home[f.tn[0]] : -1;
        li.Y = f.nt > 1 ? home[f.tn[1]] : -1;
        li.cX = (int8_t)(f.nt > 0 ? f.tc[0] : 0);
        li.cY = (int8_t)(f.nt > 1 ? f.tc[1] : 0);
        li.cG = (int8_t)f.cG;
        lin_at[{avail[v], sub[v]}].push_back(li);
    }
    S.levels.resize(max_level + 1);
    for (int32_t L = 0; L <= max_level; L++) {
        S.levels[L].prod_begin = (int64_t)S.prods.size();
        S.levels[L].prod_count = (int64_t)prod_at[L].size();
        S.prods.insert(S.prods.end(), prod_at[L].begin(), prod_at[L].end());
        S.max_level_products = std::max<int64_t>(S.max_level_products, (int64_t)prod_at[L].size());
    }
    for (auto& kv : lin_at) {
        auto& lv = S.levels[kv.first.first];
        lv.lin.push_back({(int64_t)S.lins.size(), (int64_t)kv.second.size()});
        S.lins.insert(S.lins.end(), kv.second.begin(), kv.second.end());
    }
    S.n_products = (int64_t)S.prods.size();
    return S;
}

}  // namespace sfft
