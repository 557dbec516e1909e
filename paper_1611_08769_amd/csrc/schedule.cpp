#include "schedule.hpp"

#include <algorithm>
#include <functional>
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

}  // namespace

Schedule lower(const Compact& c)
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
    for (int32_t p = 0; p < np; p++)
        if (!attached[p].empty()) max_level = std::max(max_level, level_of(p));
    for (size_t v = 0; v < n; v++)
        if (mat[v]) max_level = std::max(max_level, avail_of((int32_t)v));

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
