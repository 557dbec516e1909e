#include "netlist.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <stdexcept>
#include <unordered_map>

namespace sfft {

// ---------------------------------------------------------------------------
// twiddles
// ---------------------------------------------------------------------------
static int64_t round_half_away(double v)
{
    double a = std::floor(std::fabs(v) + 0.5);
    return v >= 0 ? (int64_t)a : -(int64_t)a;
}

void twiddle(int j, int m, int f, int64_t* cr, int64_t* ci)
{
    const double ang = 2.0 * M_PI * (double)j / (double)m;
    const double scale = std::ldexp(1.0, f);
    *cr = round_half_away(std::cos(ang) * scale);
    *ci = round_half_away(-std::sin(ang) * scale);
}

// ---------------------------------------------------------------------------
// construction
// ---------------------------------------------------------------------------
static inline bool is_const(int32_t v) { return v == kZero || v == kOne; }

Netlist::Netlist(bool nand) : nand_only(nand)
{
    t = {T_C0, T_C1};
    a = {-1, -1};
    b = {-1, -1};
}

int32_t Netlist::node(int8_t type, int32_t x, int32_t y)
{
    const int32_t id = (int32_t)t.size();
    t.push_back(type);
    a.push_back(x);
    b.push_back(y);
    return id;
}

int32_t Netlist::input()
{
    const int32_t id = (int32_t)t.size();
    t.push_back(T_IN);
    a.push_back(n_inputs++);
    b.push_back(-1);
    return id;
}

int32_t Netlist::NAND(int32_t l, int32_t r)
{
    if (l == kZero || r == kZero) return kOne;
    if (l == kOne && r == kOne) return kZero;
    if (l == kOne) return NOT(r);
    if (r == kOne) return NOT(l);
    return node(T_NAND, l, r);
}

int32_t Netlist::NOT(int32_t x)
{
    if (x == kZero) return kOne;
    if (x == kOne) return kZero;
    if (nand_only) return node(T_NAND, x, x);
    return node(T_NOT, x, -1);
}

int32_t Netlist::AND(int32_t l, int32_t r)
{
    if (l == kZero || r == kZero) return kZero;
    if (l == kOne) return r;
    if (r == kOne) return l;
    if (nand_only) {
        const int32_t n = node(T_NAND, l, r);
        return node(T_NAND, n, n);
    }
    return node(T_AND, l, r);
}

int32_t Netlist::XOR(int32_t l, int32_t r)
{
    if (l == kZero) return r;
    if (r == kZero) return l;
    if (l == kOne) return NOT(r);
    if (r == kOne) return NOT(l);
    if (nand_only) {
        const int32_t n = node(T_NAND, l, r);
        const int32_t x = node(T_NAND, l, n);
        const int32_t y = node(T_NAND, r, n);
        return node(T_NAND, x, y);
    }
    return node(T_XOR, l, r);
}

int32_t Netlist::OR(int32_t l, int32_t r)
{
    if (l == kOne || r == kOne) return kOne;
    if (l == kZero) return r;
    if (r == kZero) return l;
    if (nand_only) {
        const int32_t x = node(T_NAND, l, l);
        const int32_t y = node(T_NAND, r, r);
        return node(T_NAND, x, y);
    }
    return node(T_OR, l, r);
}

int32_t Netlist::XADD(int32_t x, int32_t y)
{
    if (x == kZero) return y;
    if (y == kZero) return x;
    if (x == kOne || y == kOne) throw std::logic_error("XADD with constant one");
    return node(T_XADD, x, y);
}

std::pair<int32_t, int32_t> Netlist::HA(int32_t x, int32_t y)
{
    const int32_t s = XOR(x, y);
    const int32_t c = AND(x, y);
    return {s, c};
}

std::pair<int32_t, int32_t> Netlist::FA(int32_t x, int32_t y, int32_t c, AdderMode mode)
{
    const int32_t in[3] = {x, y, c};
    if (is_const(x) || is_const(y) || is_const(c)) {
        int32_t nc[3];
        int n = 0, K = 0;
        for (int i = 0; i < 3; i++) {
            if (in[i] == kOne) K++;
            else if (in[i] != kZero) nc[n++] = in[i];
        }
        if (n == 2) {
            if (K == 0) return HA(nc[0], nc[1]);
            const int32_t xo = XOR(nc[0], nc[1]);
            const int32_t s = NOT(xo);
            const int32_t o = OR(nc[0], nc[1]);
            return {s, o};
        }
        if (n == 1) {
            if (K == 0) return {nc[0], kZero};
            if (K == 1) {
                const int32_t s = NOT(nc[0]);
                return {s, nc[0]};
            }
            return {nc[0], kOne};
        }
        return {(K & 1) ? kOne : kZero, (K >> 1) ? kOne : kZero};
    }
    const int32_t A = AND(x, y);
    const int32_t X = XOR(x, y);
    int32_t P, S;
    if (mode == kRipple) {
        P = AND(c, X);
        S = XOR(c, X);
    } else {
        P = AND(X, c);
        S = XOR(X, c);
    }
    const int32_t cy = nand_only ? OR(A, P) : XADD(A, P);
    return {S, cy};
}

std::vector<int32_t> Netlist::add(const std::vector<int32_t>& x, const std::vector<int32_t>& y)
{
    std::vector<int32_t> out;
    int32_t carry = kZero;
    for (size_t i = 0; i < x.size(); i++) {
        auto sc = FA(x[i], y[i], carry, kRipple);
        out.push_back(sc.first);
        carry = sc.second;
    }
    return out;
}

std::vector<int32_t> Netlist::sub(const std::vector<int32_t>& x, const std::vector<int32_t>& y)
{
    std::vector<int32_t> out;
    int32_t carry = kOne;
    for (size_t i = 0; i < x.size(); i++) {
        const int32_t ny = NOT(y[i]);
        auto sc = FA(x[i], ny, carry, kRipple);
        out.push_back(sc.first);
        carry = sc.second;
    }
    return out;
}

std::vector<int32_t> Netlist::mul_const(const std::vector<int32_t>& x, int64_t c, int f)
{
    const int F = (int)x.size();
    const int W = f + F;
    // c as a 2F-bit two's-complement pattern
    const uint64_t mask = (F * 2 >= 64) ? ~0ull : ((1ull << (2 * F)) - 1);
    const uint64_t cu = (uint64_t)c & mask;
    std::vector<std::vector<int32_t>> cols(W);
    for (int i = 0; i < 2 * F; i++) {
        if (!((cu >> i) & 1ull)) continue;
        for (int j = 0; i + j < W; j++) cols[i + j].push_back(x[std::min(j, F - 1)]);
    }
    auto tall = [&]() {
        for (auto& col : cols)
            if (col.size() > 2) return true;
        return false;
    };
    while (tall()) {
        std::vector<std::vector<int32_t>> nxt(W);
        for (int w = 0; w < W; w++) {
            const auto& col = cols[w];
            size_t p = 0;
            while (col.size() - p >= 3) {
                auto sc = FA(col[p], col[p + 1], col[p + 2], kCsa);
                p += 3;
                nxt[w].push_back(sc.first);
                if (w + 1 < W) nxt[w + 1].push_back(sc.second);
            }
            if (col.size() - p == 2) {
                auto sc = HA(col[p], col[p + 1]);
                nxt[w].push_back(sc.first);
                if (w + 1 < W) nxt[w + 1].push_back(sc.second);
            } else if (col.size() - p == 1) {
                nxt[w].push_back(col[p]);
            }
        }
        cols.swap(nxt);
    }
    std::vector<int32_t> sums;
    int32_t carry = kZero;
    for (int w = 0; w < W; w++) {
        const int32_t u = cols[w].size() > 0 ? cols[w][0] : kZero;
        const int32_t v = cols[w].size() > 1 ? cols[w][1] : kZero;
        auto sc = FA(u, v, carry, kRipple);
        sums.push_back(sc.first);
        carry = sc.second;
    }
    return std::vector<int32_t>(sums.begin() + f, sums.begin() + f + F);
}

static int ilog2(int n)
{
    int l = 0;
    while ((1 << l) < n) l++;
    return l;
}

static int bitrev(int i, int lg)
{
    int r = 0;
    for (int k = 0; k < lg; k++) {
        r = (r << 1) | (i & 1);
        i >>= 1;
    }
    return r;
}

std::vector<Netlist::Cplx> Netlist::fft1d(const std::vector<Cplx>& xs, int f)
{
    const int N = (int)xs.size();
    const int lg = ilog2(N);
    std::vector<Cplx> x(N);
    for (int i = 0; i < N; i++) x[i] = xs[bitrev(i, lg)];
    const int64_t one = (int64_t)1 << f;
    for (int s = 1; s <= lg; s++) {
        const int m = 1 << s, h = m / 2;
        for (int g = 0; g < N; g += m) {
            for (int j = 0; j < h; j++) {
                int64_t cr, ci;
                twiddle(j, m, f, &cr, &ci);
                const Cplx A = x[g + j], B = x[g + j + h];
                Cplx Xi, Xj;
                if (cr == one && ci == 0) {
                    Xi.re = add(A.re, B.re);
                    Xi.im = add(A.im, B.im);
                    Xj.re = sub(A.re, B.re);
                    Xj.im = sub(A.im, B.im);
                } else if (cr == 0 && ci == -one) {
                    Xi.re = add(A.re, B.im);
                    Xi.im = sub(A.im, B.re);
                    Xj.re = sub(A.re, B.im);
                    Xj.im = add(A.im, B.re);
                } else {
                    const auto m_rr = mul_const(B.re, cr, f);
                    const auto m_ii = mul_const(B.im, ci, f);
                    const auto tr = sub(m_rr, m_ii);
                    const auto m_ir = mul_const(B.im, cr, f);
                    const auto m_ri = mul_const(B.re, ci, f);
                    const auto ti = add(m_ir, m_ri);
                    Xi.re = add(A.re, tr);
                    Xi.im = add(A.im, ti);
                    Xj.re = sub(A.re, tr);
                    Xj.im = sub(A.im, ti);
                }
                x[g + j] = Xi;
                x[g + j + h] = Xj;
            }
        }
    }
    return x;
}

Netlist build_fft_netlist(const Shape& s)
{
    Netlist nl(s.nand_only);
    const int npts = s.points();
    std::vector<Netlist::Cplx> words(npts);
    for (int v = 0; v < npts; v++) {
        for (int i = 0; i < s.F; i++) words[v].re.push_back(nl.input());
        for (int i = 0; i < s.F; i++) words[v].im.push_back(s.is_complex ? nl.input() : kZero);
    }
    std::vector<Netlist::Cplx> out(npts);
    if (s.dims == 1) {
        out = nl.fft1d(words, s.f);
    } else {
        const int S = s.len;
        std::vector<std::vector<Netlist::Cplx>> rows;
        for (int r = 0; r < S; r++) {
            std::vector<Netlist::Cplx> row(words.begin() + r * S, words.begin() + (r + 1) * S);
            rows.push_back(nl.fft1d(row, s.f));
        }
        for (int c = 0; c < S; c++) {
            std::vector<Netlist::Cplx> col;
            for (int r = 0; r < S; r++) col.push_back(rows[r][c]);
            auto y = nl.fft1d(col, s.f);
            for (int r = 0; r < S; r++) out[r * S + c] = y[r];
        }
    }
    for (int v = 0; v < npts; v++) {
        nl.outputs.insert(nl.outputs.end(), out[v].re.begin(), out[v].re.end());
        nl.outputs.insert(nl.outputs.end(), out[v].im.begin(), out[v].im.end());
    }
    return nl;
}

// ---------------------------------------------------------------------------
// DCE / sharing
// ---------------------------------------------------------------------------
static int arity(int8_t t)
{
    if (t == T_NOT) return 1;
    if (t >= T_AND) return 2;
    return 0;
}

Compact compact(const Netlist& nl)
{
    const size_t n = nl.t.size();
    std::vector<uint8_t> live(n, 0);
    live[0] = live[1] = 1;
    std::vector<int32_t> stack(nl.outputs.begin(), nl.outputs.end());
    while (!stack.empty()) {
        const int32_t v = stack.back();
        stack.pop_back();
        if (live[v]) continue;
        live[v] = 1;
        const int ar = arity(nl.t[v]);
        if (ar >= 1) stack.push_back(nl.a[v]);
        if (ar >= 2) stack.push_back(nl.b[v]);
    }
    for (size_t v = 0; v < n; v++)
        if (nl.t[v] == T_IN) live[v] = 1;
    std::vector<int32_t> remap(n, -1);
    Compact c;
    for (size_t v = 0; v < n; v++) {
        if (!live[v]) continue;
        remap[v] = (int32_t)c.t.size();
        const int8_t ty = nl.t[v];
        c.t.push_back(ty);
        const int ar = arity(ty);
        if (ty == T_IN) {
            c.a.push_back(nl.a[v]);
            c.b.push_back(-1);
        } else {
            c.a.push_back(ar >= 1 ? remap[nl.a[v]] : -1);
            c.b.push_back(ar >= 2 ? remap[nl.b[v]] : -1);
        }
    }
    for (int32_t o : nl.outputs) c.outputs.push_back(remap[o]);
    c.n_inputs = nl.n_inputs;
    return c;
}

Compact share(const Compact& c)
{
    const size_t n = c.size();
    std::vector<int32_t> rep(n);
    std::unordered_map<uint64_t, int32_t> seen;
    seen.reserve(n * 2);
    Compact out;
    std::vector<int32_t> newid(n, -1);
    for (size_t v = 0; v < n; v++) {
        const int8_t ty = c.t[v];
        const int ar = arity(ty);
        int32_t x = ar >= 1 ? newid[c.a[v]] : -1;
        int32_t y = ar >= 2 ? newid[c.b[v]] : -1;
        if (ty == T_IN || ty == T_C0 || ty == T_C1) {
            newid[v] = (int32_t)out.t.size();
            out.t.push_back(ty);
            out.a.push_back(c.a[v]);
            out.b.push_back(c.b[v]);
            continue;
        }
        const uint64_t key = ((uint64_t)(uint8_t)ty << 56) ^ ((uint64_t)(uint32_t)x << 28) ^ (uint64_t)(uint32_t)y;
        // key collisions are resolved by checking the stored node
        auto it = seen.find(key);
        if (it != seen.end()) {
            const int32_t u = it->second;
            if (out.t[u] == ty && out.a[u] == x && out.b[u] == y) {
                newid[v] = u;
                continue;
            }
        }
        newid[v] = (int32_t)out.t.size();
        out.t.push_back(ty);
        out.a.push_back(x);
        out.b.push_back(y);
        if (it == seen.end()) seen.emplace(key, newid[v]);
    }
    for (int32_t o : c.outputs) out.outputs.push_back(newid[o]);
    out.n_inputs = c.n_inputs;
    (void)rep;
    return out;
}

// ---------------------------------------------------------------------------
// SHA-256 (FIPS 180-4)
// ---------------------------------------------------------------------------
namespace {
struct Sha256 {
    uint32_t h[8] = {0x6a09e667, 0xbb67ae85, 0x3c6ef372, 0xa54ff53a,
                     0x510e527f, 0x9b05688c, 0x1f83d9ab, 0x5be0cd19};
    uint8_t buf[64];
    size_t fill = 0;
    uint64_t total = 0;

    static uint32_t rotr(uint32_t x, int n) { return (x >> n) | (x << (32 - n)); }

    void block(const uint8_t* p)
    {
        static const uint32_t K[64] = {
            0x428a2f98, 0x71374491, 0xb5c0fbcf, 0xe9b5dba5, 0x3956c25b, 0x59f111f1, 0x923f82a4, 0xab1c5ed5,
            0xd807aa98, 0x12835b01, 0x243185be, 0x550c7dc3, 0x72be5d74, 0x80deb1fe, 0x9bdc06a7, 0xc19bf174,
            0xe49b69c1, 0xefbe4786, 0x0fc19dc6, 0x240ca1cc, 0x2de92c6f, 0x4a7484aa, 0x5cb0a9dc, 0x76f988da,
            0x983e5152, 0xa831c66d, 0xb00327c8, 0xbf597fc7, 0xc6e00bf3, 0xd5a79147, 0x06ca6351, 0x14292967,
            0x27b70a85, 0x2e1b2138, 0x4d2c6dfc, 0x53380d13, 0x650a7354, 0x766a0abb, 0x81c2c92e, 0x92722c85,
            0xa2bfe8a1, 0xa81a664b, 0xc24b8b70, 0xc76c51a3, 0xd192e819, 0xd6990624, 0xf40e3585, 0x106aa070,
            0x19a4c116, 0x1e376c08, 0x2748774c, 0x34b0bcb5, 0x391c0cb3, 0x4ed8aa4a, 0x5b9cca4f, 0x682e6ff3,
            0x748f82ee, 0x78a5636f, 0x84c87814, 0x8cc70208, 0x90befffa, 0xa4506ceb, 0xbef9a3f7, 0xc67178f2};
        uint32_t w[64];
        for (int i = 0; i < 16; i++)
            w[i] = (uint32_t)p[4 * i] << 24 | (uint32_t)p[4 * i + 1] << 16 | (uint32_t)p[4 * i + 2] << 8 | p[4 * i + 3];
        for (int i = 16; i < 64; i++) {
            const uint32_t s0 = rotr(w[i - 15], 7) ^ rotr(w[i - 15], 18) ^ (w[i - 15] >> 3);
            const uint32_t s1 = rotr(w[i - 2], 17) ^ rotr(w[i - 2], 19) ^ (w[i - 2] >> 10);
            w[i] = w[i - 16] + s0 + w[i - 7] + s1;
        }
        uint32_t a = h[0], b = h[1], c = h[2], d = h[3], e = h[4], f = h[5], g = h[6], hh = h[7];
        for (int i = 0; i < 64; i++) {
            const uint32_t S1 = rotr(e, 6) ^ rotr(e, 11) ^ rotr(e, 25);
            const uint32_t ch = (e & f) ^ (~e & g);
            const uint32_t t1 = hh + S1 + ch + K[i] + w[i];
            const uint32_t S0 = rotr(a, 2) ^ rotr(a, 13) ^ rotr(a, 22);
            const uint32_t mj = (a & b) ^ (a & c) ^ (b & c);
            const uint32_t t2 = S0 + mj;
            hh = g; g = f; f = e; e = d + t1; d = c; c = b; b = a; a = t1 + t2;
        }
        h[0] += a; h[1] += b; h[2] += c; h[3] += d; h[4] += e; h[5] += f; h[6] += g; h[7] += hh;
    }

    void update(const void* data, size_t len)
    {
        const uint8_t* p = (const uint8_t*)data;
        total += len;
        while (len) {
            const size_t take = std::min(len, 64 - fill);
            std::memcpy(buf + fill, p, take);
            fill += take;
            p += take;
            len -= take;
            if (fill == 64) {
                block(buf);
                fill = 0;
            }
        }
    }

    std::string hex()
    {
        const uint64_t bits = total * 8;
        const uint8_t pad = 0x80;
        update(&pad, 1);
        const uint8_t zero = 0;
        while (fill != 56) update(&zero, 1);
        uint8_t lenb[8];
        for (int i = 0; i < 8; i++) lenb[i] = (uint8_t)(bits >> (56 - 8 * i));
        update(lenb, 8);
        static const char* dig = "0123456789abcdef";
        std::string s;
        for (int i = 0; i < 8; i++)
            for (int k = 28; k >= 0; k -= 4) s.push_back(dig[(h[i] >> k) & 15]);
        return s;
    }
};
}  // namespace

std::string netlist_hash(const Compact& c)
{
    Sha256 sh;
    std::vector<uint8_t> buf;
    buf.reserve(9 * 4096);
    auto put32 = [&](uint32_t v) {
        for (int i = 0; i < 4; i++) buf.push_back((uint8_t)(v >> (8 * i)));
    };
    for (size_t v = 0; v < c.size(); v++) {
        buf.push_back((uint8_t)c.t[v]);
        put32((uint32_t)c.a[v]);
        put32((uint32_t)c.b[v]);
        if (buf.size() > 9 * 4000) {
            sh.update(buf.data(), buf.size());
            buf.clear();
        }
    }
    put32((uint32_t)c.outputs.size());
    for (int32_t o : c.outputs) put32((uint32_t)o);
    sh.update(buf.data(), buf.size());
    return sh.hex();
}

NetStats netlist_stats(const Compact& c)
{
    NetStats st{};
    st.nodes = (int64_t)c.size();
    std::vector<int32_t> level(c.size(), 0);
    std::unordered_map<uint64_t, int32_t> prods;
    std::vector<int64_t> width;
    for (size_t v = 0; v < c.size(); v++) {
        const int8_t ty = c.t[v];
        if (ty == T_NOT) {
            st.nots++;
            level[v] = level[c.a[v]];
        } else if (ty == T_XADD) {
            st.gates++;
            level[v] = std::max(level[c.a[v]], level[c.b[v]]);
        } else if (is_product_type(ty)) {
            st.gates++;
            level[v] = 1 + std::max(level[c.a[v]], level[c.b[v]]);
            const uint64_t key = (uint64_t)(uint32_t)c.a[v] << 32 | (uint32_t)c.b[v];
            if (prods.emplace(key, level[v]).second) {
                if ((int64_t)width.size() <= level[v]) width.resize(level[v] + 1, 0);
                width[level[v]]++;
                st.products++;
            }
        }
    }
    for (size_t L = 0; L < width.size(); L++) {
        if (width[L]) st.depth = (int64_t)L;
        st.max_width = std::max(st.max_width, width[L]);
    }
    return st;
}

// ---------------------------------------------------------------------------
// noise bound with exact multi-precision integers
// ---------------------------------------------------------------------------
namespace {
// numbers stored in an arena as little-endian uint32 limbs
struct Arena {
    std::vector<uint32_t> limbs;
    std::vector<uint32_t> off, len;
};

void big_axpy(std::vector<uint32_t>& out, const uint32_t* x, uint32_t xl, const uint32_t* y, uint32_t yl, uint64_t s)
{
    // out = x + s*y
    const uint32_t n = std::max(xl, yl) + 3;
    out.assign(n, 0);
    uint64_t carry = 0;
    for (uint32_t i = 0; i < n; i++) {
        unsigned __int128 v = carry;
        if (i < xl) v += x[i];
        if (i < yl) v += (unsigned __int128)y[i] * s;
        out[i] = (uint32_t)v;
        carry = (uint64_t)(v >> 32);
    }
    while (!out.empty() && out.back() == 0) out.pop_back();
}

int big_bitlen(const uint32_t* x, uint32_t l)
{
    while (l && x[l - 1] == 0) l--;
    if (!l) return 0;
    return 32 * (int)(l - 1) + (32 - __builtin_clz(x[l - 1]));
}

bool big_less(const uint32_t* x, uint32_t xl, const uint32_t* y, uint32_t yl)
{
    while (xl && x[xl - 1] == 0) xl--;
    while (yl && y[yl - 1] == 0) yl--;
    if (xl != yl) return xl < yl;
    for (uint32_t i = xl; i-- > 0;)
        if (x[i] != y[i]) return x[i] < y[i];
    return false;
}
}  // namespace

int noise_bits(const Compact& c, int64_t nct)
{
    // B(IN) = m = Nct; B(NOT x) = B(x); B(AND/OR) = B(l) + Nct B(r);
    // B(XOR) = B(l) + (2 Nct - 1) B(r); B(XADD) = B(x) + B(y).
    Arena ar;
    ar.off.assign(c.size(), 0);
    ar.len.assign(c.size(), 0);
    ar.limbs.reserve(c.size() * 8);
    std::vector<uint32_t> tmp;
    auto store = [&](size_t v, const std::vector<uint32_t>& x) {
        ar.off[v] = (uint32_t)ar.limbs.size();
        ar.len[v] = (uint32_t)x.size();
        ar.limbs.insert(ar.limbs.end(), x.begin(), x.end());
    };
    for (size_t v = 0; v < c.size(); v++) {
        const int8_t ty = c.t[v];
        if (ty == T_IN) {
            tmp.clear();
            uint64_t m = (uint64_t)nct;
            while (m) {
                tmp.push_back((uint32_t)m);
                m >>= 32;
            }
            store(v, tmp);
        } else if (ty == T_NOT) {
            ar.off[v] = ar.off[c.a[v]];
            ar.len[v] = ar.len[c.a[v]];
        } else if (is_product_type(ty) || ty == T_XADD) {
            // AND, OR, NAND: B(l) + Nct B(r); XOR: B(l) + (2 Nct - 1) B(r); XADD: B(l) + B(r)
            const uint64_t s = ty == T_XADD ? 1 : ty == T_XOR ? (uint64_t)(2 * nct - 1) : (uint64_t)nct;
            const int32_t l = c.a[v], r = c.b[v];
            // copy operands out first: the arena may reallocate on store
            std::vector<uint32_t> X(ar.limbs.begin() + ar.off[l], ar.limbs.begin() + ar.off[l] + ar.len[l]);
            std::vector<uint32_t> Y(ar.limbs.begin() + ar.off[r], ar.limbs.begin() + ar.off[r] + ar.len[r]);
            big_axpy(tmp, X.data(), (uint32_t)X.size(), Y.data(), (uint32_t)Y.size(), s);
            store(v, tmp);
        }
    }
    const uint32_t* best = nullptr;
    uint32_t bl = 0;
    for (int32_t o : c.outputs) {
        const uint32_t* x = ar.limbs.data() + ar.off[o];
        if (!best || big_less(best, bl, x, ar.len[o])) {
            best = x;
            bl = ar.len[o];
        }
    }
    return (best ? big_bitlen(best, bl) : 0) + 3;
}

int choose_k(const Compact& c, int n_lwe, int k_limit)
{
    int k = 32;
    while (k <= k_limit) {
        const int g = noise_bits(c, (int64_t)(n_lwe + 1) * k);
        if (g <= k) return k;
        k = (g + 31) / 32 * 32;
    }
    return -1;
}

}  // namespace sfft
