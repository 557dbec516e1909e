/*
 * Oracle: GSW13 ciphertext arithmetic over q = 2^k in plain C.
 * TEST INFRASTRUCTURE ONLY: only tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this file's library.  It shares no code with the
 * HIP path.
 *
 * The paper (section "Notation and Background") uses the scheme of Gentry,
 * Sahai and Waters (2013): LWE-based, ciphertexts are integer matrices over
 * Z_q, evaluation offers addition and a ciphertext-ciphertext multiplication
 * that is a matrix-matrix product (section "Time/Space Complexities"), and the
 * NAND gate.  With q = 2^k and ell = k bits per element, a flattened
 * ciphertext C (binary, Nct x Nct, Nct = (n+1)k) is stored packed as
 * C' = C*G (Nct x (n+1) elements of Z_q) where G is the gadget matrix with
 * G[r][b] = 2^(r mod k) when b = r div k, else 0; the bits of C' are exactly C.
 *
 *   product       P   = BitDecomp(C'_L) * C'_R mod q  (packed Flatten(C_L*C_R))
 *   AND = P,  XOR = L + R - 2P,  OR = L + R - P,  NOT = G - C',  XADD = X + Y,
 *   NAND = G - P
 *   Enc(mu)       C'  = mu*G + Rbits*A mod q
 *
 * Layout (the library's interchange format): row-major, Nct rows, each row
 * (n+1) elements of kw = k/32 little-endian uint32 limbs.  The packed row is
 * its own bit decomposition (element b, bit t is bit b*k + t of the row).
 *
 * Every element operation is mod 2^k per element: no carry crosses an
 * element boundary.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

/* OpenMP threads the oracle's parallel loops use (and a setter, for timing
   the oracle on one core). */
int or_threads(void) { return omp_get_max_threads(); }
void or_set_threads(int n) { omp_set_num_threads(n); }

/* SplitMix64 finaliser (Steele, Lea and Flood, OOPSLA 2014). */
static uint64_t sm_mix(uint64_t z)
{
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ULL;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return z;
}

/* i-th output of a SplitMix64 stream whose state starts at mix(seed + dom*gamma). */
uint64_t or_word(uint64_t seed, uint64_t dom, uint64_t i)
{
    return sm_mix(sm_mix(seed + dom * GAMMA) + (i + 1) * GAMMA);
}

void or_words(uint64_t seed, uint64_t dom, uint64_t i0, int64_t count, uint64_t *out)
{
    for (int64_t i = 0; i < count; i++)
        out[i] = or_word(seed, dom, i0 + (uint64_t)i);
}

/* P = BitDecomp(L) * R mod 2^k.  The exact integer dot product of a bit row
 * with a column of R is accumulated limb by limb (each limb sum < nct*2^32,
 * so it fits 64 bits) and then carried once, dropping the carry out of the
 * element's top limb (the reduction mod 2^k). */
void or_product(int nct, int n1, int kw, const uint32_t *L, const uint32_t *R, uint32_t *P)
{
    const int W = n1 * kw;
#pragma omp parallel
    {
        uint64_t *acc = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)W);
#pragma omp for schedule(static)
        for (int r = 0; r < nct; r++) {
            memset(acc, 0, sizeof(uint64_t) * (size_t)W);
            const uint32_t *lrow = L + (size_t)r * W;
            for (int j = 0; j < nct; j++) {
                if ((lrow[j >> 5] >> (j & 31)) & 1u) {
                    const uint32_t *rrow = R + (size_t)j * W;
                    for (int w = 0; w < W; w++)
                        acc[w] += rrow[w];
                }
            }
            uint32_t *prow = P + (size_t)r * W;
            for (int e = 0; e < n1; e++) {
                uint64_t carry = 0;
                for (int w = 0; w < kw; w++) {
                    uint64_t v = acc[e * kw + w] + carry;
                    prow[e * kw + w] = (uint32_t)v;
                    carry = v >> 32;
                }
            }
        }
        free(acc);
    }
}

/* dst = ca*X + cb*Y + cc*Z + cg*G  (mod 2^k per element); X/Y/Z may be NULL
 * when their coefficient is 0.  Coefficients are small signed integers. */
static void lincomb(int nct, int n1, int kw, uint32_t *dst,
                    int ca, const uint32_t *X, int cb, const uint32_t *Y,
                    int cc, const uint32_t *Z, int cg)
{
    const int W = n1 * kw;
    const int k = 32 * kw;
#pragma omp parallel for schedule(static)
    for (int r = 0; r < nct; r++) {
        const int br = r / k, tr = r % k;
        for (int e = 0; e < n1; e++) {
            int64_t carry = 0; /* signed carry between limbs */
            for (int w = 0; w < kw; w++) {
                size_t o = (size_t)r * W + (size_t)e * kw + w;
                int64_t v = carry;
                if (ca) v += (int64_t)ca * (int64_t)X[o];
                if (cb) v += (int64_t)cb * (int64_t)Y[o];
                if (cc) v += (int64_t)cc * (int64_t)Z[o];
                if (cg && e == br && (tr >> 5) == w)
                    v += (int64_t)cg * (int64_t)((uint64_t)1 << (tr & 31));
                /* floor division by 2^32 for the carry, low 32 bits kept */
                uint32_t lo = (uint32_t)(uint64_t)v;
                carry = (v - (int64_t)lo) / ((int64_t)1 << 32);
                dst[o] = lo;
            }
        }
    }
}

/* Enc(mu) = mu*G + Rbits*A with Rbits (nct x m, m = nct) drawn bit by bit
 * from domain 4: row `row` of ciphertext `ct_id` uses words
 * ct_id*nct*M + row*M + j/64 (M = ceil(m/64)), bit j mod 64 is R[row][j]. */
void or_encrypt(int nct, int n1, int kw, const uint32_t *A, const int32_t *mu,
                int64_t n_ct, uint64_t seed, uint64_t first_ct_id, uint32_t *out)
{
    const int W = n1 * kw;
    const int m = nct;
    const uint64_t M = (uint64_t)(m + 63) / 64;
    uint32_t *Rb = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)nct * W);
    for (int64_t c = 0; c < n_ct; c++) {
        const uint64_t id = first_ct_id + (uint64_t)c;
        memset(Rb, 0, sizeof(uint32_t) * (size_t)nct * W);
        for (int row = 0; row < nct; row++) {
            uint64_t wd = 0;
            for (int j = 0; j < m; j++) {
                if (j % 64 == 0)
                    wd = or_word(seed, 4, id * (uint64_t)nct * M + (uint64_t)row * M + (uint64_t)(j / 64));
                if ((wd >> (j % 64)) & 1u)
                    Rb[(size_t)row * W + (j >> 5)] |= 1u << (j & 31);
            }
        }
        uint32_t *dst = out + (size_t)c * nct * W;
        or_product(nct, n1, kw, Rb, A, dst);
        if (mu[c] & 1)
            lincomb(nct, n1, kw, dst, 1, dst, 0, NULL, 0, NULL, 1);
    }
    free(Rb);
}

/* single gates, for unit tests */
void or_gate(int nct, int n1, int kw, int type, const uint32_t *X, const uint32_t *Y, uint32_t *out)
{
    const size_t n = (size_t)nct * n1 * kw;
    uint32_t *P = NULL;
    if (type == 4 || type == 5 || type == 6 || type == 8) {
        P = (uint32_t *)malloc(sizeof(uint32_t) * n);
        or_product(nct, n1, kw, X, Y, P);
    }
    switch (type) {
    case 3: lincomb(nct, n1, kw, out, -1, X, 0, NULL, 0, NULL, 1); break;   /* NOT  */
    case 4: memcpy(out, P, sizeof(uint32_t) * n); break;                   /* AND  */
    case 5: lincomb(nct, n1, kw, out, 1, X, 1, Y, -2, P, 0); break;        /* XOR  */
    case 6: lincomb(nct, n1, kw, out, 1, X, 1, Y, -1, P, 0); break;        /* OR   */
    case 7: lincomb(nct, n1, kw, out, 1, X, 1, Y, 0, NULL, 0); break;      /* XADD */
    case 8: lincomb(nct, n1, kw, out, 0, NULL, 0, NULL, -1, P, 1); break;  /* NAND */
    default: break;
    }
    free(P);
}

/* Evaluate a netlist (node arrays in construction order; type codes
 * IN=0 CONST0=1 CONST1=2 NOT=3 AND=4 XOR=5 OR=6 XADD=7 NAND=8; node 0/1 are the
 * constants) on input ciphertexts and write one ciphertext per output.
 * Constant outputs are the noiseless 0 and G.  Each node's ciphertext is
 * freed after its last use; the product of an (l, r) pair is kept while the
 * next gate on the same pair still needs it.  Returns 0, or -1 on an
 * allocation failure. */
int or_eval(int nct, int n1, int kw, int n_nodes, const int8_t *type, const int32_t *na,
            const int32_t *nb, int n_outputs, const int32_t *outputs,
            const uint32_t *inputs, uint32_t *out)
{
    const size_t csz = (size_t)nct * n1 * kw;
    int32_t *last = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_nodes);
    uint32_t **buf = (uint32_t **)calloc((size_t)n_nodes, sizeof(uint32_t *));
    if (!last || !buf) return -1;
    for (int v = 0; v < n_nodes; v++) last[v] = -1;
    for (int v = 0; v < n_nodes; v++) {
        if (type[v] >= 3) last[na[v]] = v;
        if (type[v] >= 4) last[nb[v]] = v;
    }
    for (int o = 0; o < n_outputs; o++) last[outputs[o]] = n_nodes;

    uint32_t *P = (uint32_t *)malloc(sizeof(uint32_t) * csz);
    int pl = -1, pr = -1;
    int rc = 0;
    for (int v = 0; v < n_nodes && rc == 0; v++) {
        int t = type[v];
        if (t == 0) {
            buf[v] = (uint32_t *)(inputs + (size_t)na[v] * csz);
            continue;
        }
        if (t == 1 || t == 2) continue;
        if (last[v] < 0) continue; /* unused */
        uint32_t *dst = (uint32_t *)malloc(sizeof(uint32_t) * csz);
        if (!dst) { rc = -1; break; }
        const uint32_t *X = buf[na[v]];
        const uint32_t *Y = (t >= 4) ? buf[nb[v]] : NULL;
        if (((t >= 4 && t <= 6) || t == 8) && !(pl == na[v] && pr == nb[v])) {
            or_product(nct, n1, kw, X, Y, P);
            pl = na[v];
            pr = nb[v];
        }
        switch (t) {
        case 3: lincomb(nct, n1, kw, dst, -1, X, 0, NULL, 0, NULL, 1); break;
        case 4: memcpy(dst, P, sizeof(uint32_t) * csz); break;
        case 5: lincomb(nct, n1, kw, dst, 1, X, 1, Y, -2, P, 0); break;
        case 6: lincomb(nct, n1, kw, dst, 1, X, 1, Y, -1, P, 0); break;
        case 7: lincomb(nct, n1, kw, dst, 1, X, 1, Y, 0, NULL, 0); break;
        case 8: lincomb(nct, n1, kw, dst, 0, NULL, 0, NULL, -1, P, 1); break;
        }
        buf[v] = dst;
        /* release operands whose last use was this node */
        int ops[2] = {na[v], (t >= 4) ? nb[v] : -1};
        for (int q = 0; q < 2; q++) {
            int u = ops[q];
            if (u >= 2 && last[u] == v && type[u] != 0 && buf[u]) {
                if (q == 1 && ops[0] == u) continue;
                free(buf[u]);
                buf[u] = NULL;
            }
        }
    }
    if (rc == 0) {
        for (int o = 0; o < n_outputs; o++) {
            int v = outputs[o];
            uint32_t *dst = out + (size_t)o * csz;
            if (v == 0) {
                memset(dst, 0, sizeof(uint32_t) * csz);
            } else if (v == 1) {
                memset(dst, 0, sizeof(uint32_t) * csz);
                lincomb(nct, n1, kw, dst, 0, NULL, 0, NULL, 0, NULL, 1);
            } else {
                memcpy(dst, buf[v], sizeof(uint32_t) * csz);
            }
        }
    }
    for (int v = 0; v < n_nodes; v++)
        if (buf[v] && type[v] != 0) free(buf[v]);
    free(buf);
    free(last);
    free(P);
    return rc;
}
