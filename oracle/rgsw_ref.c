/*
 * Oracle: ring-GSW ciphertext arithmetic over R_p = Z_p[X]/(X^d + 1) in plain C.
 * TEST INFRASTRUCTURE ONLY: only tests, the smoke check and the CPU-baseline
 * leg of the benchmark load this file's library.  It shares no code with the
 * HIP path.
 *
 * The paper evaluates its circuits with the GSW13 scheme (section "Notation
 * and Background"): ciphertexts are matrices, the product of two ciphertexts
 * is a matrix product after bit decomposition, and NAND, AND, XOR and OR are
 * affine in that product (Lemma "binary gates").  GSW13 also has a ring
 * instantiation, in which the matrix entries are polynomials of R_p.  This
 * file is that instantiation, written from its definition:
 *
 *   v = (1, -s),  s in R_p small;  ell = bit length of p;  N = 2*ell rows
 *   G = I_2 (x) (1, 2, 4, ..., 2^(ell-1))^T              (N x 2 over R_p)
 *   Enc(m)   C = m*G + Z,  row r of Z = (a_r*s + e_r, a_r)  so  Z*v = e
 *   G^-1(C)  the N x N matrix of binary polynomials with G^-1(C)*G = C:
 *            entry (i, c*ell + j) holds bit j of every coefficient of C[i][c]
 *   product  P = G^-1(L) * R                              (N x 2 over R_p)
 *   AND = P,  XOR = L + R - 2P,  OR = L + R - P,  NAND = G - P,  NOT = G - L,
 *   XADD = L + R
 *   Dec      phase of row ell-1: (C*v)[ell-1] = m*2^(ell-1) + e; coefficient 0
 *            decides m (|centred value| > p/4 reads 1)
 *
 * Polynomial products are computed by the definition of the negacyclic
 * product (x^d = -1), coefficient by coefficient, with 128-bit integers.
 *
 * Layout: a ciphertext is N rows x 2 columns x d coefficients, uint64 in
 * [0, p), row-major (row, column, coefficient).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

typedef unsigned __int128 u128;

/* OpenMP threads the oracle's parallel loops use. */
int rg_threads(void) { return omp_get_max_threads(); }

static uint64_t addm(uint64_t a, uint64_t b, uint64_t p) { u128 s = (u128)a + b; return (uint64_t)(s % p); }
static uint64_t subm(uint64_t a, uint64_t b, uint64_t p) { return a >= b ? a - b : (uint64_t)((u128)a + p - b); }

/* out = a * b in Z_p[X]/(X^d + 1):  out_k = sum_{i+j=k} a_i b_j - sum_{i+j=k+d} a_i b_j. */
void rg_negmul(uint64_t p, int d, const uint64_t *a, const uint64_t *b, uint64_t *out)
{
    for (int k = 0; k < d; k++) {
        u128 pos = 0, neg = 0;
        for (int i = 0; i < d; i++) {
            int j = k - i;
            if (j >= 0) {
                pos += (u128)a[i] * b[j] % p;
            } else {
                neg += (u128)a[i] * b[j + d] % p;
            }
        }
        out[k] = subm((uint64_t)(pos % p), (uint64_t)(neg % p), p);
    }
}

/* Encrypt n bits.  s: d coefficients in [0,p).  a: n*N*d uniform in [0,p).
 * e: n*N*d small signed errors.  m: n bits.  ct: n ciphertexts. */
void rg_encrypt(uint64_t p, int d, int ell, const uint64_t *s, const uint64_t *a, const int64_t *e,
                const uint8_t *m, int64_t n, uint64_t *ct)
{
    const int N = 2 * ell;
    #pragma omp parallel for collapse(2) schedule(static)
    for (int64_t c = 0; c < n; c++) {
        for (int r = 0; r < N; r++) {
            const uint64_t *ar = a + (c * N + r) * (int64_t)d;
            const int64_t *er = e + (c * N + r) * (int64_t)d;
            uint64_t *row = ct + (c * N + r) * 2 * (int64_t)d;
            rg_negmul(p, d, ar, s, row);                       /* a_r * s */
            for (int t = 0; t < d; t++) {
                uint64_t et = er[t] >= 0 ? (uint64_t)er[t] % p : p - (uint64_t)(-er[t]) % p;
                row[t] = addm(row[t], et % p, p);              /* + e_r   */
                row[d + t] = ar[t];                            /* a_r     */
            }
            if (m[c]) {                                        /* + m*G   */
                int col = r / ell, j = r % ell;
                row[col * d] = addm(row[col * d], ((uint64_t)1 << j) % p, p);
            }
        }
    }
}

/* Row i of G^-1(L) * R: both output polynomials.  scratch: d words. */
static void product_row(uint64_t p, int d, int ell, const uint64_t *L, const uint64_t *R, int i,
                        uint64_t *out0, uint64_t *out1, uint64_t *bits, uint64_t *tmp)
{
    const int N = 2 * ell;
    memset(out0, 0, sizeof(uint64_t) * d);
    memset(out1, 0, sizeof(uint64_t) * d);
    for (int jj = 0; jj < N; jj++) {
        int col = jj / ell, j = jj % ell;
        const uint64_t *src = L + ((int64_t)i * 2 + col) * d;
        for (int t = 0; t < d; t++) bits[t] = (src[t] >> j) & 1;  /* digit polynomial */
        const uint64_t *r0 = R + ((int64_t)jj * 2 + 0) * d;
        const uint64_t *r1 = R + ((int64_t)jj * 2 + 1) * d;
        rg_negmul(p, d, bits, r0, tmp);
        for (int t = 0; t < d; t++) out0[t] = addm(out0[t], tmp[t], p);
        rg_negmul(p, d, bits, r1, tmp);
        for (int t = 0; t < d; t++) out1[t] = addm(out1[t], tmp[t], p);
    }
}

/* out[c] = gate(L[c], R[c]) for n ciphertext pairs.  op: 3 NOT (R ignored),
 * 4 AND, 5 XOR, 6 OR, 7 XADD, 8 NAND, 9 PRODUCT (= AND).  Returns 0, or -1
 * for an unknown op. */
int rg_gate(uint64_t p, int d, int ell, int op, const uint64_t *L, const uint64_t *R, uint64_t *out,
            int64_t n)
{
    if (op < 3 || op > 9) return -1;
    const int N = 2 * ell;
    const int64_t ct = (int64_t)N * 2 * d;
    #pragma omp parallel
    {
        uint64_t *P = malloc(sizeof(uint64_t) * 4 * d);
        uint64_t *bits = P + 2 * d, *tmp = P + 3 * d;
        #pragma omp for collapse(2) schedule(dynamic)
        for (int64_t c = 0; c < n; c++) {
            for (int i = 0; i < N; i++) {
                const uint64_t *Lc = L + c * ct, *Rc = R + c * ct;
                uint64_t *o = out + c * ct + (int64_t)i * 2 * d;
                const uint64_t *li = Lc + (int64_t)i * 2 * d, *ri = Rc + (int64_t)i * 2 * d;
                int needP = (op == 4 || op == 5 || op == 6 || op == 8 || op == 9);
                if (needP) product_row(p, d, ell, Lc, Rc, i, P, P + d, bits, tmp);
                for (int t = 0; t < 2 * d; t++) {
                    uint64_t g = (t % d == 0 && t / d == i / ell) ? ((uint64_t)1 << (i % ell)) % p : 0;
                    uint64_t v;
                    switch (op) {
                    case 3: v = subm(g, li[t], p); break;
                    case 4: case 9: v = P[t]; break;
                    case 5: v = subm(addm(li[t], ri[t], p), addm(P[t], P[t], p), p); break;
                    case 6: v = subm(addm(li[t], ri[t], p), P[t], p); break;
                    case 7: v = addm(li[t], ri[t], p); break;
                    default: v = subm(g, P[t], p); break;
                    }
                    o[t] = v;
                }
            }
        }
        free(P);
    }
    return 0;
}

/* Rows of gate outputs, one by one: for sample q, row rows[q] of
 * op(L[cts[q]], R[cts[q]]) into out + q*2*d.  op as for rg_gate. */
int rg_gate_rows(uint64_t p, int d, int ell, int op, const uint64_t *L, const uint64_t *R, const int64_t *cts,
                 const int32_t *rows, int64_t count, uint64_t *out)
{
    if (op < 3 || op > 9) return -1;
    const int N = 2 * ell;
    const int64_t ct = (int64_t)N * 2 * d;
    #pragma omp parallel
    {
        uint64_t *P = malloc(sizeof(uint64_t) * 4 * d);
        uint64_t *bits = P + 2 * d, *tmp = P + 3 * d;
        #pragma omp for schedule(dynamic)
        for (int64_t q = 0; q < count; q++) {
            const int64_t c = cts[q];
            const int i = rows[q];
            const uint64_t *Lc = L + c * ct, *Rc = R + c * ct;
            const uint64_t *li = Lc + (int64_t)i * 2 * d, *ri = Rc + (int64_t)i * 2 * d;
            uint64_t *o = out + q * 2 * d;
            if (op != 3 && op != 7) product_row(p, d, ell, Lc, Rc, i, P, P + d, bits, tmp);
            for (int t = 0; t < 2 * d; t++) {
                uint64_t g = (t % d == 0 && t / d == i / ell) ? ((uint64_t)1 << (i % ell)) % p : 0;
                uint64_t v;
                switch (op) {
                case 3: v = subm(g, li[t], p); break;
                case 4: case 9: v = P[t]; break;
                case 5: v = subm(addm(li[t], ri[t], p), addm(P[t], P[t], p), p); break;
                case 6: v = subm(addm(li[t], ri[t], p), P[t], p); break;
                case 7: v = addm(li[t], ri[t], p); break;
                default: v = subm(g, P[t], p); break;
                }
                o[t] = v;
            }
        }
        free(P);
    }
    return 0;
}

/* Blind rotation (the core of FHEW/TFHE-style refresh, written for this
 * scheme's ring-GSW ciphertexts as the key): m ring-LWE accumulators acc[j] =
 * (b, a), 2d words each, and n ring-GSW encryptions bk[i] of bits s_i.  Step i
 * replaces acc[j] by the CMux of bk[i] between acc[j] and X^r acc[j]
 * (r = rot[j*n + i] in [0, 2d)):
 *     acc <- acc + G^-1(X^r acc - acc) * bk[i]
 * (external product: the row vector of digit polynomials of X^r acc - acc
 * times the 2*ell x 2 matrix bk[i]).  X^r is applied as a product with the
 * monomial X^r (X^d = -1).  So acc[j] ends as an encryption of
 * X^(sum_i r_i s_i) times what it encrypted. */
void rg_blind_rotate(uint64_t p, int d, int ell, const uint64_t *bk, int64_t n, const int32_t *rot, uint64_t *acc,
                     int64_t m)
{
    const int64_t ct = (int64_t)2 * ell * 2 * d;
    #pragma omp parallel
    {
        uint64_t *w = malloc(sizeof(uint64_t) * 9 * d);
        uint64_t *mono = w, *diff = w + d, *o0 = w + 3 * d, *o1 = w + 4 * d, *bits = w + 5 * d, *tmp = w + 6 * d;
        #pragma omp for schedule(dynamic)
        for (int64_t j = 0; j < m; j++) {
            uint64_t *a = acc + j * 2 * d;
            for (int64_t i = 0; i < n; i++) {
                int r = rot[j * n + i];
                memset(mono, 0, sizeof(uint64_t) * d);
                if (r < d) mono[r] = 1; else mono[r - d] = p - 1;       /* X^r */
                for (int col = 0; col < 2; col++) {
                    rg_negmul(p, d, mono, a + col * d, tmp);
                    for (int t = 0; t < d; t++) diff[col * d + t] = subm(tmp[t], a[col * d + t], p);
                }
                product_row(p, d, ell, diff, bk + i * ct, 0, o0, o1, bits, tmp);
                for (int t = 0; t < d; t++) {
                    a[t] = addm(a[t], o0[t], p);
                    a[d + t] = addm(a[d + t], o1[t], p);
                }
            }
        }
        free(w);
    }
}

/* Gate bootstrapping within the ring scheme (FHEW-style refresh, without the
 * final key switch).  Input: m LWE ciphertexts (a_0..a_{n-1}, b) mod p under
 * a binary secret of n bits s_i, encrypting mu in {0,1} as
 * b - <a, s> = mu*p/2 + e.  The key bk holds ring-GSW encryptions of the s_i.
 *   1. modulus switch to 2d: x~ = floor((x*2d + floor(p/2)) / p) mod 2d
 *   2. accumulator (X^(b~ + d/2) * TV, 0) with TV = Delta*(1 + X + ... + X^(d-1)),
 *      Delta = floor(p/4); rotations r_i = -a~_i mod 2d
 *   3. blind rotation: the accumulator encrypts X^(b~ + d/2 - sum a~_i s_i) TV,
 *      whose coefficient 0 is -Delta when that exponent lies in (0, d) and
 *      +Delta in (d, 2d)
 *   4. sample extraction of coefficient 0, plus Delta on b: an LWE ciphertext
 *      (a'_0..a'_{d-1}, b') under the ring secret's coefficients with
 *      a'_0 = a_0, a'_t = -a_{d-t}, whose phase is mu*2*Delta + fresh error.
 * out: m x (d+1) words. */
static void bootstrap_delta(uint64_t p, int d, int ell, const uint64_t *bk, int64_t n, const uint64_t *lwe,
                            int64_t m, uint64_t *out, uint64_t delta)
{
    const uint64_t two_d = 2 * (uint64_t)d;
    uint64_t *acc = malloc(sizeof(uint64_t) * 2 * d * (m > 0 ? m : 1));
    int32_t *rot = malloc(sizeof(int32_t) * (n * m > 0 ? n * m : 1));
    for (int64_t j = 0; j < m; j++) {
        const uint64_t *c = lwe + j * (n + 1);
        for (int64_t i = 0; i < n; i++) {
            uint64_t ai = (uint64_t)(((u128)c[i] * two_d + p / 2) / p) % two_d;
            rot[j * n + i] = (int32_t)((two_d - ai) % two_d);
        }
        uint64_t bt = (uint64_t)(((u128)c[n] * two_d + p / 2) / p) % two_d;
        uint64_t k = (bt + (uint64_t)d / 2) % two_d;
        for (int u = 0; u < d; u++) {
            /* coefficient u of X^k * TV: +Delta if (u - k) mod 2d < d, else -Delta */
            uint64_t t = ((uint64_t)u + two_d - k) % two_d;
            acc[j * 2 * d + u] = t < (uint64_t)d ? delta : p - delta;
            acc[j * 2 * d + d + u] = 0;
        }
    }
    rg_blind_rotate(p, d, ell, bk, n, rot, acc, m);
    for (int64_t j = 0; j < m; j++) {
        const uint64_t *A = acc + j * 2 * d;
        uint64_t *o = out + j * (d + 1);
        o[0] = A[d];
        for (int t = 1; t < d; t++) o[t] = (p - A[d + d - t]) % p;
        o[d] = addm(A[0], delta, p);
    }
    free(acc);
    free(rot);
}

void rg_bootstrap(uint64_t p, int d, int ell, const uint64_t *bk, int64_t n, const uint64_t *lwe, int64_t m,
                  uint64_t *out)
{
    bootstrap_delta(p, d, ell, bk, n, lwe, m, out, p / 4);
}

/* Key switching of m LWE ciphertexts (a'_0..a'_{d-1}, b') mod p under the
 * ring secret's coefficients to the LWE secret of n coefficients, with the
 * key-switching key ksk[t][k] = an LWE encryption (n+1 words) under the LWE
 * secret of s_ring[t] * 2^(4k), t < d, k < 16 (base-16 digits of a'_t):
 *   out = (0, ..., 0, b') - sum_{t,k} digit_k(a'_t) * ksk[t][k]
 * out: m x (n+1) words. */
void rg_keyswitch(uint64_t p, int d, int64_t n, const uint64_t *ksk, const uint64_t *in, int64_t m, uint64_t *out)
{
    const int K = 16;
    #pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < m; j++) {
        const uint64_t *c = in + j * (d + 1);
        uint64_t *o = out + j * (n + 1);
        for (int64_t q = 0; q <= n; q++) {
            u128 sum = 0;
            for (int t = 0; t < d; t++)
                for (int k = 0; k < K; k++) {
                    uint64_t dig = (c[t] >> (4 * k)) & 15;
                    sum += (u128)dig * ksk[((int64_t)t * K + k) * (n + 1) + q];
                }
            uint64_t v = (uint64_t)(sum % p);
            o[q] = subm(q == n ? c[d] : 0, v, p);
        }
    }
}

/* Bootstrapped binary gates (FHEW-style) on LWE ciphertexts mod p under a
 * binary secret of n bits, bits encoded as mu * 2 * q8, q8 = floor(p/8):
 *   combine  c = cx*x + cy*y + (0, .., 0, k*q8): AND (1, 1, -1), OR (1, 1, 1),
 *            NAND (-1, -1, 5), XOR (2, 2, 0) -- so that the phase of c lies
 *            in (-p/4, p/4) for a 0 result and in (p/4, 3p/4) for a 1, at
 *            least p/8 from either edge
 *   refresh  the bootstrap with Delta = q8 (accumulator value and the constant
 *            added at extraction): phase mu * 2 * q8 under the ring secret
 *   switch   back to the LWE secret with ksk (as rg_keyswitch).
 * gate: 4 AND, 5 XOR, 6 OR, 8 NAND.  x, y, out: m x (n+1) words.  Returns 0,
 * or -1 for another gate. */
int rg_gate_bootstrap(uint64_t p, int d, int ell, int gate, const uint64_t *bk, int64_t n, const uint64_t *ksk,
                      const uint64_t *x, const uint64_t *y, int64_t m, uint64_t *out)
{
    int64_t cx, cy, k;
    switch (gate) {
    case 4: cx = 1, cy = 1, k = -1; break;
    case 6: cx = 1, cy = 1, k = 1; break;
    case 8: cx = -1, cy = -1, k = 5; break;
    case 5: cx = 2, cy = 2, k = 0; break;
    default: return -1;
    }
    const uint64_t q8 = p / 8;
    uint64_t *c = malloc(sizeof(uint64_t) * (n + 1) * (m > 0 ? m : 1));
    uint64_t *mid = malloc(sizeof(uint64_t) * (d + 1) * (m > 0 ? m : 1));
    for (int64_t j = 0; j < m * (n + 1); j++) {
        u128 v = ((u128)(uint64_t)(cx < 0 ? p + cx : cx) * x[j] + (u128)(uint64_t)(cy < 0 ? p + cy : cy) * y[j]) % p;
        if (j % (n + 1) == n) v = (v + (u128)(uint64_t)(k < 0 ? p + k : k) * q8) % p;
        c[j] = (uint64_t)v;
    }
    bootstrap_delta(p, d, ell, bk, n, c, m, mid, q8);
    rg_keyswitch(p, d, n, ksk, mid, m, out);
    free(c);
    free(mid);
    return 0;
}

/* Phase of one row: C[row][0] - C[row][1]*s  (d coefficients). */
void rg_phase(uint64_t p, int d, int ell, const uint64_t *ct, int row, const uint64_t *s, uint64_t *out)
{
    (void)ell;
    const uint64_t *c0 = ct + (int64_t)row * 2 * d, *c1 = c0 + d;
    rg_negmul(p, d, c1, s, out);
    for (int t = 0; t < d; t++) out[t] = subm(c0[t], out[t], p);
}

/* Decrypt n ciphertexts to bits from coefficient 0 of row ell-1's phase. */
void rg_decrypt(uint64_t p, int d, int ell, const uint64_t *ct, int64_t n, const uint64_t *s, uint8_t *m)
{
    const int64_t sz = (int64_t)2 * ell * 2 * d;
    #pragma omp parallel
    {
        uint64_t *ph = malloc(sizeof(uint64_t) * d);
        #pragma omp for schedule(static)
        for (int64_t c = 0; c < n; c++) {
            rg_phase(p, d, ell, ct + c * sz, ell - 1, s, ph);
            uint64_t x = ph[0];
            uint64_t mag = x <= p / 2 ? x : p - x;
            m[c] = mag > p / 4;
        }
        free(ph);
    }
}
