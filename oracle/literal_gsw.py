"""Oracle: textbook GSW13 with explicit N x N binary ciphertexts and the
BitDecomp / BitDecomp^-1 / Flatten / Powersof2 operators, for tiny parameters.
TEST INFRASTRUCTURE ONLY.

This is the scheme the paper builds on (section "Notation and Background":
Gentry-Sahai-Waters 2013, key generation, encryption, decryption, addition,
multiplication and NAND, all on matrices over Z_q) written in the form of the
GSW13 paper itself: a ciphertext is a binary N x N matrix C, decryption takes
a row C_i with v_i = 2^i in (q/4, q/2] and rounds <C_i, v>/v_i, and every
evaluation ends with Flatten.  It is deliberately independent of the packed
representation used everywhere else so that tests can pin the identity
BitDecomp^-1(C) = packed ciphertext and the packed gate formulas against it.
Entries are Python ints (numpy object arrays): slow, exact, for N <= ~64.
"""
from __future__ import annotations

import numpy as np

from . import prng


class LiteralGSW:
    def __init__(self, n_lwe: int, k: int, seed: int):
        self.n = n_lwe
        self.k = k
        self.q = 1 << k
        self.l = k  # bits per element (2^l >= q)
        self.N = (n_lwe + 1) * self.l
        self.m = self.N
        self.seed = seed
        q = self.q
        t = [prng.zq_element(seed, 1, i, k) for i in range(n_lwe)]
        self.s = [1] + [(-x) % q for x in t]
        self.v = self.powersof2(self.s)
        B = [[prng.zq_element(seed, 2, j * n_lwe + i, k) for i in range(n_lwe)] for j in range(self.m)]
        e = [prng.ternary(seed, 3, j) for j in range(self.m)]
        b = [(sum(B[j][i] * t[i] for i in range(n_lwe)) + e[j]) % q for j in range(self.m)]
        self.A = np.array([[b[j]] + B[j] for j in range(self.m)], dtype=object)

    # -- the GSW13 operators ---------------------------------------------------
    def bitdecomp(self, a):
        """(n+1)-vector over Z_q -> N bits, element by element, LSB first."""
        out = []
        for x in a:
            x = int(x) % self.q
            out.extend((x >> j) & 1 for j in range(self.l))
        return out

    def bitdecomp_inv(self, a):
        """N-vector (any integers) -> (n+1)-vector sum_j 2^j a_{i,j} mod q."""
        out = []
        for i in range(self.n + 1):
            out.append(sum((1 << j) * int(a[i * self.l + j]) for j in range(self.l)) % self.q)
        return out

    def flatten(self, a):
        return self.bitdecomp(self.bitdecomp_inv(a))

    def powersof2(self, b):
        out = []
        for x in b:
            out.extend(((1 << j) * int(x)) % self.q for j in range(self.l))
        return out

    def flatten_mat(self, M):
        return np.array([self.flatten(list(row)) for row in M], dtype=object)

    # -- scheme ------------------------------------------------------------------
    def mask(self, ct_id: int):
        """R in {0,1}^(N x m), bits from generator domain 4."""
        M = (self.m + 63) // 64
        R = np.zeros((self.N, self.m), dtype=object)
        for row in range(self.N):
            for j in range(self.m):
                w = prng.word(self.seed, 4, ct_id * self.N * M + row * M + j // 64)
                R[row, j] = (w >> (j % 64)) & 1
        return R

    def enc(self, mu: int, ct_id: int):
        RA = self.mask(ct_id).dot(self.A) % self.q
        BD = np.array([self.bitdecomp(list(row)) for row in RA], dtype=object)
        eye = np.eye(self.N, dtype=int).astype(object)
        return self.flatten_mat(mu * eye + BD)

    def dec(self, C) -> int:
        i = self.l - 2 if self.q // 4 >= (1 << (self.l - 1)) else self.l - 1
        vi = self.v[i]
        assert self.q // 4 < vi <= self.q // 2
        x = sum(int(C[i, j]) * int(self.v[j]) for j in range(self.N)) % self.q
        return ((2 * x + vi) // (2 * vi)) % 2  # nearest integer to x / v_i, mod 2

    def add(self, C1, C2):
        return self.flatten_mat(C1 + C2)

    def mult(self, C1, C2):
        return self.flatten_mat(C1.dot(C2))

    def nand(self, C1, C2):
        eye = np.eye(self.N, dtype=int).astype(object)
        return self.flatten_mat(eye - C1.dot(C2))

    # gates of the circuit, each a single Flatten of a linear form in
    # C1, C2, C1*C2 and I
    def AND(self, C1, C2):
        return self.mult(C1, C2)

    def XOR(self, C1, C2):
        return self.flatten_mat(C1 + C2 - 2 * C1.dot(C2))

    def OR(self, C1, C2):
        return self.flatten_mat(C1 + C2 - C1.dot(C2))

    def NOT(self, C):
        eye = np.eye(self.N, dtype=int).astype(object)
        return self.flatten_mat(eye - C)

    def XADD(self, C1, C2):
        return self.add(C1, C2)

    def packed(self, C):
        """BitDecomp^-1 of every row: the (N x (n+1)) packed form."""
        return [self.bitdecomp_inv(list(row)) for row in C]
