"""Oracle: ring-GSW over R_p = Z_p[X]/(X^d + 1).  TEST INFRASTRUCTURE ONLY.

GSW13's ring instantiation of the scheme the paper evaluates its circuits
with (section "Notation and Background"; gates as in Lemma "binary gates"):
matrix entries are polynomials of R_p, with p = 2^62 - 2^16 + 1, a prime
with 2^16 | p - 1 (so R_p has negacyclic transforms for every d <= 2^15).
The arithmetic is in rgsw_ref.c, by the definitions written out in its
header; polynomial products there are the negacyclic convolution itself.

Ciphertext layout: (2*ell rows, 2 columns, d coefficients) uint64 in
[0, p), ell = 62.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

P = (1 << 62) - (1 << 16) + 1
ELL = 62
ROWS = 2 * ELL

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rgsw_ref.c")
_LIB = os.path.join(_HERE, "librgsw_ref.so")

NOT, AND, XOR, OR, XADD, NAND, PRODUCT = 3, 4, 5, 6, 7, 8, 9


def build(force: bool = False) -> str:
    """Compile the C core with gcc (OpenMP, portable x86-64-v3 code)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-fopenmp", "-shared", "-fPIC",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
        u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
        c = ctypes
        L.rg_threads.restype = c.c_int
        L.rg_threads.argtypes = []
        L.rg_negmul.argtypes = [c.c_uint64, c.c_int, u64p, u64p, u64p]
        L.rg_encrypt.argtypes = [c.c_uint64, c.c_int, c.c_int, u64p, u64p, i64p, u8p, c.c_int64, u64p]
        L.rg_gate.restype = c.c_int
        L.rg_gate.argtypes = [c.c_uint64, c.c_int, c.c_int, c.c_int, u64p, u64p, u64p, c.c_int64]
        L.rg_gate_rows.restype = c.c_int
        L.rg_gate_rows.argtypes = [c.c_uint64, c.c_int, c.c_int, c.c_int, u64p, u64p, i64p,
                                   np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS"), c.c_int64, u64p]
        L.rg_blind_rotate.argtypes = [c.c_uint64, c.c_int, c.c_int, u64p, c.c_int64,
                                      np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS"), u64p, c.c_int64]
        L.rg_bootstrap.argtypes = [c.c_uint64, c.c_int, c.c_int, u64p, c.c_int64, u64p, c.c_int64, u64p]
        L.rg_keyswitch.argtypes = [c.c_uint64, c.c_int, c.c_int64, u64p, u64p, c.c_int64, u64p]
        L.rg_gate_bootstrap.restype = c.c_int
        L.rg_gate_bootstrap.argtypes = [c.c_uint64, c.c_int, c.c_int, c.c_int, u64p, c.c_int64, u64p, u64p, u64p,
                                        c.c_int64, u64p]
        L.rg_phase.argtypes = [c.c_uint64, c.c_int, c.c_int, u64p, c.c_int, u64p, u64p]
        L.rg_decrypt.argtypes = [c.c_uint64, c.c_int, c.c_int, u64p, c.c_int64, u64p, u8p]
        _lib = L
    return _lib


def _u64(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint64))


def mod_p(signed) -> np.ndarray:
    """Signed small integers -> their residues in [0, p)."""
    v = np.asarray(signed, dtype=np.int64)
    return np.where(v >= 0, v.astype(np.uint64), np.uint64(P) - (-v).astype(np.uint64))


def negmul(a, b) -> np.ndarray:
    """a*b in Z_p[X]/(X^d + 1), by the negacyclic convolution."""
    a, b = _u64(a), _u64(b)
    out = np.zeros_like(a)
    lib().rg_negmul(P, a.shape[0], a, b, out)
    return out


def encrypt(draws) -> np.ndarray:
    """Ciphertexts (n, ROWS, 2, d) of draws.bits under secret draws.s with masks
    draws.a and errors draws.e (paper_1611_08769_amd.workloads.ring_draws)."""
    n, rows, d = draws.a.shape
    assert rows == ROWS
    out = np.zeros((n, ROWS, 2, d), dtype=np.uint64)
    lib().rg_encrypt(P, d, ELL, _u64(mod_p(draws.s)), _u64(draws.a),
                     np.ascontiguousarray(draws.e, dtype=np.int64), draws.bits, n, out)
    return out


def gate(op: int, L, R=None) -> np.ndarray:
    """out[c] = op(L[c], R[c]) for stacks of ciphertexts (n, ROWS, 2, d)."""
    L = _u64(L)
    R = L if R is None else _u64(R)
    assert L.shape == R.shape and L.shape[1:3] == (ROWS, 2)
    out = np.zeros_like(L)
    if lib().rg_gate(P, L.shape[3], ELL, op, L, R, out, L.shape[0]) != 0:
        raise ValueError("unknown gate %d" % op)
    return out


def gate_rows(op: int, L, R, cts, rows) -> np.ndarray:
    """Rows rows[q] of op(L[cts[q]], R[cts[q]]), one by one: (count, 2, d)."""
    L, R = _u64(L), _u64(R)
    cts = np.ascontiguousarray(cts, dtype=np.int64)
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    d = L.shape[3]
    out = np.zeros((len(cts), 2, d), dtype=np.uint64)
    if lib().rg_gate_rows(P, d, ELL, op, L, R, cts, rows, len(cts), out) != 0:
        raise ValueError("unknown gate %d" % op)
    return out


def blind_rotate(bk, rot, acc) -> np.ndarray:
    """Blind rotation of ring-LWE accumulators acc (m, 2, d) by the ring-GSW
    key bk (n, ROWS, 2, d) with rotations rot (m, n) in [0, 2d): returns the
    accumulators after the n CMux steps (see rgsw_ref.c)."""
    bk = _u64(bk)
    out = np.array(acc, dtype=np.uint64, copy=True, order="C")
    rot = np.ascontiguousarray(rot, dtype=np.int32)
    m, n = rot.shape
    assert bk.shape[0] == n and out.shape == (m, 2, bk.shape[3])
    lib().rg_blind_rotate(P, bk.shape[3], ELL, bk, n, rot, out, m)
    return out


def bootstrap(bk, lwe) -> np.ndarray:
    """Gate bootstrapping of LWE ciphertexts lwe (m, n+1) mod p under the
    binary secret whose bits bk (n, ROWS, 2, d) encrypts: returns (m, d+1) LWE
    ciphertexts under the ring secret's coefficients (see rgsw_ref.c)."""
    bk, lwe = _u64(bk), _u64(lwe)
    m, n1 = lwe.shape
    assert bk.shape[0] == n1 - 1
    d = bk.shape[3]
    out = np.zeros((m, d + 1), dtype=np.uint64)
    lib().rg_bootstrap(P, d, ELL, bk, n1 - 1, lwe, m, out)
    return out


def keyswitch(ksk, lwe) -> np.ndarray:
    """Key switching of LWE ciphertexts lwe (m, d+1) under the ring secret to
    the LWE secret of the key-switching key ksk (d, 16, n+1): (m, n+1)."""
    ksk, lwe = _u64(ksk), _u64(lwe)
    d, K, n1 = ksk.shape
    assert K == 16 and lwe.shape[1] == d + 1
    out = np.zeros((lwe.shape[0], n1), dtype=np.uint64)
    lib().rg_keyswitch(P, d, n1 - 1, ksk, lwe, lwe.shape[0], out)
    return out


def gate_bootstrap(gate: int, bk, ksk, x, y) -> np.ndarray:
    """Bootstrapped gate (4 AND, 5 XOR, 6 OR, 8 NAND) on LWE ciphertexts x, y
    (m, n+1) mod p, bits encoded as mu * 2 * floor(p/8): (m, n+1) outputs in
    the same encoding under the same secret (see rgsw_ref.c)."""
    bk, ksk, x, y = _u64(bk), _u64(ksk), _u64(x), _u64(y)
    m, n1 = x.shape
    out = np.zeros_like(x)
    if lib().rg_gate_bootstrap(P, bk.shape[3], ELL, gate, bk, n1 - 1, ksk, x, y, m, out) != 0:
        raise ValueError("gate must be 4, 5, 6 or 8")
    return out


def lwe_phase(c, s_signed) -> int:
    """b - <a, s> mod p of one LWE ciphertext (a_0..a_{k-1}, b)."""
    k = len(c) - 1
    return (int(c[k]) - sum(int(c[i]) * int(s_signed[i]) for i in range(k))) % P


def rlwe_phase(acc, s_signed) -> np.ndarray:
    """b - a*s of one ring-LWE ciphertext (2, d)."""
    acc = _u64(acc)
    out = np.zeros(acc.shape[1], dtype=np.uint64)
    lib().rg_phase(P, acc.shape[1], ELL, acc, 0, _u64(mod_p(s_signed)), out)
    return out


def phase(ct, row: int, s_signed) -> np.ndarray:
    """C[row][0] - C[row][1]*s for one ciphertext (ROWS, 2, d)."""
    ct = _u64(ct)
    out = np.zeros(ct.shape[2], dtype=np.uint64)
    lib().rg_phase(P, ct.shape[2], ELL, ct, row, _u64(mod_p(s_signed)), out)
    return out


def decrypt(ct, s_signed) -> np.ndarray:
    """Bits of a stack of ciphertexts (n, ROWS, 2, d)."""
    ct = _u64(ct)
    out = np.zeros(ct.shape[0], dtype=np.uint8)
    lib().rg_decrypt(P, ct.shape[3], ELL, ct, ct.shape[0], _u64(mod_p(s_signed)), out)
    return out


def centred(x) -> np.ndarray:
    """Residues in [0, p) -> signed representatives in (-p/2, p/2] (Python ints)."""
    return np.array([int(v) if int(v) <= P // 2 else int(v) - P for v in np.asarray(x).ravel()],
                    dtype=object).reshape(np.shape(x))
