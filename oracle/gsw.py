"""Oracle: GSW13 over q = 2^k -- key generation, encryption, netlist
evaluation and decryption.  TEST INFRASTRUCTURE ONLY: the product path never
imports this module; tests, the smoke check and the benchmark's CPU-baseline
leg do.

Paper, section "Notation and Background": the scheme of Gentry, Sahai and
Waters (2013), LWE-based, with key generation (public/secret pair),
encryption, decryption and evaluation (addition, multiplication and NAND on
matrix ciphertexts over Z_q).  The paper does not fix parameters; this oracle
takes q = 2^k, ell = k, Nct = (n+1)k, m = Nct and errors in {-1, 0, 1}
(the readings are listed in the repository's design notes).  Nothing here is
secure at the sizes used: the parameters are sized for correctness only.

Secret s = (1, -t) and public A = [B t + e | B] satisfy A s = e.
A packed ciphertext C' = C G satisfies C' s = mu G s + e_C, so row k-1
(gadget entry 2^(k-1) on s_0 = 1) decrypts by rounding its inner product
with s to the nearest multiple of q/2.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

from . import prng

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsw_ref.c")
_LIB = os.path.join(_HERE, "libgsw_ref.so")


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
        u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
        i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        i8p = np.ctypeslib.ndpointer(dtype=np.int8, flags="C_CONTIGUOUS")
        u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")
        L.or_threads.restype = ctypes.c_int
        L.or_threads.argtypes = []
        L.or_set_threads.restype = None
        L.or_set_threads.argtypes = [ctypes.c_int]
        L.or_word.restype = ctypes.c_uint64
        L.or_word.argtypes = [ctypes.c_uint64] * 3
        L.or_words.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, u64p]
        L.or_product.argtypes = [ctypes.c_int] * 3 + [u32p, u32p, u32p]
        L.or_encrypt.argtypes = [ctypes.c_int] * 3 + [u32p, i32p, ctypes.c_int64, ctypes.c_uint64,
                                                      ctypes.c_uint64, u32p]
        L.or_gate.argtypes = [ctypes.c_int] * 4 + [u32p, u32p, u32p]
        L.or_eval.restype = ctypes.c_int
        L.or_eval.argtypes = [ctypes.c_int] * 4 + [i8p, i32p, i32p, ctypes.c_int, i32p, u32p, u32p]
        _lib = L
    return _lib


@dataclass(frozen=True)
class Params:
    n_lwe: int
    k: int

    def __post_init__(self):
        if self.k % 32 or self.k <= 0 or self.n_lwe < 1:
            raise ValueError("k must be a positive multiple of 32 and n >= 1")

    @property
    def n1(self):
        return self.n_lwe + 1

    @property
    def kw(self):
        return self.k // 32

    @property
    def nct(self):
        return self.n1 * self.k

    @property
    def m(self):
        return self.nct

    @property
    def q(self):
        return 1 << self.k

    @property
    def ct_words(self):
        return self.nct * self.n1 * self.kw

    def dims(self):
        return (self.nct, self.n1, self.kw)


# ---------------------------------------------------------------------------
# element <-> limb conversion
# ---------------------------------------------------------------------------
def to_limbs(vals, kw):
    """Python ints (mod 2^(32 kw)) -> uint32 limbs, little-endian."""
    out = np.zeros((len(vals), kw), dtype=np.uint32)
    for i, v in enumerate(vals):
        b = int(v).to_bytes(4 * kw, "little")
        out[i] = np.frombuffer(b, dtype="<u4")
    return out


def from_limbs(limbs) -> int:
    return int.from_bytes(np.ascontiguousarray(limbs, dtype="<u4").tobytes(), "little")


def gadget(p: Params) -> np.ndarray:
    """G as a packed ciphertext: row r = b*k + t holds 2^t in element b."""
    G = np.zeros((p.nct, p.n1, p.kw), dtype=np.uint32)
    for r in range(p.nct):
        b, t = divmod(r, p.k)
        G[r, b, t // 32] = np.uint32(1 << (t % 32))
    return G


# ---------------------------------------------------------------------------
# keys
# ---------------------------------------------------------------------------
@dataclass
class Keys:
    params: Params
    s: list  # n+1 ints mod q
    A: np.ndarray  # (m, n1, kw) uint32
    e: list  # m ints in {-1, 0, 1}


def keygen(p: Params, seed: int) -> Keys:
    q = p.q
    t = [prng.zq_element(seed, 1, i, p.k) for i in range(p.n_lwe)]
    s = [1] + [(-ti) % q for ti in t]
    A_int = []
    e = []
    for j in range(p.m):
        Bj = [prng.zq_element(seed, 2, j * p.n_lwe + i, p.k) for i in range(p.n_lwe)]
        ej = prng.ternary(seed, 3, j)
        bj = (sum(Bj[i] * t[i] for i in range(p.n_lwe)) + ej) % q
        A_int.append([bj] + Bj)
        e.append(ej)
    A = np.zeros((p.m, p.n1, p.kw), dtype=np.uint32)
    for j in range(p.m):
        A[j] = to_limbs(A_int[j], p.kw)
    return Keys(p, s, A, e)


# ---------------------------------------------------------------------------
# encryption / evaluation / decryption
# ---------------------------------------------------------------------------
def encrypt(keys: Keys, bits, seed: int, first_ct_id: int = 0) -> np.ndarray:
    """Packed ciphertexts (len(bits), Nct, n1, kw) of the given bits; the mask
    of ciphertext i uses counter id first_ct_id + i."""
    p = keys.params
    bits = np.ascontiguousarray(np.asarray(bits, dtype=np.int32) & 1)
    out = np.zeros((len(bits),) + p.dims(), dtype=np.uint32)
    if len(bits):
        lib().or_encrypt(p.nct, p.n1, p.kw, np.ascontiguousarray(keys.A).reshape(-1), bits,
                         len(bits), seed, first_ct_id, out.reshape(-1))
    return out


def product(p: Params, L: np.ndarray, R: np.ndarray) -> np.ndarray:
    out = np.zeros(p.dims(), dtype=np.uint32)
    lib().or_product(p.nct, p.n1, p.kw, np.ascontiguousarray(L).reshape(-1),
                     np.ascontiguousarray(R).reshape(-1), out.reshape(-1))
    return out


def gate(p: Params, gtype: int, X: np.ndarray, Y: np.ndarray | None = None) -> np.ndarray:
    out = np.zeros(p.dims(), dtype=np.uint32)
    Y = X if Y is None else Y
    lib().or_gate(p.nct, p.n1, p.kw, gtype, np.ascontiguousarray(X).reshape(-1),
                  np.ascontiguousarray(Y).reshape(-1), out.reshape(-1))
    return out


def evaluate(p: Params, cn, inputs: np.ndarray) -> np.ndarray:
    """Evaluate a compacted netlist (oracle.netlist.Compact) on packed input
    ciphertexts (n_inputs, Nct, n1, kw); returns (n_outputs, Nct, n1, kw)."""
    t = np.ascontiguousarray(np.array(cn.t, dtype=np.int8))
    a = np.ascontiguousarray(np.array(cn.a, dtype=np.int32))
    b = np.ascontiguousarray(np.array(cn.b, dtype=np.int32))
    outs = np.ascontiguousarray(np.array(cn.outputs, dtype=np.int32))
    inputs = np.ascontiguousarray(inputs, dtype=np.uint32)
    assert inputs.shape[0] == cn.n_inputs
    out = np.zeros((len(cn.outputs),) + p.dims(), dtype=np.uint32)
    rc = lib().or_eval(p.nct, p.n1, p.kw, len(cn.t), t, a, b, len(outs), outs,
                       inputs.reshape(-1) if inputs.size else np.zeros(1, np.uint32),
                       out.reshape(-1))
    if rc != 0:
        raise MemoryError("oracle evaluation ran out of memory")
    return out


def row_phase(keys: Keys, ct: np.ndarray, r: int) -> int:
    """<C'_r, s> mod q."""
    p = keys.params
    return sum(from_limbs(ct[r, b]) * keys.s[b] for b in range(p.n1)) % p.q


def decrypt(keys: Keys, ct: np.ndarray) -> int:
    p = keys.params
    x = row_phase(keys, ct, p.k - 1)
    return ((x + (1 << (p.k - 2))) % p.q) >> (p.k - 1)


def decrypt_many(keys: Keys, cts: np.ndarray) -> list[int]:
    return [decrypt(keys, c) for c in cts]


def centered(v: int, q: int) -> int:
    v %= q
    return v - q if v >= q // 2 else v


def max_noise(keys: Keys, ct: np.ndarray, mu: int) -> int:
    """max_r |<C'_r, s> - mu*2^t_r*s_b_r| (centred mod q): the noise e of
    C' s = mu G s + e, over every row."""
    p = keys.params
    worst = 0
    for r in range(p.nct):
        b, t = divmod(r, p.k)
        e = centered(row_phase(keys, ct, r) - mu * (1 << t) * keys.s[b], p.q)
        worst = max(worst, abs(e))
    return worst
