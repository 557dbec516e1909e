"""GPU parity: the HIP path against the CPU oracle, bit for bit.

Every ciphertext operation here is integer arithmetic mod 2^k, so the bar is
exact equality of every ciphertext word, and decryptions equal to the
integer fixed-point emulation."""
import sys

import numpy as np
import pytest
import torch

from oracle import fixedpoint as fx
from oracle import gsw
from oracle import netlist as N
from paper_1611_08769_amd import api
from paper_1611_08769_amd import sfft as S
from paper_1611_08769_amd import workloads as WL

pytestmark = pytest.mark.gpu


def say(msg):
    print("[gpu-case]", msg, flush=True)
    sys.stdout.flush()


def up(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a).reshape(a.shape[0], -1).view(np.int32)).cuda()


def down(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy().view(np.uint32)


def lib_keys(n, k, seed):
    p = S.params(n, k)
    return api.keygen(p, seed), gsw.keygen(gsw.Params(n, k), seed)


GEOS = [(1, 32), (1, 64), (2, 96), (1, 192), (1, 224), (3, 128)]


@pytest.mark.parametrize("n,k", GEOS)
def test_encrypt_matches_oracle(n, k):
    say("encrypt n=%d k=%d" % (n, k))
    keys, okeys = lib_keys(n, k, 11)
    bits = [int(b) for b in np.random.default_rng(k).integers(0, 2, 24)]
    ct = api.encrypt_words(keys, bits, 1, seed=11, first_ct_id=7)
    want = gsw.encrypt(okeys, bits, seed=11, first_ct_id=7)
    assert np.array_equal(down(ct), want.reshape(len(bits), -1))
    assert list(api.decrypt_bits(keys, ct)) == bits


@pytest.mark.parametrize("n,k", GEOS)
def test_gates_match_oracle(n, k):
    say("gates n=%d k=%d" % (n, k))
    keys, okeys = lib_keys(n, k, 5)
    op = okeys.params
    bits = [0, 1, 1, 0]
    cts = gsw.encrypt(okeys, bits, seed=5)
    d = up(cts)
    for g in (S.GATE_AND, S.GATE_XOR, S.GATE_OR, S.GATE_NAND, S.GATE_PRODUCT, S.GATE_NOT, S.GATE_XADD):
        for i, j in [(0, 1), (1, 2), (2, 3), (1, 1)]:
            if g == S.GATE_XADD and bits[i] & bits[j]:
                continue
            out = api.gate(keys, g, d[i:i + 1], d[j:j + 1])
            og = {S.GATE_NAND: None, S.GATE_PRODUCT: 4}.get(g, g)
            if og is None:
                want = gsw.gate(op, 3, gsw.gate(op, 4, cts[i], cts[j]))
            else:
                want = gsw.gate(op, og, cts[i], cts[j])
            assert np.array_equal(down(out).reshape(-1), want.reshape(-1)), (g, i, j)


@pytest.mark.parametrize("n,k", [(1, 32), (1, 96), (3, 64), (1, 416)])
def test_product_on_arbitrary_words(n, k):
    """The product kernel on uniformly random words (not ciphertexts): every
    limb carry pattern, all-ones words included."""
    say("random product n=%d k=%d" % (n, k))
    op = gsw.Params(n, k)
    rng = np.random.default_rng(n * 1000 + k)
    L = rng.integers(0, 2**32, op.dims(), dtype=np.uint64).astype(np.uint32)
    R = rng.integers(0, 2**32, op.dims(), dtype=np.uint64).astype(np.uint32)
    R[::3] = 0xFFFFFFFF
    L[1::5] = 0xFFFFFFFF
    p = S.params(n, k)
    dl, dr = up(L[None]), up(R[None])
    for g, og in [(S.GATE_AND, 4), (S.GATE_XOR, 5), (S.GATE_OR, 6)]:
        out = api.gate(p, g, dl, dr)
        assert np.array_equal(down(out).reshape(-1), gsw.gate(op, og, L, R).reshape(-1)), g


def _fft_case(dims, L, F, f, cplx, n, seed, sig=None):
    nl = N.build_fft_netlist(dims, L, F, f, cplx)
    cn = N.Compact(nl)
    k = N.choose_k(cn, n)
    if sig is None:
        if dims == 1:
            sig = WL.uniform_pm1(seed, L, F, f, cplx)
        else:
            sig = WL.image(seed, L, F, f)
    # the library side quantises with its own code; so does the oracle side
    words_lib = api.signal_words(sig)
    re = fx.quantize(np.asarray(sig.re).ravel(), F, f)
    words_or = np.stack([re, fx.quantize(np.asarray(sig.im).ravel(), F, f)], 1).ravel() if cplx else re
    assert np.array_equal(words_lib, words_or)
    return cn, k, sig, words_or


@pytest.mark.parametrize("dims,L,F,f,cplx", [
    (1, 2, 6, 3, True), (1, 4, 8, 4, True), (1, 8, 8, 4, False), (2, 4, 6, 3, False), (1, 8, 6, 3, True),
    # k = 288: 20 digits per row (8 lanes per row, 512-row tiles, two tiles, ragged tail); this is the shape
    # that exposed a race on the staged L words between waves at a chunk boundary
    (1, 16, 8, 4, True),
])
def test_fft_bit_exact_small(dims, L, F, f, cplx):
    """Whole encrypted FFTs: every output ciphertext equals the oracle's,
    decryptions equal the integer emulation."""
    n, seed = 1, 1
    cn, k, sig, words = _fft_case(dims, L, F, f, cplx, n, seed)
    say("fft dims=%d L=%d F=%d f=%d cplx=%d k=%d" % (dims, L, F, f, cplx, k))
    keys, okeys = lib_keys(n, k, seed)
    ct_in = api.encrypt_words(keys, words, F, seed=seed)
    plan = api.Plan(dims, L, F, f, cplx, keys.params)
    ct_out = plan.execute(ct_in)
    got = down(ct_out)
    o_in = gsw.encrypt(okeys, fx.words_to_bits(words, F), seed=seed)
    assert np.array_equal(down(ct_in), o_in.reshape(o_in.shape[0], -1))
    o_out = gsw.evaluate(okeys.params, cn, o_in)
    assert np.array_equal(got, o_out.reshape(o_out.shape[0], -1))
    npts = L if dims == 1 else L * L
    dec = api.decrypt_words(keys, ct_out, 2 * npts, F)
    shape = (1, L) if dims == 1 else (1, L, L)
    re = fx.quantize(np.asarray(sig.re), F, f).reshape(shape)
    im = fx.quantize(np.asarray(sig.im), F, f).reshape(shape) if cplx else np.zeros(shape, np.int64)
    er, ei = fx.fft_fixed(dims, re, im, F, f)
    assert dec.tolist() == np.stack([er.ravel(), ei.ravel()], 1).ravel().tolist()
    plan.close()


def test_fft_cfg_n8_real_q8_4():
    """1D N=8 real, Q(8,4), n=1: the smallest named workload, bit-exact."""
    sig, n, seed = WL.workload("fft1d_n8_real_q8.4")
    cn, k, sig, words = _fft_case(1, 8, 8, 4, False, n, seed, sig)
    say("fft cfg n8 real k=%d" % k)
    keys, okeys = lib_keys(n, k, seed)
    ct_in = api.encrypt_words(keys, words, 8, seed=seed)
    plan = api.Plan(1, 8, 8, 4, False, keys.params)
    got = down(plan.execute(ct_in))
    o_out = gsw.evaluate(okeys.params, cn, gsw.encrypt(okeys, fx.words_to_bits(words, 8), seed=seed))
    assert np.array_equal(got, o_out.reshape(o_out.shape[0], -1))
    plan.close()
