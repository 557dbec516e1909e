"""GPU: every matrix-core tiling that transposes the right operands in a pass
before the product launch (the 128-row chunk layout of the 512-thread kernel
and the 64-row layout of the 256-thread kernel, with its column splits of
whole elements and its rows that are not whole quads of words), forced on a
small encrypted FFT plan at chosen ciphertext geometries, gives the oracle's
ciphertexts bit for bit.  The plan's products
carry every epilogue form of the adders: AND, XOR and carries that add an
extra operand (the paper's Lemma "evaluation": the encrypted circuit
decrypts to the plain one)."""
import sys

import numpy as np
import pytest
import torch

from oracle import fixedpoint as fx
from oracle import gsw
from oracle import netlist as N
from paper_1611_08769_amd import api
from paper_1611_08769_amd import sfft as S

pytestmark = pytest.mark.gpu

SHAPE = (1, 2, 4, 2, True)  # N = 2 complex Q(4,2): 28 products in 4 levels


def _eps(n1, k, cf):
    """Elements per column split of the 256-thread kernel (the library's
    rule, restated to pick test geometries): the whole row where it fits
    64 cf byte columns, else the most whole elements that fit with every
    split on a multiple of 4 words."""
    W = n1 * k // 32
    if 4 * W <= 64 * cf:
        return n1
    if W % 4:
        return 0
    for e in range(n1 - 1, 0, -1):
        if e * k // 8 <= 64 * cf and (e * k // 32) % 4 == 0:
            return e
    return 0


def _served(n1, k, cf):
    e = _eps(n1, k, cf)
    if not e or 4 * n1 * k // 32 > 384:  # rows of at most 12 fragments
        return None
    cs = -(-n1 // e)
    ww = n1 * k // 32 if cs == 1 else e * k // 32  # words of a split row
    if cs > 1 and (ww % 4 or ww // 4 > 16):  # split rows: whole quads
        return None
    return cs if -(-(4 * ww) // 32) > 2 * (cf - 1) else None


def _ragged(nf):
    """A row of an odd number of words in nf fragments (a partial last
    fragment and unit, a half chunk of R at the end, quads of words that
    span rows), of n + 1 >= 3 elements of at least 2 limbs."""
    for w in range(8 * nf - 1, 8 * nf - 8, -2):
        for d in range(3, w // 2 + 1):
            if w % d == 0:
                return (d - 1, 32 * (w // d))
    raise AssertionError(nf)


def _geos(f):
    threads, rg, cgw, cf, pre = f[:5]
    nf = cgw * cf
    if pre == 1:
        return [(1, 128 * nf), _ragged(nf)]  # rows filling nf fragments; a ragged odd row
    # the 256-thread kernel: rows filling nf fragments; 4 elements of an odd
    # number of limbs (elements end inside quads); whole rows that are not
    # whole quads of words, which its epilogue takes two rows (an even
    # number of words: 2 elements of an odd number of limbs) or four rows
    # (an odd number: 3 elements of an odd number of limbs) at a time, a
    # quad then ending one row and starting the next (short rows: passes of
    # 32 or 64 rows, the last one partial where the tile is 32 or 96 rows)
    w2 = max(w for w in range(2, 16 * cf + 1, 4))
    wodd = max(w for w in range(3, 16 * cf + 1, 6))
    out = [(1, 128 * nf), (3, 32 * (4 * cf - 1)), (1, 32 * (w2 // 2)), (2, 32 * (wodd // 3))]
    if cf == 1:
        # rows of 5 words (Nct = 160): epilogue passes of 64 rows, the
        # second row tile's 32 rows a partial pass
        out.append((4, 32))
    # and the smallest geometry served in more than one column split
    best = None
    for n in (1, 2, 3):
        for k in range(32, 1025, 32):
            cs = _served(n + 1, k, cf)
            if cs and cs > 1 and (best is None or (n + 1) * k < (best[0] + 1) * best[1]):
                best = (n, k)
    if best:
        out.append(best)
    if pre == 3:
        # the tilings that transpose R in the workgroup hold all of its
        # chunks (64 rows of 4 cf KB, and 1 KB of bits of L) in 160 KB
        out = [(n, k) for n, k in out if -(-(n + 1) * k // 64) * (4 * cf + 1) * 1024 + 528 <= 160 * 1024]
    return out


def _cases():
    out = []
    for ti in range(S.sfft_tiling_count()):
        f = S.sfft_tiling_describe(ti)
        if f[6] == 1 and f[4] > 0:
            out += [(ti, g) for g in _geos(f)]
    return out


@pytest.mark.parametrize("ti,geo", _cases(), ids=lambda v: str(v))
def test_transposition_tiling_plan_matches_oracle(ti, geo):
    n, k = geo
    print("[gpu-case] plan tiling %d n=%d k=%d" % (ti, n, k), flush=True)
    sys.stdout.flush()
    dims, L, F, f, cplx = SHAPE
    p = S.params(n, k)
    rng = np.random.default_rng(ti * 131 + k)
    words = rng.integers(-(1 << (F - 1)), 1 << (F - 1), 2 * L).astype(np.int64)
    keys = api.keygen(p, 7)
    ct_in = api.encrypt_words(keys, words, F, seed=7)
    api.set_tiling(p, ti)
    try:
        plan = api.Plan(dims, L, F, f, cplx, p)
        assert plan.info.tiling == ti
        ct_out = plan.execute(ct_in)
        torch.cuda.synchronize()
        got = ct_out.cpu().numpy().view(np.uint32)
        plan.close()
    finally:
        api.set_tiling(p, -1)
    cn = N.Compact(N.build_fft_netlist(dims, L, F, f, cplx))
    okeys = gsw.keygen(gsw.Params(n, k), 7)
    want = gsw.evaluate(okeys.params, cn, gsw.encrypt(okeys, fx.words_to_bits(words, F), seed=7))
    assert np.array_equal(got, want.reshape(want.shape[0], -1)), (ti, geo)
    dec = api.decrypt_words(keys, ct_out, 2 * L, F)
    er, ei = fx.fft1d_fixed(words[0::2][None], words[1::2][None], F, f)
    assert dec.tolist() == np.stack([er[0], ei[0]], 1).ravel().tolist()
