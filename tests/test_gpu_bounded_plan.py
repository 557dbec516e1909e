"""GPU: a plan with a bounded workspace (list-scheduled levels,
sfft_plan_create_bounded) writes the same ciphertexts as the unbounded plan,
bit for bit, in a workspace within its bound, and its outputs decrypt to the
fixed-point emulation (the paper's Lemma "evaluation")."""
import sys

import numpy as np
import pytest
import torch

from oracle import fixedpoint as fx
from paper_1611_08769_amd import api

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [(1, 8, 8, 4, False), (2, 4, 8, 4, True)], ids=str)
def test_bounded_plan_matches_unbounded(shape):
    dims, L, F, f, cplx = shape
    print("[gpu-case] bounded plan", shape, flush=True)
    sys.stdout.flush()
    rng = np.random.default_rng(L * 7 + dims)
    pts = L if dims == 1 else L * L
    words = rng.integers(-(1 << (F - 1)), 1 << (F - 1), pts * (2 if cplx else 1)).astype(np.int64)
    p = api.size_params(dims, L, F, f, cplx, 1)
    keys = api.keygen(p, 11)
    ct_in = api.encrypt_words(keys, words, F, seed=11)
    free = api.Plan(dims, L, F, f, cplx, p)
    want = free.execute(ct_in)
    lim = free.ws_bytes // 2
    bnd = api.Plan(dims, L, F, f, cplx, p, ws_limit_bytes=lim)
    assert bnd.ws_bytes <= lim and bnd.info.levels > free.info.levels
    got = bnd.execute(ct_in)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    dec = api.decrypt_words(keys, got, 2 * pts, F)
    if dims == 1:
        re, im = (words, np.zeros_like(words)) if not cplx else (words[0::2], words[1::2])
        er, ei = fx.fft1d_fixed(re[None], im[None], F, f)
    else:
        re = words[0::2].reshape(1, L, L) if cplx else words.reshape(1, L, L)
        im = words[1::2].reshape(1, L, L) if cplx else np.zeros((1, L, L), np.int64)
        er, ei = fx.fft_fixed(2, re, im, F, f)
    assert dec.tolist() == np.stack([er.ravel(), ei.ravel()], 1).ravel().tolist()
    free.close()
    bnd.close()
