"""GPU, the paper-literal NAND-only circuit (every gate a NAND): ciphertexts
equal the oracle's evaluation of the same netlist (N=4, complex, Q(6,3)) and
decryptions equal the integer emulation (also N=8 real Q(8,4), the smallest
named workload's shape in NAND form)."""
import sys

import numpy as np
import pytest
import torch

from oracle import fixedpoint as fx
from oracle import gsw
from oracle import netlist as N
from paper_1611_08769_amd import api
from paper_1611_08769_amd import workloads as WL

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape,with_ciphertexts", [((1, 4, 6, 3, True), True), ((1, 8, 8, 4, False), False)])
def test_nand_only_fft(shape, with_ciphertexts):
    dims, L, F, f, cplx = shape
    print("[gpu-case] nand-only %s" % (shape,), flush=True)
    sys.stdout.flush()
    sig = WL.uniform_pm1(11, L, F, f, cplx)
    p = api.size_params(dims, L, F, f, cplx, 1, nand_only=True)
    keys = api.keygen(p, 11)
    words = api.signal_words(sig)
    ct_in = api.encrypt_words(keys, words, F, seed=11)
    plan = api.Plan(dims, L, F, f, cplx, p, nand_only=True)
    ct_out = plan.execute(ct_in)
    torch.cuda.synchronize()
    re = fx.quantize(np.asarray(sig.re), F, f).reshape(1, L)
    im = fx.quantize(np.asarray(sig.im), F, f).reshape(1, L) if cplx else np.zeros((1, L), np.int64)
    er, ei = fx.fft_fixed(1, re, im, F, f)
    dec = api.decrypt_words(keys, ct_out, 2 * L, F)
    assert dec.tolist() == np.stack([er.ravel(), ei.ravel()], 1).ravel().tolist()
    if with_ciphertexts:
        cn = N.Compact(N.build_fft_netlist(dims, L, F, f, cplx, nand_only=True))
        okeys = gsw.keygen(gsw.Params(1, p.k), 11)
        want = gsw.evaluate(okeys.params, cn, gsw.encrypt(okeys, fx.words_to_bits(words, F), seed=11))
        assert np.array_equal(ct_out.cpu().numpy().view(np.uint32), want.reshape(want.shape[0], -1))
    plan.close()
