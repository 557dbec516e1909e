"""Decryption of device ciphertexts by every route the library offers, on
fresh encryptions (GSW decryption: the top gadget row of a ciphertext times
the secret key, rounded to its most significant bit): on the null stream, on
a side stream, and from a host copy of the whole ciphertexts.  Each route
must give back the encrypted words exactly, for several moduli (one, a few
and many 32-bit limbs) and a ragged count of ciphertexts.
"""
import sys

import numpy as np
import pytest
import torch

from paper_1611_08769_amd import api
from paper_1611_08769_amd import sfft as S

pytestmark = pytest.mark.gpu

CASES = [(64, 12, 1), (192, 16, 37), (640, 24, 129), (928, 8, 5)]


@pytest.mark.parametrize("k,F,count", CASES, ids=lambda c: str(c))
def test_decrypt_routes(k, F, count):
    print("[gpu-case] decrypt routes k=%d F=%d count=%d" % (k, F, count), flush=True)
    sys.stdout.flush()
    p = S.sfft_params(1, k, k * 2, 1)
    rng = np.random.default_rng(k + F)
    words = rng.integers(-(1 << (F - 1)), 1 << (F - 1), count)
    keys = api.keygen(p, 11)
    ct = api.encrypt_words(keys, words, F, seed=11)
    torch.cuda.synchronize()
    assert api.decrypt_words(keys, ct, count, F).tolist() == words.tolist()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        assert api.decrypt_words(keys, ct, count, F, stream=side).tolist() == words.tolist()
    host = np.ascontiguousarray(ct.cpu().numpy())
    out = np.zeros(count, dtype=np.int32)
    S.sfft_decrypt(p, keys.sk_host.ctypes.data, host.ctypes.data, count, F, 0, out.ctypes.data)
    assert out.tolist() == words.tolist()
    bits = api.decrypt_bits(keys, ct)
    want = ((words[:, None] >> np.arange(F)[None, :]) & 1).ravel()
    assert bits.tolist() == want.tolist()
