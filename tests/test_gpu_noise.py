"""GPU: the measured noise of output ciphertexts (sfft_noise_bits, host
arithmetic on rows read from the device) equals, in bits, the oracle's
measurement of the same ciphertexts (C' s = mu G s + e over every row, the
paper's Lemma "decryption"), and stays within the plan's worst-case bound,
for fresh encryptions and for the outputs of an encrypted FFT."""
import sys

import numpy as np
import pytest
import torch

from oracle import gsw
from paper_1611_08769_amd import api
from paper_1611_08769_amd import sfft as S

pytestmark = pytest.mark.gpu


def test_noise_measurement_matches_oracle_and_bound():
    print("[gpu-case] noise of N=8 real Q(8,4) outputs", flush=True)
    sys.stdout.flush()
    dims, L, F, f, cplx = 1, 8, 8, 4, False
    rng = np.random.default_rng(5)
    words = rng.integers(-(1 << (F - 1)), 1 << (F - 1), L).astype(np.int64)
    p = api.size_params(dims, L, F, f, cplx, 1)
    keys = api.keygen(p, 9)
    okeys = gsw.keygen(gsw.Params(p.n_lwe, p.k), 9)
    ct_in = api.encrypt_words(keys, words, F, seed=9)
    plan = api.Plan(dims, L, F, f, cplx, p)
    ct_out = plan.execute(ct_in)
    torch.cuda.synchronize()
    dec = api.decrypt_words(keys, ct_out, 2 * L, F)
    stream = torch.cuda.current_stream().cuda_stream
    for cts, bits in ((ct_in[:6], [(int(words[j // F]) >> (j % F)) & 1 for j in range(6)]),
                      (ct_out[5:17], [(int(dec[j // F]) >> (j % F)) & 1 for j in range(5, 17)])):
        sub = cts.contiguous()
        mu = np.array(bits, dtype=np.int32)
        got = S.sfft_noise_bits(p, keys.sk_host.ctypes.data, sub.data_ptr(), sub.shape[0], mu.ctypes.data, stream)
        host = sub.cpu().numpy().view(np.uint32).reshape(sub.shape[0], -1)
        want = max(gsw.max_noise(okeys, host[i].reshape(okeys.params.dims()), int(bits[i]))
                   for i in range(sub.shape[0]))
        assert got == want.bit_length()
        assert got <= plan.info.noise_bound_bits < p.k - 2
    plan.close()
