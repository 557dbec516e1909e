"""GPU: sfft_execute_noalloc (the encrypted FFT with its workspace in the
library's fixed device array, for callers that cannot allocate) gives the
same ciphertexts as sfft_execute with a caller workspace, on two calls in a
row, the second on a smaller plan; a plan whose workspace exceeds the array
is refused before anything runs."""
import sys

import numpy as np
import pytest
import torch

from paper_1611_08769_amd import api
from paper_1611_08769_amd import sfft as S

pytestmark = pytest.mark.gpu


def _run(shape, seed):
    dims, L, F, f, cplx = shape
    rng = np.random.default_rng(seed)
    pts = L if dims == 1 else L * L
    words = rng.integers(-(1 << (F - 1)), 1 << (F - 1), pts * (2 if cplx else 1)).astype(np.int64)
    p = api.size_params(dims, L, F, f, cplx, 1)
    keys = api.keygen(p, seed)
    ct_in = api.encrypt_words(keys, words, F, seed=seed)
    plan = api.Plan(dims, L, F, f, cplx, p)
    assert plan.ws_bytes <= S.SFFT_NOALLOC_WS_BYTES
    want = plan.execute(ct_in)
    got = torch.zeros_like(want)
    stream = torch.cuda.current_stream().cuda_stream
    S.sfft_execute_noalloc(plan.handle, ct_in.data_ptr(), got.data_ptr(), stream)
    torch.cuda.synchronize()
    same = torch.equal(got, want)
    plan.close()
    return same


def test_noalloc_matches_execute_twice_second_smaller():
    # N=8 real Q(8,4): 5.8 MB of workspace; then N=4 complex Q(8,4): 0.6 MB
    for shape, seed in [((1, 8, 8, 4, False), 21), ((1, 4, 8, 4, True), 22)]:
        print("[gpu-case] noalloc", shape, flush=True)
        sys.stdout.flush()
        assert _run(shape, seed), shape


def test_noalloc_refuses_a_workspace_beyond_the_array():
    p = api.size_params(1, 16, 16, 8, True, 1)  # 183 MB of workspace
    plan = api.Plan(1, 16, 16, 8, True, p)
    assert plan.ws_bytes > S.SFFT_NOALLOC_WS_BYTES
    with pytest.raises(S.SfftError) as ei:
        S.sfft_execute_noalloc(plan.handle, 0, 0, torch.cuda.current_stream().cuda_stream)
    assert ei.value.code == S.SFFT_ENOMEM
    plan.close()
