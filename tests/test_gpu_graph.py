"""GPU: a plan replayed through its captured HIP graph gives the eager
ciphertexts on every replay, with other eager work and synchronisations
between the replays, and re-captures when the buffers change."""
import sys

import pytest
import torch

from paper_1611_08769_amd import api
from paper_1611_08769_amd import sfft as S
from paper_1611_08769_amd import workloads as WL

pytestmark = pytest.mark.gpu


def _pre_tiling(p):
    for ti in range(S.sfft_tiling_count()):
        f = S.sfft_tiling_describe(ti)
        if f[6] == 1 and f[4] == 1:
            try:
                api.set_tiling(p, ti)
                return ti
            except S.SfftError:
                continue
    return None


@pytest.mark.parametrize("pre", [False, True])
def test_graph_replays_equal_eager(pre):
    print("[gpu-case] graph replay fft1d_n8_real_q8.4 pre=%d" % pre, flush=True)
    sys.stdout.flush()
    sig, n, seed = WL.workload("fft1d_n8_real_q8.4")
    p = api.size_params(1, 8, 8, 4, False, n)
    if pre:
        # the captured sequence includes the transposition launches
        assert _pre_tiling(p) is not None
    try:
        _replays(sig, p, seed)
    finally:
        api.set_tiling(p, -1)


def _replays(sig, p, seed):
    keys = api.keygen(p, seed)
    ct_in = api.encrypt_words(keys, api.signal_words(sig), 8, seed=seed)
    plan = api.Plan(1, 8, 8, 4, False, p)
    want = plan.execute(ct_in).clone()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    out = torch.zeros_like(want)
    for rep in range(4):
        out.zero_()
        torch.cuda.synchronize()
        plan.execute_graph(ct_in, out, stream=s)
        s.synchronize()
        assert torch.equal(out, want), rep
        # unrelated eager work between replays
        x = torch.arange(1 << 20, device="cuda", dtype=torch.int32)
        assert int((x & 1).sum()) == 1 << 19
        torch.cuda.synchronize()
    # other buffers: captured again
    out2 = torch.zeros_like(want)
    plan.execute_graph(ct_in, out2, stream=s)
    s.synchronize()
    assert torch.equal(out2, want)
    plan.close()
