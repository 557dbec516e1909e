"""GPU: requests of different shapes and parameter sets batched through the
request loop produce exactly the ciphertexts each produces alone, and those
decrypt to the integer fixed-point emulation (one request also checked
against the CPU oracle)."""
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

MIX = [
    (1, 8, 8, 4, False), (1, 4, 6, 3, True), (1, 16, 8, 4, True), (2, 4, 8, 4, False),
    (1, 8, 12, 6, True), (1, 8, 8, 4, True),
]


def say(msg):
    print("[gpu-case]", msg, flush=True)
    sys.stdout.flush()


def _request(i, sh):
    dims, L, F, f, cplx = sh
    seed = 100 + i
    sig = WL.uniform_pm1(seed, L, F, f, cplx) if dims == 1 else WL.image(seed, L, F, f)
    p = api.size_params(dims, L, F, f, cplx, 1)
    keys = api.keygen(p, seed)
    words = api.signal_words(sig)
    ct_in = api.encrypt_words(keys, words, F, seed=seed)
    return sig, p, keys, words, ct_in


def _emulate(sh, sig):
    dims, L, F, f, cplx = sh
    shape = (1, L) if dims == 1 else (1, L, L)
    re = fx.quantize(np.asarray(sig.re), F, f).reshape(shape)
    im = fx.quantize(np.asarray(sig.im), F, f).reshape(shape) if cplx else np.zeros(shape, np.int64)
    er, ei = fx.fft_fixed(dims, re, im, F, f)
    return np.stack([er.ravel(), ei.ravel()], 1).ravel()


def _pre_tiling(p):
    """A matrix-core tiling with the transposition pass that serves p, or None."""
    for ti in range(S.sfft_tiling_count()):
        f = S.sfft_tiling_describe(ti)
        if f[6] == 1 and f[4] == 1:
            try:
                api.set_tiling(p, ti)
                return ti
            except S.SfftError:
                continue
    return None


@pytest.mark.parametrize("staggered,pre", [(False, False), (True, False), (False, True)])
def test_batched_equals_alone(staggered, pre):
    say("server mix staggered=%d pre=%d" % (staggered, pre))
    reqs = [_request(i, sh) for i, sh in enumerate(MIX)]
    if pre:
        # every geometry of the mix on a transposition-pass tiling: merged
        # launches transpose each request's right operands into its own
        # workspace scratch
        for r in reqs:
            assert _pre_tiling(r[1]) is not None
    try:
        _batched_equals_alone(staggered, reqs)
    finally:
        if pre:
            for r in reqs:
                api.set_tiling(r[1], -1)


def _batched_equals_alone(staggered, reqs):
    outs_mix, outs_alone, tickets = [], [], []
    srv = api.Server(8 << 30)
    plans = []
    for i, (sh, (sig, p, keys, words, ct_in)) in enumerate(zip(MIX, reqs)):
        plan = api.Plan(*sh, p)
        plans.append(plan)
        out = torch.zeros((plan.info.n_outputs, plan.ct_words), dtype=torch.int32, device="cuda")
        outs_mix.append(out)
        # odd requests share the caller's compiled plan, even ones let the server compile
        tickets.append(srv.submit_plan(plan, ct_in, out) if i % 2 else srv.submit(*sh, p, ct_in, out))
        outs_alone.append(plan.execute(ct_in))
        if staggered and i == 2:
            for _ in range(3):
                srv.step()
    srv.drain()
    torch.cuda.synchronize()
    st = srv.stats()
    assert st.completed == len(MIX)
    assert st.max_active >= 3
    for i, (sh, (sig, p, keys, words, ct_in)) in enumerate(zip(MIX, reqs)):
        done, lat = srv.poll(tickets[i])
        assert done and lat > 0
        assert torch.equal(outs_mix[i], outs_alone[i]), (i, sh)
        npts = sh[1] if sh[0] == 1 else sh[1] ** 2
        dec = api.decrypt_words(keys, outs_mix[i], 2 * npts, sh[2])
        assert dec.tolist() == _emulate(sh, sig).tolist(), (i, sh)
    # one request against the oracle, bit for bit
    sh = MIX[0]
    sig, p, keys, words, ct_in = reqs[0]
    cn = N.Compact(N.build_fft_netlist(*sh))
    okeys = gsw.keygen(gsw.Params(1, p.k), 100)
    want = gsw.evaluate(okeys.params, cn, gsw.encrypt(okeys, fx.words_to_bits(words, sh[2]), seed=100))
    got = outs_mix[0].cpu().numpy().view(np.uint32)
    assert np.array_equal(got, want.reshape(want.shape[0], -1))
    srv.close()
    for plan in plans:
        plan.close()
