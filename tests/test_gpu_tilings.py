"""GPU: every product-kernel tiling, forced on a geometry it serves, gives
the oracle's gate outputs bit for bit; the tuner records a tiling that
plans then use."""
import sys

import numpy as np
import pytest
import torch

from oracle import gsw
from paper_1611_08769_amd import api
from paper_1611_08769_amd import sfft as S

pytestmark = pytest.mark.gpu

# (n_lwe, k) per digit-slot width: digits per row (n+1) * ceil(k/30) fill it
GEOS = {16: (1, 224), 32: (1, 480), 48: (1, 704), 64: (1, 960), 80: (1, 1184), 96: (1, 1440), 128: (3, 960)}


def _mfma_geos(nf):
    """Two geometries with nf 32-byte fragments per row: one filling them
    (n=1, 4W = 32 nf bytes) and a ragged one (4W = 32 nf - 12 bytes, W odd,
    so Nct = 32 W is an odd multiple of 32: a half chunk of R at the end and
    a partial row tile)."""
    w = 8 * nf - 3
    n1 = next(d for d in range(3, w + 1) if w % d == 0)
    return [(1, 128 * nf), (n1 - 1, 32 * (w // n1))]


def _cases():
    out = []
    for ti in range(S.sfft_tiling_count()):
        f = S.sfft_tiling_describe(ti)
        if f[6] == 0:
            out.append((ti, GEOS[f[1] * f[2]]))
        elif f[4] >= 2:
            # the 256-thread kernel serves rows of whole quads of words only
            # (its other geometries: tests/test_gpu_tiling_plans.py)
            out.append((ti, _mfma_geos(f[2] * f[3])[0]))
        else:
            for geo in _mfma_geos(f[2] * f[3]):
                out.append((ti, geo))
    return out


@pytest.mark.parametrize("ti,geo", _cases(), ids=lambda v: str(v))
def test_tiling_matches_oracle(ti, geo):
    n, k = geo
    print("[gpu-case] tiling %d n=%d k=%d" % (ti, n, k), flush=True)
    sys.stdout.flush()
    p = S.params(n, k)
    op = gsw.Params(n, k)
    rng = np.random.default_rng(ti * 7919 + k)
    L = rng.integers(0, 2**32, op.dims(), dtype=np.uint64).astype(np.uint32)
    R = rng.integers(0, 2**32, op.dims(), dtype=np.uint64).astype(np.uint32)
    R[::5] = 0xFFFFFFFF
    dl = torch.from_numpy(L.reshape(1, -1).view(np.int32)).cuda()
    dr = torch.from_numpy(R.reshape(1, -1).view(np.int32)).cuda()
    api.set_tiling(p, ti)
    try:
        for g, og in [(S.GATE_AND, 4), (S.GATE_XOR, 5)]:
            out = api.gate(p, g, dl, dr)
            torch.cuda.synchronize()
            got = out.cpu().numpy().view(np.uint32).reshape(-1)
            assert np.array_equal(got, gsw.gate(op, og, L, R).reshape(-1)), (ti, g)
    finally:
        api.set_tiling(p, -1)


def test_tuner_records_a_tiling_plans_use():
    p = S.params(1, 224)
    best, rates = api.tune(p, reps=2)
    assert best in rates and rates[best] == max(rates.values()) > 0
    plan = api.Plan(1, 8, 8, 4, False, p)
    assert plan.info.tiling == best
    plan.close()
    api.set_tiling(p, -1)
    plan = api.Plan(1, 8, 8, 4, False, p)
    assert S.sfft_tiling_describe(plan.info.tiling)[6] == 1  # the matrix-core default
    plan.close()


def test_plan_tuner_switches_plan_and_keeps_results():
    """Plan-level tuning on a small FFT: the plan switches to the fastest
    tiling and still gives the same ciphertexts as the default tiling."""
    from paper_1611_08769_amd import workloads as WL
    sig, n, seed = WL.workload("fft1d_n8_real_q8.4")
    p = api.size_params(1, 8, 8, 4, False, n)
    keys = api.keygen(p, seed)
    ct_in = api.encrypt_words(keys, api.signal_words(sig), 8, seed=seed)
    ref = api.Plan(1, 8, 8, 4, False, p)
    want = ref.execute(ct_in).clone()
    ref.close()
    plan = api.Plan(1, 8, 8, 4, False, p)
    best, rates = plan.tune(ct_in, reps=2)
    assert plan.info.tiling == best and rates[best] == max(rates.values())
    got = plan.execute(ct_in)
    torch.cuda.synchronize()
    assert torch.equal(got, want)
    plan.close()
    api.set_tiling(p, -1)
