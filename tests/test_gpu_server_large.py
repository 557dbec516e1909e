"""GPU: requests at the shapes of the batched and served mixes, run through
the request loop together, against the same plans run alone, the integer
fixed-point emulation and the CPU oracle.

The mix holds real requests of both mixes (workloads "batch4_req<i>" and
"serve5_req<i>": same signal, keys and encryption seeds as the benchmark):
a 1D N=128 request at F=24 (k=928), a 1D N=256 request and a 16x16 image at
Q(16,8), and five small requests whose outputs the oracle wrote beforehand
(tests/golden/make_golden.py).  Every output decrypts to the emulation
(Theorem 1 / Lemma "evaluation": the circuit computes the fixed-point FFT
exactly), every request's ciphertexts are bit-identical alone and in the mix
(tolerance 0: all arithmetic is integer), and the five are bit-identical to
the oracle's.  Both step policies of the loop run: lockstep and
least-remaining-work fill.
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest
import torch

from oracle import fixedpoint as fx
from paper_1611_08769_amd import api
from paper_1611_08769_amd import workloads as WL

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
LARGE = ["batch4_req3", "serve5_req4", "serve5_req12"]
GOLDEN = ["batch4_req0", "batch4_req1", "batch4_req6", "serve5_req8", "serve5_req16"]


def say(msg):
    print("[gpu-case]", msg, flush=True)
    sys.stdout.flush()


def _sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u4").tobytes()).hexdigest()


def _emulate(sig):
    shape = (1, sig.length) if sig.dims == 1 else (1, sig.length, sig.length)
    re = fx.quantize(np.asarray(sig.re), sig.F, sig.f).reshape(shape)
    im = (fx.quantize(np.asarray(sig.im), sig.F, sig.f).reshape(shape) if sig.is_complex
          else np.zeros(shape, np.int64))
    er, ei = fx.fft_fixed(sig.dims, re, im, sig.F, sig.f)
    return np.stack([er.ravel(), ei.ravel()], 1).ravel()


class Req:
    def __init__(self, name):
        self.name = name
        self.sig, n, self.seed = WL.workload(name)
        s = self.sig
        self.params = api.size_params(s.dims, s.length, s.F, s.f, s.is_complex, n)
        self.keys = api.keygen(self.params, self.seed)
        self.ct_in = api.encrypt_words(self.keys, api.signal_words(s), s.F, seed=self.seed)
        self.plan = api.Plan(s.dims, s.length, s.F, s.f, s.is_complex, self.params)
        gpath = os.path.join(HERE, "golden", "ciphertexts_%s.json" % name)
        self.golden = json.load(open(gpath)) if os.path.exists(gpath) else None

    def out(self):
        return torch.zeros((self.plan.info.n_outputs, self.plan.ct_words), dtype=torch.int32, device="cuda")


@pytest.fixture(scope="module")
def mix():
    reqs = []
    for name in LARGE + GOLDEN:
        say("mix request %s" % name)
        reqs.append(Req(name))
    alone = []
    for r in reqs:
        say("alone %s k=%d" % (r.name, r.params.k))
        o = r.plan.execute(r.ct_in)
        torch.cuda.synchronize()
        r.plan._ws = None  # one plan workspace alive at a time
        alone.append(o)
    torch.cuda.empty_cache()
    yield reqs, alone
    for r in reqs:
        r.plan.close()


def test_mix_shapes():
    """The mix covers the extremes it is meant to."""
    shapes = {}
    for name in LARGE + GOLDEN:
        s = WL.workload(name)[0]
        shapes[name] = (s.dims, s.length, s.F)
    assert shapes["batch4_req3"] == (1, 128, 24)
    assert shapes["serve5_req4"] == (1, 256, 16)
    assert shapes["serve5_req12"] == (2, 16, 16)
    assert shapes["serve5_req16"] == (2, 8, 16)


def test_alone_matches_emulation_and_oracle(mix):
    reqs, alone = mix
    for r, o in zip(reqs, alone):
        say("check alone %s" % r.name)
        s = r.sig
        dec = api.decrypt_words(r.keys, o, 2 * s.points, s.F)
        assert dec.tolist() == _emulate(s).tolist(), r.name
        if r.golden is not None:
            assert _sha(r.ct_in.cpu().numpy().view(np.uint32)) == r.golden["inputs_sha256"], r.name
            assert _sha(o.cpu().numpy().view(np.uint32)) == r.golden["outputs_sha256"], r.name
            assert dec.tolist() == r.golden["output_words"], r.name


@pytest.mark.parametrize("fill_blocks", [0, 2048])
def test_batched_equals_alone_large(mix, fill_blocks):
    reqs, alone = mix
    say("server mix of %d requests, fill_blocks=%d" % (len(reqs), fill_blocks))
    budget = sum(r.plan.ws_bytes for r in reqs) + (1 << 30)
    srv = api.Server(budget, fill_blocks=fill_blocks)
    outs, tickets = [], []
    for r in reqs:
        o = r.out()
        outs.append(o)
        tickets.append(srv.submit_plan(r.plan, r.ct_in, o))
    srv.drain()
    torch.cuda.synchronize()
    st = srv.stats()
    assert st.completed == len(reqs)
    assert st.max_active == len(reqs)
    for r, o, a, t in zip(reqs, outs, alone, tickets):
        done, lat = srv.poll(t)
        assert done and lat > 0
        assert torch.equal(o, a), r.name
        s = r.sig
        dec = api.decrypt_words(r.keys, o, 2 * s.points, s.F)
        assert dec.tolist() == _emulate(s).tolist(), r.name
        if r.golden is not None:
            assert _sha(o.cpu().numpy().view(np.uint32)) == r.golden["outputs_sha256"], r.name
    srv.close()
