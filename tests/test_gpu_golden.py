"""Full-size parity on the named workloads against expected values that the
CPU oracle alone wrote (tests/golden/make_golden.py): SHA-256 of every input
and output ciphertext and the decrypted output words.  The GPU runs the
workload exactly as bench.py does (same keys, seeds, plan and launch
configuration); the oracle took about an hour per workload to produce them.
"""
import glob
import hashlib
import json
import os
import sys

import numpy as np
import pytest

from paper_1611_08769_amd import sfft as S
from paper_1611_08769_amd import workloads as WL

GOLDEN = sorted(glob.glob(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ciphertexts_*.json")))


def _load(path):
    with open(path) as fh:
        return json.load(fh)


def _sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u4").tobytes()).hexdigest()


@pytest.mark.parametrize("path", GOLDEN, ids=[os.path.basename(p)[12:-5] for p in GOLDEN])
def test_golden_netlist_and_parameters(path):
    """Host side: the library compiles the same canonical netlist and picks
    the same modulus as the oracle did for the stored run."""
    gd = _load(path)
    sig, n, seed = WL.workload(gd["workload"])
    shp = S.shape(sig.dims, sig.length, sig.F, sig.f, sig.is_complex)
    p = S.sfft_size_params(shp, n)
    assert (n, p.k, (n + 1) * p.k, seed) == (gd["n_lwe"], gd["k"], gd["nct"], gd["seed"])
    info = S.sfft_analyze(shp, p)
    assert info.netlist_sha256.decode() == gd["netlist_sha256"]
    assert info.n_inputs == gd["n_inputs"] and info.n_outputs == gd["n_outputs"]


@pytest.mark.gpu
@pytest.mark.parametrize("path", GOLDEN, ids=[os.path.basename(p)[12:-5] for p in GOLDEN])
def test_golden_ciphertexts_bit_exact(path):
    import torch
    from paper_1611_08769_amd import api

    gd = _load(path)
    print("[gpu-case] golden", gd["workload"], flush=True)
    sys.stdout.flush()
    sig, n, seed = WL.workload(gd["workload"])
    params = api.size_params(sig.dims, sig.length, sig.F, sig.f, sig.is_complex, n)
    keys = api.keygen(params, seed)
    ct_in = api.encrypt_words(keys, api.signal_words(sig), sig.F, seed=seed)
    torch.cuda.synchronize()
    assert _sha(ct_in.cpu().numpy().view(np.uint32)) == gd["inputs_sha256"]
    plan = api.Plan(sig.dims, sig.length, sig.F, sig.f, sig.is_complex, params)
    ct_out = plan.execute(ct_in)
    torch.cuda.synchronize()
    assert _sha(ct_out.cpu().numpy().view(np.uint32)) == gd["outputs_sha256"]
    dec = api.decrypt_words(keys, ct_out, len(gd["output_words"]), sig.F)
    assert dec.tolist() == gd["output_words"]
    plan.close()
