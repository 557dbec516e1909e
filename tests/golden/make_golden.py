"""Write full-size expected values for the named workloads using only the CPU
oracle: SHA-256 of every input and output ciphertext (the oracle's
encryption and its evaluation of the canonical netlist) and the decrypted
output words.  Run:  python tests/golden/make_golden.py <workload> [...]

The workloads' signals come from paper_1611_08769_amd.workloads, the seeded
input generator shared by both sides (it draws signals only).
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import fixedpoint as fx  # noqa: E402
from oracle import gsw  # noqa: E402
from oracle import netlist as N  # noqa: E402
from paper_1611_08769_amd import workloads as WL  # noqa: E402


def words_of(sig):
    re = fx.quantize(np.asarray(sig.re).ravel(), sig.F, sig.f)
    if sig.im is None:
        return re
    return np.stack([re, fx.quantize(np.asarray(sig.im).ravel(), sig.F, sig.f)], 1).ravel()


def sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a, dtype="<u4").tobytes()).hexdigest()


def make(name: str) -> dict:
    sig, n, seed = WL.workload(name)
    t0 = time.time()
    cn = N.Compact(N.build_fft_netlist(sig.dims, sig.length, sig.F, sig.f, sig.is_complex))
    k = N.choose_k(cn, n)
    p = gsw.Params(n, k)
    keys = gsw.keygen(p, seed)
    words = words_of(sig)
    cts = gsw.encrypt(keys, fx.words_to_bits(words, sig.F), seed=seed)
    print("[golden] %s: k=%d Nct=%d, %d inputs encrypted in %.0f s" % (name, k, p.nct, len(cts), time.time() - t0),
          flush=True)
    out = gsw.evaluate(p, cn, cts)
    print("[golden] %s: evaluated in %.0f s" % (name, time.time() - t0), flush=True)
    dec = fx.bits_to_words(gsw.decrypt_many(keys, out), sig.F)
    shape = (1, sig.length) if sig.dims == 1 else (1, sig.length, sig.length)
    re = fx.quantize(np.asarray(sig.re), sig.F, sig.f).reshape(shape)
    im = fx.quantize(np.asarray(sig.im), sig.F, sig.f).reshape(shape) if sig.is_complex else np.zeros(shape, np.int64)
    er, ei = fx.fft_fixed(sig.dims, re, im, sig.F, sig.f)
    emu = np.stack([er.ravel(), ei.ravel()], 1).ravel()
    assert dec.tolist() == emu.tolist(), "oracle decryption differs from the emulation"
    return {
        "workload": name,
        "n_lwe": n,
        "k": k,
        "nct": p.nct,
        "seed": seed,
        "netlist_sha256": cn.hash(),
        "n_inputs": int(len(cts)),
        "n_outputs": int(len(out)),
        "inputs_sha256": sha(cts),
        "outputs_sha256": sha(out),
        "output_words": [int(v) for v in dec],
        "oracle_seconds": round(time.time() - t0, 1),
        "written_by": "tests/golden/make_golden.py (CPU oracle only)",
    }


if __name__ == "__main__":
    for name in sys.argv[1:]:
        res = make(name)
        path = os.path.join(HERE, "ciphertexts_%s.json" % name)
        with open(path, "w") as fh:
            json.dump(res, fh, indent=1)
        print("[golden] wrote", path, flush=True)
