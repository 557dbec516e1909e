"""Write the expected decryptions of every request of the batched and served
mixes, using only the CPU oracle's integer fixed-point emulation (which the
encrypted FFT decrypts to exactly, the paper's Lemma "evaluation"): per
request its shape and the SHA-256 of its output words (int64, little-endian,
Re and Im interleaved, natural order).  bench.py compares the decryptions of
its batched and served runs against these.  Run:

    python tests/golden/make_mix_expect.py

The signals come from paper_1611_08769_amd.workloads, the seeded input
generator shared by both sides (it draws signals only).
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import fixedpoint as fx  # noqa: E402
from paper_1611_08769_amd import workloads as WL  # noqa: E402

BATCH = dict(seed=4, count=256, lengths=(8, 16, 32, 64, 128))
BATCH_SMALL = dict(seed=4, count=128, lengths=(8, 16, 32))
SERVE = dict(seed=5, count=64)


def expected_words(sig) -> np.ndarray:
    shape = (1, sig.length) if sig.dims == 1 else (1, sig.length, sig.length)
    re = fx.quantize(np.asarray(sig.re).ravel(), sig.F, sig.f).reshape(shape)
    im = (fx.quantize(np.asarray(sig.im).ravel(), sig.F, sig.f).reshape(shape) if sig.is_complex
          else np.zeros(shape, np.int64))
    er, ei = fx.fft_fixed(sig.dims, re, im, sig.F, sig.f)
    return np.stack([er.ravel(), ei.ravel()], 1).ravel().astype(np.int64)


def words_sha(words) -> str:
    return hashlib.sha256(np.ascontiguousarray(words, dtype="<i8").tobytes()).hexdigest()


def entry(sig) -> dict:
    return {"dims": sig.dims, "len": sig.length, "F": sig.F, "f": sig.f, "complex": bool(sig.is_complex),
            "words_sha256": words_sha(expected_words(sig))}


def main():
    out = {
        "what": "SHA-256 of the fixed-point emulation's output words per request (int64 little-endian, Re/Im "
                "interleaved, natural order); written by tests/golden/make_mix_expect.py from oracle/ only",
        "batch": dict(BATCH, lengths=list(BATCH["lengths"]),
                      requests=[entry(s) for s in WL.batch_requests(BATCH["seed"], BATCH["count"], BATCH["lengths"])]),
        "batch_small": dict(BATCH_SMALL, lengths=list(BATCH_SMALL["lengths"]),
                            requests=[entry(s) for s in WL.batch_requests(BATCH_SMALL["seed"], BATCH_SMALL["count"],
                                                                          BATCH_SMALL["lengths"])]),
        "serve": dict(SERVE, requests=[entry(s) for s in WL.served_requests(SERVE["seed"], SERVE["count"])]),
    }
    path = os.path.join(HERE, "mix_decryptions.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=0)
    print("wrote", path, len(out["batch"]["requests"]), len(out["batch_small"]["requests"]),
          len(out["serve"]["requests"]))


if __name__ == "__main__":
    main()
