"""The stored expected decryptions of the batched and served mixes
(tests/golden/mix_decryptions.json, which bench.py compares every output
against) are what the oracle's fixed-point emulation gives now for the same
seeded signals."""
import importlib.util
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def test_mix_expectations_match_the_emulation():
    spec = importlib.util.spec_from_file_location("make_mix_expect", os.path.join(HERE, "golden", "make_mix_expect.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    stored = json.load(open(os.path.join(HERE, "golden", "mix_decryptions.json")))
    sigs = {"batch": m.WL.batch_requests(m.BATCH["seed"], m.BATCH["count"], m.BATCH["lengths"]),
            "batch_small": m.WL.batch_requests(m.BATCH_SMALL["seed"], m.BATCH_SMALL["count"], m.BATCH_SMALL["lengths"]),
            "serve": m.WL.served_requests(m.SERVE["seed"], m.SERVE["count"])}
    for kind, ss in sigs.items():
        assert len(stored[kind]["requests"]) == len(ss)
        for e, sig in zip(stored[kind]["requests"], ss):
            assert e == m.entry(sig)
