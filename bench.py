"""Benchmark: encrypted FFT throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
    python bench.py --workload batch [--requests 64] [--max-len 128]
    python bench.py --workload serve [--requests 40] [--load 0.7] [--max-active 0]
    python bench.py --workload accuracy [--signals 4]
    python bench.py --workload ring_and_d1024 [--requests 128]   # ring-GSW gates
    python bench.py --workload ring_br_d1024 [--requests 1024]   # ring-GSW blind rotation
    python bench.py --workload ring_fft_<name>                  # a named FFT on bootstrapped gates

A step is one encrypted FFT of one request (every product level of the
compiled circuit, inputs already encrypted and resident in HBM).  Prints one
JSON line: canonical-netlist Boolean gates per second (AND+XOR+OR+XADD), FFT
points per second, per-step latency percentiles, the gate-product kernel's
roofline (the algorithmic work of the products per second, from HIP events
recorded around every product launch on the launch stream, against the
dense int8 matrix-core peak, or the table-lookup ceiling when the plan runs
the lookup kernel) and the CPU oracle's rate on a bounded sample of the same
products.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Gate-product kernel ceiling.  Any 4-bit table-lookup formulation reads one
# 4-byte table word per 4 L bits x 32 R bits = 128 bit-MACs, i.e. 32 bit-MAC
# per LDS byte; gfx950 LDS returns 64 banks x 4 B = 256 B/clk/CU (measured
# 204 B/clk/CU with ds_read_b128).  256 CUs at 2.4 GHz.
LDS_BYTES_PER_S = 256 * 256 * 2.4e9
PEAK_LOOKUP = LDS_BYTES_PER_S * 32.0   # 5.03e15 bit-MAC/s
# For reference, the AND + popcount formulation on the integer VALU
# (128 lanes/clk/CU, v_and_b32 + v_bcnt_u32_b32 per 32 bit-MACs).
PEAK_POPCOUNT = 256 * 128 * 2.4e9 * 16.0   # 1.26e15 bit-MAC/s
# Matrix-core kernel ceiling: MI355X dense int8 MFMA, 5.0 POP/s.  A product's
# algorithmic work, Nct^3 bit-MACs, is Nct x Nct x Nct/8 byte-MACs of its bits
# of L times the bytes of R, i.e. Nct^3 / 4 int8 operations.
PEAK_MFMA_I8 = 5.0e15                   # int8 op/s


def pct(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if xs else None


class _Window:
    """A run of consecutive nodes of a compacted netlist as a netlist of its
    own, in the oracle's Compact form (t, a, b, outputs, n_inputs)."""


def _oracle_window(cn, start, nprod):
    """Nodes [start, end) of the compacted netlist cn that hold nprod distinct
    products, as a netlist of their own: the earlier nodes they read become
    its inputs, and every node of the run that is read after it (or is an
    output) becomes one of its outputs, so the oracle evaluates each of its
    gates, linear ones included."""
    n = len(cn.t)
    last = [-1] * n
    for v in range(n):
        if cn.t[v] >= 3:
            last[cn.a[v]] = v
        if cn.t[v] >= 4:
            last[cn.b[v]] = v
    for o in cn.outputs:
        last[o] = n
    seen, end = set(), start
    while end < n and len(seen) < nprod:
        if cn.t[end] in (4, 5, 6, 8):
            seen.add((cn.a[end], cn.b[end]))
        end += 1
    w = _Window()
    w.t, w.a, w.b = [1, 2], [-1, -1], [-1, -1]  # the constants keep ids 0 and 1
    remap = {0: 0, 1: 1}
    body = [v for v in range(start, end) if cn.t[v] >= 3]
    for v in body:  # earlier nodes read by the run: its inputs
        for u in ((cn.a[v],) if cn.t[v] == 3 else (cn.a[v], cn.b[v])):
            if u < start and u not in remap:
                remap[u] = len(w.t)
                w.a.append(len(w.t) - 2)
                w.t.append(0)
                w.b.append(-1)
    w.n_inputs = len(w.t) - 2
    for v in body:
        remap[v] = len(w.t)
        w.t.append(cn.t[v])
        w.a.append(remap[cn.a[v]])
        w.b.append(remap[cn.b[v]] if cn.t[v] >= 4 else -1)
    w.outputs = [remap[v] for v in body if last[v] >= end]
    return w, len(seen)


def cpu_baseline(workload, nct, n1, kw, gates, canon_products, budget_s=12.0):
    """The oracle timed on the host: (1) a whole encrypted FFT of the small
    1D N=8 real Q(8,4) workload (n = 1, k = 192), decrypted against the
    fixed-point emulation; (2) on the named workload, a run of consecutive
    nodes from the middle of its canonical netlist (products and the linear
    gates between them, as the oracle evaluates them) sized to about
    budget_s, extrapolated to the whole FFT by its canonical products; (3)
    the oracle's product alone, on all threads and on one."""
    from oracle import fixedpoint as fx
    from oracle import gsw
    from oracle import netlist as N
    from paper_1611_08769_amd import workloads as WL

    threads = int(gsw.lib().or_threads())
    # (1) the small workload end to end
    sig, n_lwe, seed = WL.workload("fft1d_n8_real_q8.4")
    cn1 = N.Compact(N.build_fft_netlist(sig.dims, sig.length, sig.F, sig.f, sig.is_complex))
    keys = gsw.keygen(gsw.Params(n_lwe, 192), seed)
    words = fx.quantize(np.asarray(sig.re).ravel(), sig.F, sig.f)
    cts = gsw.encrypt(keys, fx.words_to_bits(words, sig.F), seed=seed)
    t0 = time.perf_counter()
    out = gsw.evaluate(keys.params, cn1, cts)
    full_s = time.perf_counter() - t0
    bits = gsw.decrypt_many(keys, out)
    got = [sum(b << i for i, b in enumerate(bits[j * sig.F:(j + 1) * sig.F])) for j in range(len(bits) // sig.F)]
    got = [v - (1 << sig.F) if v >= 1 << (sig.F - 1) else v for v in got]
    er, ei = fx.fft1d_fixed(words[None], np.zeros((1, sig.length), np.int64), sig.F, sig.f)
    exact = got == np.stack([er[0], ei[0]], 1).ravel().tolist()
    print("[bench] oracle: N=8 FFT in %.2f s (decrypts %s)" % (full_s, "exactly" if exact else "WRONG"),
          file=sys.stderr, flush=True)

    # (3) the product alone (also sizes the window)
    p = gsw.Params(n1 - 1, 32 * kw)
    rng = np.random.default_rng(0)
    L = rng.integers(0, 2**32, p.dims(), dtype=np.uint64).astype(np.uint32)
    R = rng.integers(0, 2**32, p.dims(), dtype=np.uint64).astype(np.uint32)
    gsw.product(p, L, R)  # warm the library and page in

    def per_product(budget):
        n, t0 = 0, time.perf_counter()
        while True:
            gsw.product(p, L, R)
            n += 1
            dt = time.perf_counter() - t0
            if dt >= budget and n >= 2:
                return dt / n, n

    t_prod, n_prod = per_product(1.0)
    gsw.lib().or_set_threads(1)
    try:
        t_one, n_one = per_product(budget_s / 4)
    finally:
        gsw.lib().or_set_threads(threads)

    # (2) a window of the named workload's own netlist
    wsig, _, _ = WL.workload(workload)
    cn = N.Compact(N.build_fft_netlist(wsig.dims, wsig.length, wsig.F, wsig.f, wsig.is_complex))

    def run_window(nprod):
        win, wprods = _oracle_window(cn, len(cn.t) // 2, nprod)
        ins = rng.integers(0, 2**32, (win.n_inputs,) + p.dims(), dtype=np.uint64).astype(np.uint32)
        t0 = time.perf_counter()
        gsw.evaluate(p, win, ins)
        return win, wprods, time.perf_counter() - t0

    _, pilot_prods, pilot_s = run_window(64)  # sizes the timed window
    win, wprods, win_s = run_window(max(64, int(budget_s * pilot_prods / pilot_s)))
    fft_s = win_s / wprods * canon_products
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {
        "value": gates / fft_s,
        "unit": "gates/s",
        "cores": threads,
        "kind": "oracle",
        "sample": "%d consecutive netlist nodes from the middle of the FFT's canonical netlist (%d distinct products "
                  "and the linear gates between them) evaluated by the oracle in %.2f s at Nct=%d (n+1=%d, k=%d), "
                  "random input ciphertexts; one FFT = %d canonical products -> %.0f s per FFT" % (
                      len(win.t) - 2 - win.n_inputs, wprods, win_s, nct, n1, 32 * kw, canon_products, fft_s),
        "small_fft_full_run": {"workload": "fft1d_n8_real_q8.4", "s_per_fft": full_s,
                               "products": len(cn1.products()), "decrypts_exactly": exact},
        "bitmac_per_s": nct ** 3 * wprods / win_s,
        "product_only_ms": t_prod * 1e3,
        "value_1_core": gates / (t_one * canon_products),
        "bitmac_per_s_1_core": nct ** 3 / t_one,
        "sample_1_core": "%d oracle products on 1 thread, %.2f ms each (product only)" % (n_one, t_one * 1e3),
        "cpu": model,
    }


def _mix_expect(kind):
    """Expected decryptions of the batched or served mix: per request the
    SHA-256 of the fixed-point emulation's output words, written by
    tests/golden/make_mix_expect.py from the CPU oracle alone."""
    with open(os.path.join(ROOT, "tests", "golden", "mix_decryptions.json")) as fh:
        return json.load(fh)[kind]


def _kernel_source_sha() -> str:
    """SHA-256 of the product kernels' source (kernels.hip, then the kernel
    body it includes): traffic figures taken with rocprofv3 hold only for it."""
    import hashlib
    h = hashlib.sha256()
    for name in ("kernels.hip", "mfma2_body.inc"):
        with open(os.path.join(ROOT, "paper_1611_08769_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _words_sha(words) -> str:
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(np.asarray(words), dtype="<i8").tobytes()).hexdigest()


def run_batch(args, count=None):
    """Independent 1D requests (length, word width and modulus differ per
    request), each encrypted right before it starts, its output decrypted
    and checked against the expected decryptions (the fixed-point emulation,
    stored by the oracle) as soon as it completes, its buffers freed then:
    first one at a time, then all through the request loop, where they enter
    in order while the ciphertexts of those in flight fit --io-gb.  Both
    runs do the same encryptions and decryptions; each request's output
    ciphertexts (first, middle and last) are compared between the two."""
    import collections
    import hashlib
    import torch
    from paper_1611_08769_amd import api
    from paper_1611_08769_amd import sfft as S
    from paper_1611_08769_amd import workloads as WL

    lengths = tuple(n for n in (8, 16, 32, 64, 128) if n <= args.max_len)
    count = count or args.requests or 256
    sigs = WL.batch_requests(seed=4, count=count, lengths=lengths)
    expect = None
    for kind in ("batch", "batch_small"):
        exp = _mix_expect(kind)
        if tuple(exp["lengths"]) == lengths and exp["seed"] == 4 and count <= exp["count"]:
            expect = exp["requests"]
    reqs, plans = [], {}
    for sig in sigs:
        p = api.size_params(1, sig.length, sig.F, sig.f, True, 1)
        key = (sig.length, sig.F, p.k)
        if key not in plans:
            plans[key] = api.Plan(1, sig.length, sig.F, sig.f, True, p)
        reqs.append((sig, p, plans[key]))

    def encrypt(i):
        sig, p, plan = reqs[i]
        keys = api.keygen(p, 1000 + i)
        return keys, api.encrypt_words(keys, api.signal_words(sig), sig.F, seed=1000 + i)

    def finish(i, keys, ct_out, stream=None):
        sig = reqs[i][0]
        dec = api.decrypt_words(keys, ct_out, 2 * sig.length, sig.F, stream=stream)
        ok = expect is None or _words_sha(dec) == expect[i]["words_sha256"]
        n = ct_out.shape[0]
        fp = hashlib.sha256(ct_out[[0, n // 2, n - 1]].cpu().numpy().tobytes()).hexdigest()
        return ok, fp

    # The client's work in the batched run (keys, encryption, decryption,
    # fingerprints) goes through a stream of its own, which does not wait for
    # the request loop's steps on the default stream: a request's inputs are
    # complete before it is submitted (this stream synchronised), and its
    # outputs once the loop reports it done.
    io = torch.cuda.Stream()

    def encrypt_io(i):
        with torch.cuda.stream(io):
            sig, p, _ = reqs[i]
            keys = api.keygen(p, 1000 + i)
            ct = api.encrypt_words(keys, api.signal_words(sig), sig.F, seed=1000 + i, stream=io)
        io.synchronize()
        return keys, ct

    def finish_io(i, keys, ct_out):
        with torch.cuda.stream(io):
            return finish(i, keys, ct_out, stream=io)

    # every distinct plan tuned once before the clock, on an encryption of
    # its first request (the same plans run alone and in the batch)
    tuned = {}
    if not args.no_tune:
        seen = set()
        for i, (sig, p, plan) in enumerate(reqs):
            if id(plan) in seen:
                continue
            seen.add(id(plan))
            _, ct = encrypt(i)
            best, _ = plan.tune(ct)
            plan._ws = None
            del ct
            tuned["%d/%d/k%d" % (sig.length, sig.F, p.k)] = list(S.sfft_tiling_describe(best))
        torch.cuda.empty_cache()
    torch.cuda.synchronize()
    gates = sum(r[2].info.gates for r in reqs)
    points = sum(r[0].points for r in reqs)
    bitmacs = sum(float(r[2].info.exec_products) * ((r[1].n_lwe + 1) * r[1].k) ** 3 for r in reqs)
    print("[bench] batch of %d requests: %d gates, %.2e bit-MACs, %d distinct plans" % (
        len(reqs), gates, bitmacs, len(plans)), file=sys.stderr, flush=True)

    # one request at a time (same plans)
    ok_alone, fp_alone = [None] * len(reqs), [None] * len(reqs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i, (sig, p, plan) in enumerate(reqs):
        keys, ct_in = encrypt(i)
        ct_out = torch.empty((plan.info.n_outputs, plan.ct_words), dtype=torch.int32, device="cuda")
        plan.execute(ct_in, ct_out)
        torch.cuda.synchronize()
        ok_alone[i], fp_alone[i] = finish(i, keys, ct_out)
        plan._ws = None  # keep at most one plan workspace alive (stream-ordered reuse)
        del ct_in, ct_out
    t_alone = time.perf_counter() - t0
    torch.cuda.empty_cache()
    print("[bench] one at a time: %.2f s" % t_alone, file=sys.stderr, flush=True)

    # batched: the request loop, fed while the ciphertexts in flight fit
    free, _ = torch.cuda.mem_get_info()
    io_cap = args.io_gb * 1e9
    budget = int(min(free * 0.7 - io_cap, (args.budget_gb or 120.0) * 1e9))
    fill = max(0, args.fill_blocks)
    srv = api.Server(budget, max_active=args.max_active, fill_blocks=fill, serial=args.serial_groups)
    ok_batch, fp_batch, lat = [None] * len(reqs), [None] * len(reqs), [None] * len(reqs)
    waiting = collections.deque(range(len(reqs)))
    live, io_used, max_live = {}, 0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while waiting or live:
        while waiting:
            i = waiting[0]
            plan = reqs[i][2]
            io_b = (plan.info.n_inputs + plan.info.n_outputs) * plan.ct_words * 4
            if live and io_used + io_b > io_cap:
                break
            keys, ct_in = encrypt_io(i)
            ct_out = torch.empty((plan.info.n_outputs, plan.ct_words), dtype=torch.int32, device="cuda")
            live[srv.submit_plan(plan, ct_in, ct_out)] = (i, keys, ct_out, io_b, time.perf_counter())
            io_used += io_b
            waiting.popleft()
        max_live = max(max_live, len(live))
        srv.step()
        for t in list(live):
            done, _ = srv.poll(t)
            if done:
                i, keys, ct_out, io_b, t_sub = live.pop(t)
                lat[i] = time.perf_counter() - t_sub
                ok_batch[i], fp_batch[i] = finish_io(i, keys, ct_out)
                io_used -= io_b
                del ct_out
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    same = fp_batch == fp_alone
    dec_ok = all(ok_alone) and all(ok_batch)
    if not dec_ok or not same:
        print("[bench] requests whose decryption differs: alone %s, batched %s; outputs differing: %s" % (
            [i for i, o in enumerate(ok_alone) if not o], [i for i, o in enumerate(ok_batch) if not o],
            [i for i in range(len(reqs)) if fp_batch[i] != fp_alone[i]]), file=sys.stderr, flush=True)
    print("[bench] batched: %.2f s (%d steps, %d launches, up to %d in flight); outputs identical to alone: %s; "
          "decryptions equal the emulation: %s" % (t_batch, st.steps, st.launches, max_live, same, dec_ok),
          file=sys.stderr, flush=True)
    torch.cuda.empty_cache()
    fixed = (fixed_batch(reqs, encrypt, finish, fp_alone, gates_of=lambda r: r[2].info.gates,
                         mem_gb=args.fixed_batch_gb) if args.fixed_batch_gb > 0 else None)
    ops = bitmacs / 4.0 / t_batch
    return {
        "metric": "encrypted gates/s (1 GPU, batched)",
        "value": gates / t_batch,
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": t_batch * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "data": "synthetic",
        "config": {"workload": "batch_1d_mixed", "requests": len(reqs), "lengths": "%d..%d" % (lengths[0], lengths[-1]),
                   "F": "12/16/24", "n_lwe": 1, "distinct_plans": len(plans), "budget_gb": round(budget / 1e9, 1),
                   "io_gb": args.io_gb, "fill_blocks": fill, "serial_groups": bool(args.serial_groups)},
        "tilings": tuned,
        "one_at_a_time_gates_per_s": gates / t_alone,
        "one_at_a_time_s": t_alone,
        "speedup_vs_one_at_a_time": t_alone / t_batch,
        "fft_points_per_s": points / t_batch,
        "bitmac_per_s": bitmacs / t_batch,
        "roofline": {"bound": "mfma", "achieved": ops / 1e12, "peak": PEAK_MFMA_I8 / 1e12, "unit": "TOP/s",
                     "frac": ops / PEAK_MFMA_I8, "dtype": "i8", "over": "whole batched run (wall time)"},
        "latency_p50_s": pct(lat, 50),
        "latency_p99_s": pct(lat, 99),
        "max_in_flight": max_live,
        "outputs_identical_to_alone": same,
        "all_decrypt_equal": dec_ok,
        "decrypt_checked": expect is not None,
        "fixed_batch_graph": fixed,
    }


def small_plan_latency(plan, ct_in, ct_out, args, reps=20):
    """For a plan whose widest level needs at most two rounds of the GPU's
    workgroup slots: the FFT as a launch per level, as those launches
    replayed in one HIP graph (sfft_execute_graph) and in one persistent
    launch (sfft_execute_persistent), latency per FFT from HIP events, and
    the outputs of each compared bit for bit."""
    import torch
    from paper_1611_08769_amd import sfft as S
    if plan.info.max_level_products * 3 > 512:  # (128-row tiles; the small workloads have Nct <= 384)
        return None
    ref = ct_out.clone()
    got = torch.zeros_like(ct_out)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    per_level = timed(lambda: plan.execute(ct_in, got))
    same = bool(torch.equal(got, ref))
    # the same launches replayed as one HIP graph (captured on a side stream)
    got.zero_()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        graph = timed(lambda: plan.execute_graph(ct_in, got, stream=side))
    torch.cuda.synchronize()
    same = same and bool(torch.equal(got, ref))
    try:
        got.zero_()
        persistent = timed(lambda: plan.execute_persistent(ct_in, got))
    except S.SfftError as e:
        return {"ms_per_fft_launch_per_level": per_level, "ms_per_fft_graph": graph, "outputs_identical": same,
                "persistent": "not served: %s" % e}
    timeouts = S.sfft_plan_persistent_timeouts(plan.handle)
    same = same and bool(torch.equal(got, ref))
    print("[bench] small plan: launch per level %.3f ms, graph %.3f ms, persistent %.3f ms per FFT (identical %s)" % (
        per_level, graph, persistent, same), file=sys.stderr, flush=True)
    return {"ms_per_fft_launch_per_level": per_level, "ms_per_fft_graph": graph, "ms_per_fft_persistent": persistent,
            "outputs_identical": same, "barrier_timeouts": timeouts, "ffts": reps}


def output_checks(workload, keys, ct_out, sig, info, params, samples=16):
    """The timed run's outputs against the oracle's stored ones (SHA-256 of
    the output ciphertexts and the decrypted words, tests/golden, written
    from the oracle alone), and the noise measured on evenly spaced output
    ciphertexts against the plan's worst-case bound."""
    import hashlib
    import torch
    from paper_1611_08769_amd import api
    from paper_1611_08769_amd import sfft as S

    n_vals = 2 * sig.points
    dec = api.decrypt_words(keys, ct_out, n_vals, sig.F)
    parity = None
    gpath = os.path.join(ROOT, "tests", "golden", "ciphertexts_%s.json" % workload)
    if os.path.exists(gpath):
        gd = json.load(open(gpath))
        h = hashlib.sha256(np.ascontiguousarray(ct_out.cpu().numpy().view(np.uint32), dtype="<u4").tobytes())
        parity = {"outputs_sha256_equal_oracle": h.hexdigest() == gd["outputs_sha256"],
                  "decrypt_equal_oracle": dec.tolist() == gd["output_words"], "golden": os.path.basename(gpath)}
    n_out = int(info.n_outputs)
    idx = sorted({int(round(j * (n_out - 1) / (samples - 1))) for j in range(samples)})
    mu = np.array([(int(dec[j // sig.F]) >> (j % sig.F)) & 1 for j in idx], dtype=np.int32)
    sub = ct_out[torch.tensor(idx, device=ct_out.device)].contiguous()
    torch.cuda.synchronize()
    measured = S.sfft_noise_bits(keys.params, keys.sk_host.ctypes.data, sub.data_ptr(), len(idx), mu.ctypes.data,
                                 torch.cuda.current_stream().cuda_stream)
    noise = {"measured_max_bits": measured, "bound_bits": int(info.noise_bound_bits), "k": int(params.k),
             "sampled_outputs": len(idx), "what": "bit length of the largest |e| over every row of the sampled "
             "output ciphertexts (C' s = mu G s + e) against the plan's worst-case bound; decryption is correct "
             "while it stays below k - 2 bits"}
    print("[bench] outputs: parity %s; noise %d bits measured, bound %d, k = %d" % (
        parity, measured, info.noise_bound_bits, params.k), file=sys.stderr, flush=True)
    return parity, noise


def fixed_batch(reqs, encrypt, finish, fp_alone, gates_of, mem_gb):
    """The first requests of the mix whose ciphertexts and workspaces fit
    mem_gb, inputs encrypted before the clock, run as one fixed batch
    (sfft_batch: the merged levels compiled once, captured into a HIP graph
    on the first execution, replayed after) against the same requests one at
    a time (each plan executed and waited for in turn).  Device work only:
    no encryption or decryption in the timed regions.  Every output is
    compared with the one-at-a-time run of the batched bench and decrypted."""
    import torch
    from paper_1611_08769_amd import api

    take, used = [], 0.0
    for i, (sig, p, plan) in enumerate(reqs):
        need = (plan.info.n_inputs + plan.info.n_outputs) * plan.ct_words * 4 + plan.ws_bytes
        if take and used + need > mem_gb * 1e9:
            break
        take.append(i)
        used += need
    ins, outs, keyz = {}, {}, {}
    for i in take:
        keyz[i], ins[i] = encrypt(i)
        plan = reqs[i][2]
        outs[i] = torch.empty((plan.info.n_outputs, plan.ct_words), dtype=torch.int32, device="cuda")
    gates = sum(gates_of(reqs[i]) for i in take)
    # one at a time
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in take:
        reqs[i][2].execute(ins[i], outs[i])
        torch.cuda.synchronize()
    t_alone = time.perf_counter() - t0
    for i in take:
        reqs[i][2]._ws = None
    torch.cuda.empty_cache()
    batch = api.Batch([(reqs[i][2], ins[i], outs[i]) for i in take])
    stream = torch.cuda.Stream()
    for i in take:
        outs[i].zero_()
    torch.cuda.synchronize()
    batch.execute_graph(stream)  # capture, instantiate, run
    stream.synchronize()
    t0 = time.perf_counter()
    batch.execute_graph(stream)
    stream.synchronize()
    t_graph = time.perf_counter() - t0
    t0 = time.perf_counter()
    batch.execute()
    torch.cuda.synchronize()
    t_eager = time.perf_counter() - t0
    res = [finish(i, keyz[i], outs[i]) for i in take]
    same = all(res[j][1] == fp_alone[i] for j, i in enumerate(take))
    dec_ok = all(r[0] for r in res)
    out = {"requests": len(take), "ciphertexts_and_workspace_gb": round(used / 1e9, 1), "steps": batch.steps,
           "launches": batch.launches, "graph_s": t_graph, "eager_s": t_eager, "one_at_a_time_s": t_alone,
           "gates_per_s_graph": gates / t_graph, "gates_per_s_one_at_a_time": gates / t_alone,
           "speedup_graph_vs_one_at_a_time": t_alone / t_graph, "outputs_identical_to_alone": same,
           "all_decrypt_equal": dec_ok}
    print("[bench] fixed batch of %d requests: graph %.2f s, eager %.2f s, one at a time %.2f s; identical %s, "
          "decrypt %s" % (len(take), t_graph, t_eager, t_alone, same, dec_ok), file=sys.stderr, flush=True)
    batch.close()
    del ins, outs
    torch.cuda.empty_cache()
    return out


def copy_probe():
    """A plain device copy of 1 GiB, three times: the reference against which
    the HBM counters FETCH_SIZE and WRITE_SIZE are scaled."""
    import torch
    n = 256 * 1024 * 1024  # int32 elements = 1 GiB
    x = torch.ones(n, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print("[bench] copied 1 GiB three times", flush=True)


def _is_gate_product(name):
    """A gate-product launch of either kernel (encryption launches excluded)."""
    return ("k_product<" in name and "false>" in name) or "k_product_mfma<" in name or "k_product_mfma2<" in name


def _counter_rows(path, kernel_prefix):
    import csv
    vals = []
    with open(path) as f:
        for row in csv.DictReader(f):
            if row["Kernel_Name"].startswith(kernel_prefix):
                vals.append(float(row["Counter_Value"]))
    return vals


def traffic_summary(workload, fetch_csv, write_csv, copy_fetch_csv, copy_write_csv):
    """HBM bytes per k_product launch (encryption launches excluded) from the
    rocprofv3 counter CSVs of one bench step, each counter scaled by what it
    reads for the 1 GiB copy; written next to the kernel trace summaries."""
    prod = "void sfft::(anonymous namespace)::k_product"
    fetch = [v for v, n in zip(_counter_rows(fetch_csv, prod), _kernel_names(fetch_csv, prod)) if _is_gate_product(n)]
    write = [v for v, n in zip(_counter_rows(write_csv, prod), _kernel_names(write_csv, prod)) if _is_gate_product(n)]
    # the run tunes the plan first: keep the product launches of the one
    # timed FFT, which come last (one per level)
    levels = _product_levels(workload)
    fetch, write = fetch[-levels:], write[-levels:]
    cf = max(_counter_rows(copy_fetch_csv, "__amd_rocclr_copyBuffer"))
    cw = max(_counter_rows(copy_write_csv, "__amd_rocclr_copyBuffer"))
    gib = float(1 << 30)
    fetch_scale, write_scale = gib / (cf * 1024), gib / (cw * 1024)
    fk, wk = sum(fetch) / len(fetch), sum(write) / len(write)
    names = [n for n in _kernel_names(fetch_csv, prod) if _is_gate_product(n)][-levels:]
    out = {
        "workload": workload,
        "kernel": sorted(set(n.replace("void sfft::(anonymous namespace)::", "").split("(")[0] for n in names)),
        "kernel_source_sha256": _kernel_source_sha(),
        "launches": len(fetch),
        "fetch_kib_per_launch": fk,
        "write_kib_per_launch": wk,
        "fetch_scale": fetch_scale,
        "write_scale": write_scale,
        "traffic_bytes_per_launch": (fk * fetch_scale + wk * write_scale) * 1024,
        "command": "rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) --output-format csv -- python3 bench.py "
                   "--workload %s --steps 1 --warmup 0 --no-cpu-baseline; the same for python3 bench.py "
                   "--copy-probe; python3 bench.py --traffic-summary on the four CSVs (the last FFT's "
                   "product launches, after the plan tuner's)" % workload,
    }
    path = os.path.join(ROOT, "profiles", "traffic_k_product_%s.json" % workload)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def ring_traffic_summary(workload, fetch_csv, write_csv, copy_fetch_csv, copy_write_csv):
    """HBM bytes of the last ring gate call (k_ring_fwd + k_ring_product) from
    the rocprofv3 counter CSVs of a bench run, each counter scaled by what it
    reads for the 1 GiB copy."""
    import csv
    import hashlib

    def per_call(path):
        rows = [(r["Kernel_Name"], float(r["Counter_Value"])) for r in csv.DictReader(open(path))]
        fwd = [v for n, v in rows if "k_ring_fwd" in n]
        prod = [v for n, v in rows if "k_ring_product" in n]
        return fwd[-1] + prod[-1], prod[-1]

    (fk, fk_prod), (wk, wk_prod) = per_call(fetch_csv), per_call(write_csv)
    cf = max(_counter_rows(copy_fetch_csv, "__amd_rocclr_copyBuffer"))
    cw = max(_counter_rows(copy_write_csv, "__amd_rocclr_copyBuffer"))
    gib = float(1 << 30)
    fetch_scale, write_scale = gib / (cf * 1024), gib / (cw * 1024)
    src = os.path.join(ROOT, "paper_1611_08769_amd", "csrc", "ring.hip")
    out = {
        "workload": workload,
        "kernel": "k_ring_fwd + k_ring_product",
        "ring_hip_sha256": hashlib.sha256(open(src, "rb").read()).hexdigest(),
        "fetch_kib_per_call": fk,
        "write_kib_per_call": wk,
        "fetch_kib_product": fk_prod,
        "write_kib_product": wk_prod,
        "fetch_scale": fetch_scale,
        "write_scale": write_scale,
        "traffic_bytes_per_call": (fk * fetch_scale + wk * write_scale) * 1024,
        "command": "rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) --output-format csv -- python3 bench.py "
                   "--workload %s --steps 1 --warmup 0 --no-cpu-baseline; the same for python3 bench.py "
                   "--copy-probe; python3 bench.py --traffic-summary on the four CSVs (the last gate call)" % workload,
    }
    path = os.path.join(ROOT, "profiles", "traffic_k_ring_product_%s.json" % workload)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


def _product_levels(workload):
    from paper_1611_08769_amd import sfft as S
    from paper_1611_08769_amd import workloads as WL
    sig, n_lwe, _ = WL.workload(workload)
    shp = S.shape(sig.dims, sig.length, sig.F, sig.f, sig.is_complex)
    return int(S.sfft_analyze(shp, S.sfft_size_params(shp, n_lwe)).levels)


def trace_summary(workload, db_path, steps):
    """Per-kernel statistics of a rocprofv3 kernel trace (rocpd database) of
    a bench run, and the average product launch over its `steps` timed FFTs
    (the last steps x levels product launches), for comparison with the
    bench's own HIP-event average."""
    import sqlite3
    cur = sqlite3.connect(db_path).cursor()
    rows = list(cur.execute("select name, duration from kernels order by start"))
    by = {}
    for name, d in rows:
        short = name.replace("sfft::", "").replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        by.setdefault(short, []).append(d)
    print("| kernel | calls | total (ms) | average (ms) | min (ms) | max (ms) |")
    print("|:--|--:|--:|--:|--:|--:|")
    for k, v in sorted(by.items(), key=lambda kv: -sum(kv[1])):
        print("| %s | %d | %.1f | %.4f | %.4f | %.4f |" % (k, len(v), sum(v) / 1e6, sum(v) / len(v) / 1e6,
                                                        min(v) / 1e6, max(v) / 1e6))
    if workload.startswith("ring_and_d"):
        # one gate call = one forward-transform launch + one product launch
        fwd = [d for name, d in rows if "k_ring_fwd" in name][-steps:]
        prod = [d for name, d in rows if "k_ring_product" in name][-steps:]
        print("\ntimed gate calls: %d, k_ring_fwd %.3f ms + k_ring_product %.3f ms = %.3f ms" % (
            len(prod), sum(fwd) / len(fwd) / 1e6, sum(prod) / len(prod) / 1e6, (sum(fwd) + sum(prod)) / len(prod) / 1e6))
        return
    prods = [d for name, d in rows if _is_gate_product(name)]
    timed = prods[-steps * _product_levels(workload):]
    print("\ntimed product launches: %d, average %.3f ms" % (len(timed), sum(timed) / len(timed) / 1e6))


def counter_summary(workload, csv_path):
    """Per-launch averages of every counter in a rocprofv3 --pmc CSV over the
    one timed FFT's product launches (the last one per level, after the
    plan tuner's), with the ratios read from them."""
    import csv
    per = {}
    for r in csv.DictReader(open(csv_path)):
        if _is_gate_product(r["Kernel_Name"]):
            per.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    levels = _product_levels(workload)
    avg = {k: sum(v[-levels:]) / len(v[-levels:]) for k, v in per.items()}
    print("| counter | per launch |")
    print("|:--|--:|")
    for k in sorted(avg):
        print("| %s | %.4g |" % (k, avg[k]))
    if "SQ_VALU_MFMA_BUSY_CYCLES" in avg and "GRBM_GUI_ACTIVE" in avg:
        # rocprofv3's MfmaUtil: MFMA-busy cycles summed over the 1024 SIMDs
        # over the launch's GUI-active cycles of one XCD (the CSV sums
        # GRBM_GUI_ACTIVE over the 8 XCDs)
        print("\nMFMA utilisation (MFMA busy / (GUI active per XCD x 1024 SIMDs)): %.3f" % (
            avg["SQ_VALU_MFMA_BUSY_CYCLES"] / (avg["GRBM_GUI_ACTIVE"] / 8 * 1024)))
    if "SQ_INSTS_MFMA" in avg and "SQ_INSTS_VALU" in avg:
        print("MFMA instructions / VALU instructions: %.3f" % (avg["SQ_INSTS_MFMA"] / avg["SQ_INSTS_VALU"]))
    if "SQ_LDS_BANK_CONFLICT" in avg and "SQ_LDS_IDX_ACTIVE" in avg:
        print("LDS bank-conflict cycles / LDS active cycles: %.3f" % (avg["SQ_LDS_BANK_CONFLICT"] / avg["SQ_LDS_IDX_ACTIVE"]))


def _kernel_names(path, kernel_prefix):
    import csv
    with open(path) as f:
        return [r["Kernel_Name"] for r in csv.DictReader(f) if r["Kernel_Name"].startswith(kernel_prefix)]


def run_serve(args, count=None):
    """Served traffic: requests (1D and 2D, Q(16,8), n_lwe=1, their own k)
    arrive as a Poisson process; each is encrypted on arrival, queued into
    the request loop, and its buffers freed when it completes.  Plans are
    compiled before the clock starts (a server keeps its plans).  Requests
    wait on the client side while the ciphertexts of those in flight would
    exceed --io-gb; latency runs from arrival to completion."""
    import collections
    import torch
    from paper_1611_08769_amd import api
    from paper_1611_08769_amd import sfft as S
    from paper_1611_08769_amd import workloads as WL

    sigs = WL.served_requests(seed=5, count=count or args.requests or 40)
    exp = _mix_expect("serve")
    expect = exp["requests"] if exp["seed"] == 5 and len(sigs) <= exp["count"] else None
    dec_ok = [None] * len(sigs)
    plans = {}
    for sig in sigs:
        key = (sig.dims, sig.length)
        if key not in plans:
            p = api.size_params(sig.dims, sig.length, sig.F, sig.f, sig.is_complex, 1)
            # plans whose levels-as-soon-as-possible workspace passes the
            # bound get list-scheduled levels within it
            shp = S.shape(sig.dims, sig.length, sig.F, sig.f, sig.is_complex)
            lim = int(args.plan_ws_gb * 1e9) if S.sfft_analyze(shp, p).ws_bytes > args.plan_ws_gb * 1e9 else 0
            plans[key] = (p, api.Plan(sig.dims, sig.length, sig.F, sig.f, sig.is_complex, p, ws_limit_bytes=lim))
            print("[bench] plan %s: k=%d exec products %d levels %d ws %.1f GB" % (
                key, p.k, plans[key][1].info.exec_products, plans[key][1].info.levels, plans[key][1].ws_bytes / 1e9),
                file=sys.stderr, flush=True)
    if not args.no_tune:
        # plans tuned before the clock, on an encryption of their first request
        for key, (p, plan) in plans.items():
            sig = next(s for s in sigs if (s.dims, s.length) == key)
            keys = api.keygen(p, 4999)
            ct = api.encrypt_words(keys, api.signal_words(sig), sig.F, seed=4999)
            best, _ = plan.tune(ct)
            plan._ws = None
            del ct
            print("[bench] plan %s tuned: tiling %s" % (key, list(S.sfft_tiling_describe(best))), file=sys.stderr,
                  flush=True)
        torch.cuda.empty_cache()
    def work(sig):
        p, plan = plans[(sig.dims, sig.length)]
        return float(plan.info.exec_products) * ((p.n_lwe + 1) * p.k) ** 3
    mean_work = sum(work(s) for s in sigs) / len(sigs)
    rate = args.rate if args.rate > 0 else args.load * args.rate_bitmac / mean_work
    arrivals = WL.poisson_arrivals(6, len(sigs), rate)
    free, _ = torch.cuda.mem_get_info()
    budget = int(min(free * 0.65, (args.budget_gb or 180.0) * 1e9))
    fill = 2048 if args.fill_blocks < 0 else args.fill_blocks
    srv = api.Server(budget, max_active=args.max_active, fill_blocks=fill)
    print("[bench] serve: %d requests, rate %.4f /s (load %.2f of %.2e bit-MAC/s), budget %.0f GB" % (
        len(sigs), rate, args.load, args.rate_bitmac, budget / 1e9), file=sys.stderr, flush=True)

    # client work (keys, encryption, decryption) on a stream of its own that
    # does not wait for the request loop's steps (see run_batch)
    io_s = torch.cuda.Stream()
    noise, per_req = [None] * len(sigs), []
    p_of = [plans[(sg.dims, sg.length)][0] for sg in sigs]
    waiting = collections.deque(range(len(sigs)))
    client_q = collections.deque()
    live = {}
    io_used, io_cap = 0, args.io_gb * 1e9
    lat, t_done = [None] * len(sigs), [None] * len(sigs)
    t0 = time.perf_counter()
    while waiting or client_q or live:
        now = time.perf_counter() - t0
        while waiting and arrivals[waiting[0]] <= now:
            client_q.append(waiting.popleft())
        # arrived requests enter in arrival order while their ciphertexts fit
        # (with the fill policy, later ones that fit may pass one that does not)
        for i in list(client_q):
            sig = sigs[i]
            p, plan = plans[(sig.dims, sig.length)]
            io = (plan.info.n_inputs + plan.info.n_outputs) * plan.ct_words * 4
            if live and io_used + io > io_cap:
                if fill > 0:
                    continue
                break
            with torch.cuda.stream(io_s):
                keys = api.keygen(p, 5000 + i)
                ct_in = api.encrypt_words(keys, api.signal_words(sig), sig.F, seed=5000 + i, stream=io_s)
            io_s.synchronize()
            ct_out = torch.empty((plan.info.n_outputs, plan.ct_words), dtype=torch.int32, device="cuda")
            live[srv.submit_plan(plan, ct_in, ct_out)] = (i, io, keys, ct_out)
            io_used += io
            client_q.remove(i)
        if live:
            srv.step()
            now = time.perf_counter() - t0
            for t in list(live):
                if srv.poll(t)[0]:
                    i, io, keys, ct_out = live.pop(t)
                    io_used -= io
                    lat[i], t_done[i] = now - arrivals[i], now
                    # decrypted against the expected decryptions (the emulation)
                    with torch.cuda.stream(io_s):
                        dec = api.decrypt_words(keys, ct_out, 2 * sigs[i].points, sigs[i].F, stream=io_s)
                        # the noise of 4 output ciphertexts against the plan's bound
                        n_out, Fi = ct_out.shape[0], sigs[i].F
                        idx = [0, n_out // 3, (2 * n_out) // 3, n_out - 1]
                        mu = np.array([(int(dec[j // Fi]) >> (j % Fi)) & 1 for j in idx], dtype=np.int32)
                        sub = ct_out[torch.tensor(idx, device=ct_out.device)].contiguous()
                        noise[i] = S.sfft_noise_bits(p_of[i], keys.sk_host.ctypes.data, sub.data_ptr(), len(idx),
                                                     mu.ctypes.data, io_s.cuda_stream)
                        del sub
                    dec_ok[i] = expect is None or _words_sha(dec) == expect[i]["words_sha256"]
                    del ct_out
                    bound = plans[(sigs[i].dims, sigs[i].length)][1].info.noise_bound_bits
                    print("[bench] request %d (%s %d) done: latency %.2f s, noise %d bits (bound %d, k %d)" % (
                        i, "2D" if sigs[i].dims == 2 else "1D", sigs[i].length, lat[i], noise[i], bound,
                        p_of[i].k), file=sys.stderr, flush=True)
                    per_req.append({"request": i, "shape": "%dD %d" % (sigs[i].dims, sigs[i].length),
                                    "latency_s": lat[i], "noise_bits": noise[i], "noise_bound_bits": bound,
                                    "k": p_of[i].k, "decrypt_equal": dec_ok[i]})
        elif waiting:
            time.sleep(max(0.0, min(0.05, arrivals[waiting[0]] - now)))
    torch.cuda.synchronize()
    wall = max(t_done) - float(arrivals[0])
    st = srv.stats()
    srv.close()
    gates = sum(plans[(s.dims, s.length)][1].info.gates for s in sigs)
    points = sum(s.points for s in sigs)
    bitmacs = sum(work(s) for s in sigs)
    return {
        "metric": "encrypted gates/s (1 GPU, served)",
        "value": gates / wall,
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": wall * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "data": "synthetic",
        "config": {"workload": "served_poisson", "requests": len(sigs), "mix": "1D 16..256 complex / 2D 8..32 real",
                   "F": 16, "f": 8, "n_lwe": 1, "rate_per_s": rate, "load": args.load,
                   "max_active": args.max_active, "fill_blocks": fill, "budget_gb": round(budget / 1e9, 1),
                   "io_gb": args.io_gb, "plan_ws_gb": args.plan_ws_gb,
                   "plans": {"%dd_%d" % k: {"levels": int(pl.info.levels), "ws_gb": round(pl.ws_bytes / 1e9, 1)}
                             for k, (_, pl) in plans.items()}},
        "fft_points_per_s": points / wall,
        "bitmac_per_s": bitmacs / wall,
        "latency_p50_s": pct(lat, 50),
        "latency_p99_s": pct(lat, 99),
        "latency_mean_s": float(np.mean(lat)),
        "requests_detail": per_req,
        "noise_within_bound": all(r["noise_bits"] <= r["noise_bound_bits"] for r in per_req),
        "steps_run": int(st.steps),
        "max_in_flight": int(st.max_active),
        "all_decrypt_equal": all(dec_ok),
        "decrypt_checked": expect is not None,
    }


def run_accuracy(args):
    """The paper's accuracy experiment in its own format, on the encrypted
    path: random complex signals in [0, 1), Q(32,16), N = 8..128.  Each
    signal is encrypted, transformed and decrypted on the GPU; the error is
    |decrypted - float64 FFT| per real component (2N values per signal),
    summarised as the paper's Table 1 (total, mean, population variance and
    standard deviation), printed beside the paper's rows."""
    import torch
    from paper_1611_08769_amd import api
    from paper_1611_08769_amd import workloads as WL

    paper = json.load(open(os.path.join(ROOT, "tests", "golden", "table1_errors.json")))["rows_1d"]
    rows, gates, t_gpu = {}, 0, 0.0
    for n in (8, 16, 32, 64, 128):
        p = api.size_params(1, n, 32, 16, True, 1)
        plan = api.Plan(1, n, 32, 16, True, p)
        errs = []
        u = WL.Uniforms(7000 + n)
        for j in range(args.signals):
            sig = WL.unit_complex(0, n, stream=u)
            keys = api.keygen(p, 7000 + 100 * n + j)
            ct_in = api.encrypt_words(keys, api.signal_words(sig), 32, seed=7000 + 100 * n + j)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ct_out = plan.execute(ct_in)
            torch.cuda.synchronize()
            t_gpu += time.perf_counter() - t0
            gates += plan.info.gates
            w = api.decrypt_words(keys, ct_out, 2 * n, 32).astype(np.float64) / 2.0 ** 16
            exact = np.fft.fft(np.asarray(sig.re) + 1j * np.asarray(sig.im))
            errs.append(np.abs(w[0::2] - exact.real))
            errs.append(np.abs(w[1::2] - exact.imag))
        e = np.concatenate(errs)
        rows[str(n)] = {"signals": args.signals, "k": p.k, "total": float(e.sum()), "mean": float(e.mean()),
                        "variance": float(e.var()), "sd": float(e.std()), "paper": paper[str(n)]}
        print("[bench] N=%d k=%d: mean %.3e sd %.3e (paper %.3e, %.3e)" % (
            n, p.k, e.mean(), e.std(), paper[str(n)][1], paper[str(n)][3]), file=sys.stderr, flush=True)
        plan.close()
    return {
        "metric": "encrypted gates/s (1 GPU, paper accuracy format)",
        "value": gates / t_gpu,
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": t_gpu * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8",
        "data": "synthetic",
        "config": {"workload": "accuracy_q32.16", "lengths": "8..128", "signals_per_length": args.signals,
                   "inputs": "complex, real and imaginary parts uniform in [0,1)", "n_lwe": 1},
        "table1": rows,
        "table1_columns": ["total", "mean", "variance", "sd"],
    }


# Ring-GSW gate ceiling.  A modular product of two residues below 2^62 needs
# the 128-bit product of two 64-bit words: at least four 32x32->64-bit
# partial products (v_mad_u64_u32), which issue at half the VALU's full rate
# (32 lanes/clk/CU; a register-only loop measures 34 per CU per clock at
# 2.4 GHz).  256 CUs x 32 lanes x 2.4 GHz, over 4 per modular product.
PEAK_MODMUL = 256 * 32 * 2.4e9 / 4.0    # 4.92e12 modular products/s


def ring_modmuls_per_gate(d, rows=124):
    """Modular products of one product gate on the transform route: the
    forward transforms of the rows*rows digit polynomials (their first stage
    multiplies 0/1 inputs, a select), the pointwise products against both
    columns, the inverse transforms and d^-1 scaling of the 2*rows outputs,
    and the forward transforms of the right operand's 2*rows polynomials."""
    logd = d.bit_length() - 1
    half = d // 2
    digit = rows * rows * half * max(logd - 1, 0)
    pointwise = rows * rows * 2 * d
    inverse = 2 * rows * (half * logd + d)
    right = 2 * rows * half * logd
    return digit + pointwise + inverse + right


def ring_modmuls_per_cmux(d, rows=124):
    """Modular products of one CMux step of blind rotation (one row of the
    product): the rows digit transforms, the pointwise products against both
    columns, and the inverse transforms and scaling of the two sums."""
    logd = d.bit_length() - 1
    half = d // 2
    return rows * half * max(logd - 1, 0) + rows * 2 * d + 2 * (half * logd + d)


def run_ring_br(args):
    """Blind rotation at d = 1024: one step is one sfft_ring_blind_rotate call
    that runs m accumulators through n CMux steps each (a 64-bit key), key
    prepared and accumulators resident in HBM."""
    import torch
    from paper_1611_08769_amd import sfft as S
    from paper_1611_08769_amd import workloads as WL

    d = int(args.workload.rsplit("_d", 1)[1])
    m, n = args.requests or 1024, 64
    stream = torch.cuda.current_stream().cuda_stream
    rows = 2 * S.SFFT_RING_ELL
    dk = WL.ring_draws(9, n, d, rows, S.SFFT_RING_P)
    dev = [torch.from_numpy(np.ascontiguousarray(x).view(np.int64) if x.dtype == np.uint64 else x).cuda()
           for x in (dk.s, dk.a, dk.e, dk.bits)]
    bk = torch.empty((n, S.sfft_ring_ct_words(d)), dtype=torch.int64, device="cuda")
    S.sfft_ring_encrypt(d, dev[0].data_ptr(), dev[1].data_ptr(), dev[2].data_ptr(), dev[3].data_ptr(), n,
                        bk.data_ptr(), stream)
    bkt = torch.empty_like(bk)
    S.sfft_ring_bk_prepare(d, bk.data_ptr(), n, bkt.data_ptr(), stream)
    g = np.random.Generator(np.random.PCG64(10))
    t = g.integers(0, 2, size=d).astype(np.uint64)
    acc0 = np.zeros((m, 2, d), np.uint64)
    acc0[:, 0, :] = t << np.uint64(61)          # trivial encryptions of 2^61 * t
    rot = g.integers(0, 2 * d, size=(m, n)).astype(np.int32)
    acc0_d = torch.from_numpy(acc0.view(np.int64)).cuda()
    acc = torch.empty_like(acc0_d)
    rot_d = torch.from_numpy(rot).cuda()
    torch.cuda.synchronize()

    def step():
        acc.copy_(acc0_d)
        S.sfft_ring_blind_rotate(d, bkt.data_ptr(), n, rot_d.data_ptr(), acc.data_ptr(), m, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        acc.copy_(acc0_d)
        a.record()
        S.sfft_ring_blind_rotate(d, bkt.data_ptr(), n, rot_d.data_ptr(), acc.data_ptr(), m, stream)
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_s = sum(a.elapsed_time(b) for a, b in ev) / len(ev) / 1e3
    # the first accumulators decrypt to the rotated pattern (host decryption of
    # coefficient by coefficient phases, library-side arithmetic only)
    out = acc.cpu().numpy().view(np.uint64)
    ok = True
    P = S.SFFT_RING_P
    for j in range(4):
        k = int(sum(int(rot[j, i]) * int(dk.bits[i]) for i in range(n))) % (2 * d)
        want = np.roll(t, k % d)
        b, a = out[j, 0].astype(object), out[j, 1].astype(object)
        a_s = np.zeros(d, dtype=object)       # a*s for the ternary secret: sum of s_v X^v a
        for v in np.nonzero(dk.s)[0]:
            a_s += int(dk.s[v]) * np.concatenate((-a[d - v:], a[:d - v]))
        ph = [int(x) % P for x in (b - a_s)]
        got = np.array([1 if min(x, P - x) > P // 4 else 0 for x in ph], np.uint64)
        ok = ok and got.tolist() == want.tolist()
    assert ok, "blind-rotated accumulators do not decrypt to the rotated pattern"
    # full gate bootstrapping of m LWE ciphertexts (n = 64, binary secret =
    # the key's bits) through sfft_ring_bootstrap, timed the same way
    mus = g.integers(0, 2, size=m)
    lwe = np.zeros((m, n + 1), np.uint64)
    lwe[:, :n] = g.integers(0, P, size=(m, n), dtype=np.uint64)
    for j in range(m):
        lwe[j, n] = (sum(int(x) for x, bit in zip(lwe[j, :n], dk.bits) if bit) + int(mus[j]) * (P // 2)) % P
    lwe_d = torch.from_numpy(lwe.view(np.int64)).cuda()
    bs_out = torch.empty((m, d + 1), dtype=torch.int64, device="cuda")
    ws_b = S.sfft_ring_bootstrap_workspace_bytes(d, n, m)
    ws = torch.empty(ws_b // 8 + 1, dtype=torch.int64, device="cuda")

    def bootstrap():
        S.sfft_ring_bootstrap(d, bkt.data_ptr(), n, lwe_d.data_ptr(), m, bs_out.data_ptr(), ws.data_ptr(), ws_b,
                              stream)

    bootstrap()
    torch.cuda.synchronize()
    ev2 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for a_, b_ in ev2:
        a_.record()
        bootstrap()
        b_.record()
    torch.cuda.synchronize()
    bs_s = sum(a_.elapsed_time(b_) for a_, b_ in ev2) / len(ev2) / 1e3
    o = bs_out.cpu().numpy().view(np.uint64)
    for j in range(4):   # phase b' - <a', s_ring> reads mu * 2 * floor(p/4)
        ph = (int(o[j, d]) - sum(int(o[j, t]) * int(dk.s[t]) for t in range(d) if dk.s[t])) % P
        got = 1 if min(ph, P - ph) > P // 4 else 0
        assert got == int(mus[j]), "bootstrapped ciphertext %d decrypts to the wrong bit" % j
    # key switching back to the 64-bit LWE secret closes the refresh loop; the
    # key-switching key encrypts s_ring[t] * 16^k under it (errors in [-2, 2])
    ksk = np.zeros((d, 16, n + 1), np.uint64)
    ksk[:, :, :n] = g.integers(0, P, size=(d, 16, n), dtype=np.uint64)
    ke = g.integers(-2, 3, size=(d, 16))
    on = np.nonzero(dk.bits)[0]
    for t_ in range(d):
        for k_ in range(16):
            dot = sum(int(ksk[t_, k_, i]) for i in on)
            ksk[t_, k_, n] = (dot + int(dk.s[t_]) * (16 ** k_) + int(ke[t_, k_])) % P
    ksk_d = torch.from_numpy(ksk.view(np.int64)).cuda()
    ks_out = torch.empty((m, n + 1), dtype=torch.int64, device="cuda")

    def keyswitch():
        S.sfft_ring_keyswitch(d, n, ksk_d.data_ptr(), bs_out.data_ptr(), m, ks_out.data_ptr(), stream)

    keyswitch()
    torch.cuda.synchronize()
    ev3 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for a_, b_ in ev3:
        a_.record()
        keyswitch()
        b_.record()
    torch.cuda.synchronize()
    ks_s = sum(a_.elapsed_time(b_) for a_, b_ in ev3) / len(ev3) / 1e3
    o = ks_out.cpu().numpy().view(np.uint64)
    for j in range(4):   # back under the LWE secret: phase reads mu * floor(p/2)
        ph = (int(o[j, n]) - sum(int(o[j, i]) for i in on)) % P
        assert (1 if min(ph, P - ph) > P // 4 else 0) == int(mus[j]), "refreshed ciphertext %d is wrong" % j
    mm = ring_modmuls_per_cmux(d) * m * n
    return {
        "metric": "CMux steps/s of ring-GSW blind rotation (1 GPU)",
        "value": m * n / launch_s,
        "unit": "CMux/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": args.workload, "d": d, "accumulators": m, "key_bits": n, "ell": S.SFFT_RING_ELL,
                   "p": "2^62-2^16+1"},
        "blind_rotations_per_s": m / launch_s,
        "bootstraps_per_s": m / bs_s,
        "bootstrap_ms_per_call": bs_s * 1e3,
        "keyswitch_ms_per_call": ks_s * 1e3,
        "refreshes_per_s": m / (bs_s + ks_s),
        "roofline": {"bound": "alu", "achieved": mm / launch_s / 1e9, "peak": PEAK_MODMUL / 1e9,
                     "unit": "Gmodmul/s", "frac": mm / launch_s / PEAK_MODMUL, "traffic": None,
                     "kernel": "k_ring_blind_rotate", "avg_launch_ms": launch_s * 1e3,
                     "modmul_per_cmux": ring_modmuls_per_cmux(d)},
    }


def run_ring_fft(args):
    """An encrypted FFT of a named workload on bootstrapped ring-LWE gates
    (sfft_ring_fft_execute): d = 1024, a 16-bit LWE key, every binary gate a
    refresh.  One step is one FFT, inputs encrypted and resident in HBM."""
    import torch
    from paper_1611_08769_amd import api
    from paper_1611_08769_amd import sfft as S
    from paper_1611_08769_amd import workloads as WL

    name = args.workload[len("ring_fft_"):]
    sig, _, seed = WL.workload(name)
    d, n = 1024, 16
    P = S.SFFT_RING_P
    q8 = P // 8
    stream = torch.cuda.current_stream().cuda_stream
    shp = S.shape(sig.dims, sig.length, sig.F, sig.f, sig.is_complex)
    info = S.sfft_ring_plan_analyze(shp, d, n)
    rows = 2 * S.SFFT_RING_ELL
    g = np.random.Generator(np.random.PCG64(seed))
    s_lwe = g.integers(0, 2, size=n)
    dk = WL.ring_draws(seed + 100, n, d, rows, P, bits=s_lwe.astype(np.uint8))
    dev = [torch.from_numpy(np.ascontiguousarray(x).view(np.int64) if x.dtype == np.uint64 else x).cuda()
           for x in (dk.s, dk.a, dk.e, dk.bits)]
    bk = torch.empty((n, S.sfft_ring_ct_words(d)), dtype=torch.int64, device="cuda")
    S.sfft_ring_encrypt(d, dev[0].data_ptr(), dev[1].data_ptr(), dev[2].data_ptr(), dev[3].data_ptr(), n,
                        bk.data_ptr(), stream)
    bkt = torch.empty_like(bk)
    S.sfft_ring_bk_prepare(d, bk.data_ptr(), n, bkt.data_ptr(), stream)
    # key-switching key: entry [t][k] encrypts s_ring[t] * 16^k under s_lwe
    ksk = np.zeros((d, 16, n + 1), np.uint64)
    ksk[:, :, :n] = g.integers(0, P, size=(d, 16, n), dtype=np.uint64)
    on = np.nonzero(s_lwe)[0]
    ke = g.integers(-2, 3, size=(d, 16))
    for t in range(d):
        for k in range(16):
            ksk[t, k, n] = (sum(int(ksk[t, k, i]) for i in on) + int(dk.s[t]) * 16 ** k + int(ke[t, k])) % P
    ksk_d = torch.from_numpy(ksk.view(np.int64)).cuda()
    # inputs: the signal's bits (the library's own quantisation and order),
    # encrypted as mu * 2 * floor(p/8) under s_lwe
    words = api.signal_words(sig)
    bits = [(int(w) >> i) & 1 for w in words for i in range(sig.F)]
    lwe = np.zeros((len(bits), n + 1), np.uint64)
    lwe[:, :n] = g.integers(0, P, size=(len(bits), n), dtype=np.uint64)
    for j, mu in enumerate(bits):
        lwe[j, n] = (sum(int(lwe[j, i]) for i in on) + mu * 2 * q8 + int(g.integers(-2, 3))) % P
    in_d = torch.from_numpy(lwe.view(np.int64)).cuda()
    out = torch.empty((info.n_outputs, n + 1), dtype=torch.int64, device="cuda")
    ws = torch.empty(info.ws_bytes // 8 + 1, dtype=torch.int64, device="cuda")
    plan = S.sfft_ring_plan_create(shp, d, n)
    try:
        def step():
            S.sfft_ring_fft_execute(plan, bkt.data_ptr(), ksk_d.data_ptr(), in_d.data_ptr(), out.data_ptr(),
                                    ws.data_ptr(), info.ws_bytes, stream)

        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        a_, b_ = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        a_.record()
        for _ in range(args.steps):
            step()
        b_.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per = a_.elapsed_time(b_) / 1e3 / args.steps
    finally:
        S.sfft_ring_plan_destroy(plan)
    return {
        "metric": "encrypted gates/s on bootstrapped ring-LWE gates (1 GPU)",
        "value": info.gates / per,
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": args.workload, "d": d, "lwe_key_bits": n, "ell": S.SFFT_RING_ELL,
                   "p": "2^62-2^16+1", "gates": info.gates, "levels": info.levels, "calls": info.calls,
                   "max_batch": info.max_batch},
        "s_per_fft": per,
        "fft_points_per_s": sig.points / per,
        # every binary gate is one refresh: n CMux steps of the blind
        # rotation, which dominate the FFT's device time (the key switch and
        # the modulus switch are below 3% of it); the whole FFT's device
        # time is the denominator
        "roofline": {"bound": "alu", "achieved": info.gates * n * ring_modmuls_per_cmux(d) / per / 1e9,
                     "peak": PEAK_MODMUL / 1e9, "unit": "Gmodmul/s",
                     "frac": info.gates * n * ring_modmuls_per_cmux(d) / per / PEAK_MODMUL, "traffic": None,
                     "kernel": "k_ring_blind_rotate", "over": "whole FFT (device time, HIP events)",
                     "modmul_per_gate": n * ring_modmuls_per_cmux(d)},
    }


def run_ring(args):
    """Ring-GSW AND gates at d = 1024: one step is one sfft_ring_gate call
    over n ciphertext pairs (the right operands' forward transforms and the
    product kernel), inputs encrypted and resident in HBM."""
    import torch
    from oracle import rgsw as O
    from paper_1611_08769_amd import sfft as S
    from paper_1611_08769_amd import workloads as WL

    d = int(args.workload.rsplit("_d", 1)[1])
    n = args.requests or 128
    stream = torch.cuda.current_stream().cuda_stream
    cts = []
    for seed in (1, 2):
        dr = WL.ring_draws(seed, n, d, 2 * S.SFFT_RING_ELL, S.SFFT_RING_P)
        if seed == 1:
            secret = dr.s
        dev = [torch.from_numpy(np.ascontiguousarray(x).view(np.int64) if x.dtype == np.uint64 else x).cuda()
               for x in (secret, dr.a, dr.e, dr.bits)]
        ct = torch.empty((n, S.sfft_ring_ct_words(d)), dtype=torch.int64, device="cuda")
        S.sfft_ring_encrypt(d, dev[0].data_ptr(), dev[1].data_ptr(), dev[2].data_ptr(), dev[3].data_ptr(), n,
                            ct.data_ptr(), stream)
        cts.append((ct, dr.bits))
        del dev
    (X, xb), (Y, yb) = cts
    out = torch.empty_like(X)
    ws_b = S.sfft_ring_workspace_bytes(d, n)
    ws = torch.empty(ws_b // 8, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()

    def step():
        S.sfft_ring_gate(d, 4, X.data_ptr(), Y.data_ptr(), out.data_ptr(), n, ws.data_ptr(), ws_b, stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        step()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = [a.elapsed_time(b) for a, b in ev]
    dec = np.zeros(n, np.uint8)
    s = np.ascontiguousarray(secret, dtype=np.int64)
    S.sfft_ring_decrypt(d, s.ctypes.data, out.data_ptr(), n, 1, dec.ctypes.data)
    assert dec.tolist() == (xb & yb).tolist(), "ring AND decryptions differ from the plaintext"
    avg_s = sum(launch_ms) / len(launch_ms) / 1e3
    mm = ring_modmuls_per_gate(d) * n
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic_k_ring_product_%s.json" % args.workload)
    if os.path.exists(tpath) and n == 128:
        import hashlib
        tr = json.load(open(tpath))
        src = os.path.join(ROOT, "paper_1611_08769_amd", "csrc", "ring.hip")
        if hashlib.sha256(open(src, "rb").read()).hexdigest() == tr.get("ring_hip_sha256"):
            traffic = tr["traffic_bytes_per_call"]
    res = {
        "metric": "encrypted ring-GSW gates/s (1 GPU)",
        "value": n * args.steps / wall,
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": args.workload, "d": d, "gates_per_step": n, "gate": "AND", "ell": S.SFFT_RING_ELL,
                   "p": "2^62-2^16+1", "ct_bytes": S.sfft_ring_ct_words(d) * 8},
        "roofline": {"bound": "alu", "achieved": mm / avg_s / 1e9, "peak": PEAK_MODMUL / 1e9,
                     "unit": "Gmodmul/s", "frac": mm / avg_s / PEAK_MODMUL, "traffic": traffic,
                     "algorithmic_bytes": 3 * n * S.sfft_ring_ct_words(d) * 8,
                     "kernel": "k_ring_fwd + k_ring_product", "avg_launch_ms": avg_s * 1e3,
                     "modmul_per_gate": ring_modmuls_per_gate(d)},
    }
    if not args.no_cpu_baseline:
        Xh = X.cpu().numpy().view(np.uint64).reshape(n, 2 * O.ELL, 2, d)
        Yh = Y.cpu().numpy().view(np.uint64).reshape(n, 2 * O.ELL, 2, d)
        threads = int(O.lib().rg_threads())
        t1 = time.perf_counter()
        O.gate_rows(4, Xh, Yh, [0], [5])
        one = time.perf_counter() - t1
        t1 = time.perf_counter()
        O.gate_rows(4, Xh, Yh, [q % n for q in range(threads)], [(7 * q) % (2 * O.ELL) for q in range(threads)])
        allc = time.perf_counter() - t1
        res["cpu_baseline"] = {
            "value": threads / allc / (2 * O.ELL), "unit": "gates/s", "cores": threads, "kind": "oracle",
            "sample": "%d output rows of AND at d=%d on %d threads, %.2f s (a gate has %d rows)" % (
                threads, d, threads, allc, 2 * O.ELL),
            "value_1_core": 1.0 / one / (2 * O.ELL),
            "sample_1_core": "1 output row on 1 thread, %.2f s" % one,
        }
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--requests", type=int, default=0, help="batch / serve mode: number of requests (64 / 40)")
    ap.add_argument("--max-active", type=int, default=0, help="batch mode: requests in flight (0 = no limit)")
    ap.add_argument("--budget-gb", type=float, default=0.0,
                    help="batch/serve: workspace memory budget (default 120 GB batch, 180 GB serve)")
    ap.add_argument("--max-len", type=int, default=128, help="batch mode: longest request length (8..128)")
    ap.add_argument("--rate", type=float, default=0.0, help="serve mode: arrivals per second (0 = from --load)")
    ap.add_argument("--load", type=float, default=0.7, help="serve mode: offered load as a fraction of capacity")
    ap.add_argument("--rate-bitmac", type=float, default=2.0e15, help="serve mode: capacity in bit-MAC/s")
    ap.add_argument("--io-gb", type=float, default=60.0, help="serve mode: ciphertexts of requests in flight")
    ap.add_argument("--plan-ws-gb", type=float, default=40.0,
                    help="serve mode: workspace bound of plans that would need more (list-scheduled levels)")
    ap.add_argument("--signals", type=int, default=4, help="accuracy mode: signals per length")
    ap.add_argument("--fill-blocks", type=int, default=-1,
                    help="batch/serve: request-loop fill target in workgroups, 0 = lockstep "
                         "(default: 0 batch, 2048 serve)")
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="fft1d_n64_cplx_q16.8")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mix", action="store_true",
                    help="default workload: skip the batched and served runs that follow the single request")
    ap.add_argument("--batch-requests", type=int, default=256, help="default workload: requests of the batched run")
    ap.add_argument("--batch-small-requests", type=int, default=128,
                    help="default workload: requests of the batched run of small requests (N = 8..32)")
    ap.add_argument("--serial-groups", action="store_true",
                    help="batch mode: a step's launches of different tilings in turn on one stream")
    ap.add_argument("--fixed-batch-gb", type=float, default=100.0,
                    help="batch mode: ciphertexts and workspaces of the fixed batch run through a HIP graph")
    ap.add_argument("--serve-requests", type=int, default=16, help="default workload: requests of the served run")
    ap.add_argument("--no-tune", action="store_true", help="use the default tiling instead of tuning it first")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--copy-probe", action="store_true", help="only copy 1 GiB three times (counter reference)")
    ap.add_argument("--traffic-summary", nargs=4, metavar=("FETCH_CSV", "WRITE_CSV", "COPY_FETCH_CSV", "COPY_WRITE_CSV"),
                    help="write profiles/traffic_k_product_<workload>.json from rocprofv3 counter CSVs")
    ap.add_argument("--counter-summary", metavar="COUNTER_CSV",
                    help="per-launch averages of a rocprofv3 --pmc CSV over the product launches of one FFT")
    ap.add_argument("--trace-summary", metavar="RESULTS_DB",
                    help="summarise a rocprofv3 kernel trace of a bench run (its --steps timed FFTs)")
    args = ap.parse_args()
    if args.traffic_summary:
        if args.workload.startswith("ring_and_d"):
            ring_traffic_summary(args.workload, *args.traffic_summary)
        else:
            traffic_summary(args.workload, *args.traffic_summary)
        return
    if args.trace_summary:
        trace_summary(args.workload, args.trace_summary, args.steps)
        return
    if args.counter_summary:
        counter_summary(args.workload, args.counter_summary)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(requests and levels would shard across GPUs as described in the design notes)", file=sys.stderr)
        sys.exit(2)

    if args.copy_probe:
        copy_probe()
        return
    import torch
    from paper_1611_08769_amd import api
    from paper_1611_08769_amd import sfft as S
    from paper_1611_08769_amd import workloads as WL

    if args.workload == "batch":
        print(json.dumps(run_batch(args)), flush=True)
        return
    if args.workload == "accuracy":
        print(json.dumps(run_accuracy(args)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(run_serve(args)), flush=True)
        return
    if args.workload.startswith("ring_and_d"):
        print(json.dumps(run_ring(args)), flush=True)
        return
    if args.workload.startswith("ring_fft_"):
        print(json.dumps(run_ring_fft(args)), flush=True)
        return
    if args.workload.startswith("ring_br_d"):
        print(json.dumps(run_ring_br(args)), flush=True)
        return
    sig, n_lwe, seed = WL.workload(args.workload)
    cplx = sig.is_complex
    params = api.size_params(sig.dims, sig.length, sig.F, sig.f, cplx, n_lwe)
    tuned = None
    keys = api.keygen(params, seed)
    words = api.signal_words(sig)
    ct_in = api.encrypt_words(keys, words, sig.F, seed=seed)
    plan = api.Plan(sig.dims, sig.length, sig.F, sig.f, cplx, params)
    ct_out = torch.empty((plan.info.n_outputs, plan.ct_words), dtype=torch.int32, device="cuda")
    if not args.no_tune:
        # tiling chosen on the plan's own widest level, before the clock starts
        best, rates = plan.tune(ct_in, ct_out)
        tuned = {"tiling": best, "candidates": {str(k): round(v / 1e12, 1) for k, v in rates.items()}}
        print("[bench] tuner: tiling %d; Tbit-MAC/s per candidate %s" % (best, tuned["candidates"]),
              file=sys.stderr, flush=True)
    info = plan.info
    nct = (params.n_lwe + 1) * params.k
    print("[bench] workload=%s k=%d Nct=%d products=%d exec=%d levels=%d ws=%.1f GB" % (
        args.workload, params.k, nct, info.products, info.exec_products, info.levels, plan.ws_bytes / 1e9),
        file=sys.stderr, flush=True)

    for w in range(args.warmup):
        plan.execute(ct_in, ct_out)
        torch.cuda.synchronize()
        print("[bench] warmup %d done" % w, file=sys.stderr, flush=True)

    # HIP events around each level's product kernel alone, recorded by the
    # library on the stream the kernel runs on
    plan.time_products(True)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        ts = time.perf_counter()
        plan.execute(ct_in, ct_out)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
        print("[bench] step %d: %.3f s" % (s, lat[-1]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    plan.time_products(False)
    kern_ms, n_launch = plan.product_time()

    step_s = total / args.steps
    bitmac_step = float(info.exec_products) * nct ** 3
    achieved = bitmac_step * args.steps / (kern_ms / 1e3)
    npts = sig.points
    mfma = S.sfft_tiling_describe(info.tiling)[6] == 1
    if mfma:
        ops = achieved / 4.0  # int8 op/s of the algorithmic Nct^3 / 4 per product
        roofline = {"bound": "mfma", "achieved": ops / 1e12, "peak": PEAK_MFMA_I8 / 1e12, "unit": "TOP/s",
                    "frac": ops / PEAK_MFMA_I8, "dtype": "i8"}
    else:
        roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LOOKUP / 1e12, "unit": "Tbitmac/s",
                    "frac": achieved / PEAK_LOOKUP}
    desc = S.sfft_tiling_describe(info.tiling)
    roofline.update({
        "traffic": None,
        "kernel": ("k_product_mfma2" if desc[4] == 2 else "k_product_mfma") if mfma else "k_product",
        "launches": n_launch,
        "avg_launch_ms": kern_ms / max(1, n_launch),
        "bitmac_per_s": achieved,
        "frac_vs_popcount_ceiling": achieved / PEAK_POPCOUNT,
        "frac_vs_valu_lookup_ceiling": achieved / PEAK_LOOKUP,
    })
    out = {
        "metric": "encrypted gates/s (1 GPU)",
        "value": info.gates / step_s,
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # products: bits of L times bytes of R in int8 (matrix cores) or
        # 30-bit digits in u32 (lookup kernel); limb arithmetic in u32
        "dtype": "i8" if mfma else "u32",
        "data": "synthetic",
        "config": {
            "workload": args.workload,
            "dims": sig.dims, "len": sig.length, "F": sig.F, "f": sig.f, "complex": cplx,
            "n_lwe": params.n_lwe, "k": params.k, "nct": nct,
            "canonical_gates": int(info.gates), "canonical_products": int(info.products),
            "exec_products": int(info.exec_products), "levels": int(info.levels),
            "tiling": list(S.sfft_tiling_describe(info.tiling)),
        },
        "tuner": tuned,
        "fft_points_per_s": npts / step_s,
        "products_per_s": info.exec_products / step_s,
        "latency_p50_s": pct(lat, 50),
        "latency_p99_s": pct(lat, 99),
        "roofline": roofline,
        "cpu_baseline": None,
    }
    # HBM bytes per launch from rocprofv3 FETCH_SIZE / WRITE_SIZE runs of this
    # command, valid only for the kernel source they were taken with
    tpath = os.path.join(ROOT, "profiles", "traffic_k_product_%s.json" % args.workload)
    if os.path.exists(tpath):
        tr = json.load(open(tpath))
        if _kernel_source_sha() == tr.get("kernel_source_sha256"):
            out["roofline"]["traffic"] = tr["traffic_bytes_per_launch"]
            # algorithmic bytes: each ciphertext a product item reads (L, R and
            # extra operands) or writes, once
            alg = (info.prod_ct_reads + info.prod_ct_writes) * nct * nct / 8 / max(1, info.levels)
            out["roofline"]["algorithmic_bytes_per_launch"] = alg
            out["roofline"]["traffic_vs_algorithmic_bytes"] = tr["traffic_bytes_per_launch"] / alg
    out["parity"], out["noise"] = output_checks(args.workload, keys, ct_out, sig, info, params)
    out["small_plan"] = small_plan_latency(plan, ct_in, ct_out, args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload, nct, params.n_lwe + 1, params.k // 32, info.gates,
                                           info.products, args.cpu_budget)
    plan.close()
    del ct_in, ct_out
    torch.cuda.empty_cache()
    if not args.no_mix:
        # the batched mix (all requests through the request loop vs one at a
        # time) and the served mix (Poisson arrivals), each output decrypted
        # against the expected decryptions
        bt = run_batch(args, count=args.batch_requests)
        out["batch"] = {k: bt[k] for k in (
            "value", "unit", "ms_per_step", "one_at_a_time_gates_per_s", "one_at_a_time_s",
            "speedup_vs_one_at_a_time", "fft_points_per_s", "bitmac_per_s", "roofline", "latency_p50_s",
            "latency_p99_s", "max_in_flight", "outputs_identical_to_alone", "all_decrypt_equal", "decrypt_checked",
            "fixed_batch_graph")}
        out["batch"]["config"] = bt["config"]
        torch.cuda.empty_cache()
        # the same comparison on small requests (N = 8..32), whose levels
        # leave most of the GPU idle when run alone
        bs_args = argparse.Namespace(**vars(args))
        bs_args.max_len, bs_args.fixed_batch_gb = 32, 0.0
        bs = run_batch(bs_args, count=args.batch_small_requests)
        out["batch_small"] = {k: bs[k] for k in (
            "value", "unit", "ms_per_step", "one_at_a_time_gates_per_s", "one_at_a_time_s",
            "speedup_vs_one_at_a_time", "latency_p50_s", "latency_p99_s", "max_in_flight",
            "outputs_identical_to_alone", "all_decrypt_equal", "decrypt_checked")}
        out["batch_small"]["config"] = bs["config"]
        torch.cuda.empty_cache()
        sv = run_serve(args, count=args.serve_requests)
        out["serve"] = {k: sv[k] for k in (
            "value", "unit", "ms_per_step", "fft_points_per_s", "bitmac_per_s", "latency_p50_s", "latency_p99_s",
            "latency_mean_s", "max_in_flight", "all_decrypt_equal", "decrypt_checked", "noise_within_bound",
            "requests_detail")}
        out["serve"]["config"] = sv["config"]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
