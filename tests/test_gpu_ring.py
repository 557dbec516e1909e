"""GPU: ring-GSW encryption and gates through the C ABI, bit for bit against
the CPU oracle (negacyclic products by their definition), on the same seeded
draws; decryptions against the plaintext circuit."""
import sys

import numpy as np
import pytest
import torch

from oracle import rgsw as O
from paper_1611_08769_amd import sfft as S
from paper_1611_08769_amd import workloads as WL

pytestmark = pytest.mark.gpu

PRODUCT_GATES = (4, 5, 6, 8, 9)
ALL_GATES = (3, 4, 5, 6, 7, 8, 9)


def say(msg):
    print("[gpu-case]", msg, flush=True)
    sys.stdout.flush()


def _stream():
    return torch.cuda.current_stream().cuda_stream


def _dev(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    return torch.from_numpy(a).cuda()


def _host(t):
    return t.cpu().numpy().view(np.uint64)


def _encrypt(dr, d):
    n = dr.a.shape[0]
    out = torch.empty((n, O.ROWS, 2, d), dtype=torch.int64, device="cuda")
    s, a, e, b = _dev(dr.s), _dev(dr.a), _dev(dr.e), _dev(dr.bits)
    S.sfft_ring_encrypt(d, s.data_ptr(), a.data_ptr(), e.data_ptr(), b.data_ptr(), n, out.data_ptr(), _stream())
    torch.cuda.synchronize()
    return out


def _gate(op, X, Y, d):
    n = X.shape[0]
    out = torch.empty_like(X)
    ws_b = S.sfft_ring_workspace_bytes(d, n)
    ws = torch.empty(max(ws_b // 8, 1), dtype=torch.int64, device="cuda")
    S.sfft_ring_gate(d, op, X.data_ptr(), Y.data_ptr(), out.data_ptr(), n, ws.data_ptr(), ws_b, _stream())
    torch.cuda.synchronize()
    return out


def _pair(seed, n, d):
    x = WL.ring_draws(seed, n, d, O.ROWS, O.P)
    y = WL.ring_draws(seed + 1000, n, d, O.ROWS, O.P)
    y.s = x.s
    return x, y


@pytest.mark.parametrize("d,n", [(1, 3), (2, 1), (16, 3), (64, 2), (1024, 1)])
def test_encrypt_matches_oracle(d, n):
    say("ring encrypt d=%d n=%d" % (d, n))
    dr = WL.ring_draws(40 + d, n, d, O.ROWS, O.P)
    got = _host(_encrypt(dr, d))
    assert np.array_equal(got, O.encrypt(dr))


@pytest.mark.parametrize("d,n", [(1, 3), (4, 2), (16, 9), (64, 2)])
def test_gates_match_oracle(d, n):
    """Every gate, bit for bit.  n = 9 at d = 16 leaves a tail of workgroups
    outside the XCD-grouped order."""
    x, y = _pair(50 + d, n, d)
    X, Y = _encrypt(x, d), _encrypt(y, d)
    Lh, Rh = _host(X), _host(Y)
    for op in ALL_GATES:
        say("ring gate %d d=%d n=%d" % (op, d, n))
        got = _host(_gate(op, X, Y, d))
        assert np.array_equal(got, O.gate(op, Lh, Rh)), op


def test_gate_d256_matches_oracle():
    d, n = 256, 1
    say("ring AND d=%d n=%d" % (d, n))
    x, y = _pair(77, n, d)
    X, Y = _encrypt(x, d), _encrypt(y, d)
    got = _host(_gate(4, X, Y, d))
    assert np.array_equal(got, O.gate(4, _host(X), _host(Y)))


@pytest.mark.parametrize("d,n", [(1024, 16), (2048, 3)])
def test_bench_sizes_sampled_rows(d, n):
    """At the benchmark's d (and the largest d), sampled output rows against
    the oracle computed row by row: first, last, the decrypting row, both
    column blocks, in several ciphertexts."""
    say("ring AND/XOR sampled d=%d n=%d" % (d, n))
    x, y = _pair(90 + d, n, d)
    X, Y = _encrypt(x, d), _encrypt(y, d)
    Lh, Rh = _host(X), _host(Y)
    cts = [0, n - 1, n // 2, 1 % n]
    rows = [0, O.ROWS - 1, O.ELL - 1, O.ELL]
    for op in (4, 5):
        got = _host(_gate(op, X, Y, d))
        want = O.gate_rows(op, Lh, Rh, cts, rows)
        for q, (c, r) in enumerate(zip(cts, rows)):
            assert np.array_equal(got[c, r], want[q]), (op, c, r)


def test_circuit_decrypts_and_matches_oracle_decryption():
    """((a AND b) XOR c) OR (NOT e) at d = 1024 on 8 random inputs: the GPU
    decryption equals the plaintext circuit and the oracle's decryption of
    the same ciphertexts."""
    d, n = 1024, 8
    say("ring depth-3 circuit d=%d n=%d" % (d, n))
    ds = [WL.ring_draws(300 + i, n, d, O.ROWS, O.P) for i in range(4)]
    for t in ds[1:]:
        t.s = ds[0].s
    a, b, c, e = (_encrypt(t, d) for t in ds)
    t1 = _gate(4, a, b, d)
    t2 = _gate(5, t1, c, d)
    t3 = _gate(6, t2, _gate(3, e, e, d), d)
    bits = [t.bits.astype(int) for t in ds]
    want = ((bits[0] & bits[1]) ^ bits[2]) | (1 - bits[3])
    s = np.ascontiguousarray(ds[0].s, dtype=np.int64)
    got = np.zeros(n, np.uint8)
    S.sfft_ring_decrypt(d, s.ctypes.data, t3.data_ptr(), n, 1, got.ctypes.data)
    assert got.tolist() == want.tolist()
    assert O.decrypt(_host(t3), ds[0].s).tolist() == want.tolist()


def test_empty_and_errors():
    say("ring edge cases")
    d = 16
    x, y = _pair(5, 1, d)
    X, Y = _encrypt(x, d), _encrypt(y, d)
    out = torch.zeros_like(X)
    ws_b = S.sfft_ring_workspace_bytes(d, 1)
    ws = torch.empty(ws_b // 8, dtype=torch.int64, device="cuda")
    # n = 0: nothing written
    S.sfft_ring_gate(d, 4, X.data_ptr(), Y.data_ptr(), out.data_ptr(), 0, ws.data_ptr(), ws_b, _stream())
    torch.cuda.synchronize()
    assert not out.any()
    for bad in (dict(d=3), dict(d=4096), dict(gate=10), dict(ws_bytes=ws_b - 8), dict(alias=True)):
        args = dict(d=d, gate=4, ws_bytes=ws_b, alias=False)
        args.update(bad)
        o = X if args["alias"] else out
        with pytest.raises(S.SfftError) as e:
            S.sfft_ring_gate(args["d"], args["gate"], X.data_ptr(), Y.data_ptr(), o.data_ptr(), 1, ws.data_ptr(),
                             args["ws_bytes"], _stream())
        assert e.value.code == S.SFFT_EINVAL
    torch.cuda.synchronize()
    assert not out.any()


def _prepared_key(dk, d):
    """Ring-GSW key on the device, and its transformed rows."""
    bk = _encrypt(dk, d)
    n = bk.shape[0]
    bkt = torch.empty_like(bk)
    S.sfft_ring_bk_prepare(d, bk.data_ptr(), n, bkt.data_ptr(), _stream())
    return bk, bkt


@pytest.mark.parametrize("d,n,m", [(1, 3, 2), (16, 5, 3), (64, 3, 9), (1024, 2, 2)])
def test_blind_rotate_matches_oracle(d, n, m):
    """Blind rotation of m random accumulators by an n-bit key, bit for bit;
    rotations include values outside [0, 2d) (taken mod 2d) at small d."""
    say("ring blind rotation d=%d n=%d m=%d" % (d, n, m))
    dk = WL.ring_draws(500 + d, n, d, O.ROWS, O.P)
    bk, bkt = _prepared_key(dk, d)
    g = np.random.Generator(np.random.PCG64(d + n))
    lo, hi = (-3 * d, 5 * d) if d <= 64 else (0, 2 * d)
    rot = g.integers(lo, hi, size=(m, n)).astype(np.int32)
    acc = g.integers(0, O.P, size=(m, 2, d), dtype=np.uint64)
    acc_d = _dev(acc)
    rot_d = _dev(rot)
    S.sfft_ring_blind_rotate(d, bkt.data_ptr(), n, rot_d.data_ptr(), acc_d.data_ptr(), m, _stream())
    torch.cuda.synchronize()
    want = O.blind_rotate(_host(bk), np.mod(rot, 2 * d), acc)
    assert np.array_equal(_host(acc_d), want)


def test_blind_rotate_decrypts_to_rotated_test_polynomial():
    """d = 1024, a 16-bit key, 8 accumulators (TV, 0) with TV = 2^61 * t: the
    decrypted pattern is t rotated by sum r_i s_i (negacyclic)."""
    d, n, m = 1024, 16, 8
    say("ring blind rotation decrypt d=%d n=%d m=%d" % (d, n, m))
    dk = WL.ring_draws(700, n, d, O.ROWS, O.P)
    _, bkt = _prepared_key(dk, d)
    g = np.random.Generator(np.random.PCG64(701))
    t = g.integers(0, 2, size=d).astype(np.uint64)
    acc = np.zeros((m, 2, d), np.uint64)
    acc[:, 0, :] = t << np.uint64(61)
    rot = g.integers(0, 2 * d, size=(m, n)).astype(np.int32)
    acc_d, rot_d = _dev(acc), _dev(rot)
    S.sfft_ring_blind_rotate(d, bkt.data_ptr(), n, rot_d.data_ptr(), acc_d.data_ptr(), m, _stream())
    torch.cuda.synchronize()
    out = _host(acc_d)
    for j in range(m):
        k = int(sum(int(rot[j, i]) * int(dk.bits[i]) for i in range(n))) % (2 * d)
        want = np.roll(t, k % d)                  # X^k moves coefficient u to u + k (sign irrelevant)
        ph = O.rlwe_phase(out[j], dk.s)
        got = np.array([1 if min(int(v), O.P - int(v)) > O.P // 4 else 0 for v in ph])
        assert got.tolist() == want.tolist(), j


def test_blind_rotate_edge_cases():
    say("ring blind rotation edge cases")
    d = 16
    dk = WL.ring_draws(5, 2, d, O.ROWS, O.P)
    bk, bkt = _prepared_key(dk, d)
    acc = torch.zeros((1, 2, d), dtype=torch.int64, device="cuda")
    rot = torch.zeros((1, 2), dtype=torch.int32, device="cuda")
    # n = 0 and m = 0 leave the accumulator alone
    acc.fill_(7)
    S.sfft_ring_blind_rotate(d, bkt.data_ptr(), 0, rot.data_ptr(), acc.data_ptr(), 1, _stream())
    S.sfft_ring_blind_rotate(d, bkt.data_ptr(), 2, rot.data_ptr(), acc.data_ptr(), 0, _stream())
    torch.cuda.synchronize()
    assert bool((acc == 7).all())
    for args in ((3, bkt.data_ptr(), 2, rot.data_ptr(), acc.data_ptr(), 1), (d, 0, 2, rot.data_ptr(), acc.data_ptr(), 1),
                 (d, bkt.data_ptr(), -1, rot.data_ptr(), acc.data_ptr(), 1)):
        with pytest.raises(S.SfftError) as e:
            S.sfft_ring_blind_rotate(*args, _stream())
        assert e.value.code == S.SFFT_EINVAL
    with pytest.raises(S.SfftError):
        S.sfft_ring_bk_prepare(d, bk.data_ptr(), 2, bk.data_ptr(), _stream())


def _lwe_inputs(seed, m, n, mus, B=3):
    """LWE ciphertexts mod p of bits mus under a binary secret (test-side
    encryption with Python integers): b = <a, s> + mu*floor(p/2) + e."""
    g = np.random.Generator(np.random.PCG64(seed))
    s = g.integers(0, 2, size=n)
    lwe = np.zeros((m, n + 1), np.uint64)
    for j in range(m):
        a = g.integers(0, O.P, size=n, dtype=np.uint64)
        e = int(g.integers(-B, B + 1))
        lwe[j, :n] = a
        lwe[j, n] = (sum(int(x) * int(y) for x, y in zip(a, s)) + int(mus[j]) * (O.P // 2) + e) % O.P
    return s, lwe


def _bootstrap(dk, lwe, d):
    n = lwe.shape[1] - 1
    m = lwe.shape[0]
    _, bkt = _prepared_key(dk, d)
    lwe_d = _dev(lwe)
    out = torch.zeros((m, d + 1), dtype=torch.int64, device="cuda")
    ws_b = S.sfft_ring_bootstrap_workspace_bytes(d, n, m)
    ws = torch.empty(ws_b // 8 + 1, dtype=torch.int64, device="cuda")
    S.sfft_ring_bootstrap(d, bkt.data_ptr(), n, lwe_d.data_ptr(), m, out.data_ptr(), ws.data_ptr(), ws_b, _stream())
    torch.cuda.synchronize()
    return _host(out)


@pytest.mark.parametrize("d,n,m", [(16, 4, 5), (64, 6, 3), (1024, 3, 2)])
def test_bootstrap_matches_oracle(d, n, m):
    say("ring bootstrap d=%d n=%d m=%d" % (d, n, m))
    g = np.random.Generator(np.random.PCG64(900 + d))
    mus = g.integers(0, 2, size=m)
    s_lwe, lwe = _lwe_inputs(901 + d, m, n, mus)
    dk = WL.ring_draws(902 + d, n, d, O.ROWS, O.P, bits=s_lwe.astype(np.uint8))
    got = _bootstrap(dk, lwe, d)
    want = O.bootstrap(O.encrypt(dk), lwe)
    assert np.array_equal(got, want)


def test_bootstrap_refreshes_noisy_bits():
    """d = 1024, a 32-bit LWE key, 16 inputs with errors up to p/16: every
    output decrypts (under the ring secret) to its input bit, with a phase
    within the blind rotation's bound of mu * 2 * floor(p/4)."""
    d, n, m = 1024, 32, 16
    say("ring bootstrap refresh d=%d n=%d m=%d" % (d, n, m))
    g = np.random.Generator(np.random.PCG64(950))
    mus = g.integers(0, 2, size=m)
    s_lwe, lwe = _lwe_inputs(951, m, n, mus, B=O.P // 16)
    dk = WL.ring_draws(952, n, d, O.ROWS, O.P, bits=s_lwe.astype(np.uint8))
    out = _bootstrap(dk, lwe, d)
    bound = n * 2 * O.ELL * d * 2
    for j in range(m):
        ph = O.lwe_phase(out[j], dk.s)
        err = ((ph - int(mus[j]) * 2 * (O.P // 4) + O.P // 2) % O.P) - O.P // 2
        assert abs(err) <= bound, (j, err)


def _ksk(seed, s_ring, s_lwe, B):
    """Key-switching key (test-side encryption with Python integers): entry
    [t][k] encrypts s_ring[t] * 16^k under s_lwe, errors in [-B, B]."""
    g = np.random.Generator(np.random.PCG64(seed))
    d, n = len(s_ring), len(s_lwe)
    ksk = np.zeros((d, 16, n + 1), np.uint64)
    ksk[:, :, :n] = g.integers(0, O.P, size=(d, 16, n), dtype=np.uint64)
    e = g.integers(-B, B + 1, size=(d, 16))
    on = [i for i in range(n) if s_lwe[i]]
    for t in range(d):
        for k in range(16):
            dot = sum(int(ksk[t, k, i]) for i in on)
            ksk[t, k, n] = (dot + int(s_ring[t]) * (16 ** k) + int(e[t, k])) % O.P
    return ksk


def _keyswitch(ksk, lwe, d):
    n = ksk.shape[2] - 1
    m = lwe.shape[0]
    k_d, in_d = _dev(ksk), _dev(lwe)
    out = torch.zeros((m, n + 1), dtype=torch.int64, device="cuda")
    S.sfft_ring_keyswitch(d, n, k_d.data_ptr(), in_d.data_ptr(), m, out.data_ptr(), _stream())
    torch.cuda.synchronize()
    return _host(out)


@pytest.mark.parametrize("d,n,m", [(16, 5, 4), (1024, 32, 3)])
def test_keyswitch_matches_oracle(d, n, m):
    say("ring key switch d=%d n=%d m=%d" % (d, n, m))
    g = np.random.Generator(np.random.PCG64(980 + d))
    s_ring = g.integers(-1, 2, size=d)
    s_lwe = g.integers(0, 2, size=n)
    ksk = _ksk(981 + d, s_ring, s_lwe, 2)
    lwe = g.integers(0, O.P, size=(m, d + 1), dtype=np.uint64)
    assert np.array_equal(_keyswitch(ksk, lwe, d), O.keyswitch(ksk, lwe))


def test_refresh_round_trip_d1024():
    """LWE ciphertexts under a 32-bit binary secret with errors up to p/16,
    bootstrapped and key-switched back twice: every round decrypts under the
    same secret to the input bits with an error inside the two steps' bound."""
    d, n, m = 1024, 32, 8
    say("ring refresh round trip d=%d n=%d m=%d" % (d, n, m))
    g = np.random.Generator(np.random.PCG64(990))
    mus = g.integers(0, 2, size=m)
    s_lwe, lwe = _lwe_inputs(991, m, n, mus, B=O.P // 16)
    dk = WL.ring_draws(992, n, d, O.ROWS, O.P, bits=s_lwe.astype(np.uint8))
    ksk = _ksk(993, dk.s, s_lwe, 2)
    bound = n * 2 * O.ELL * d * 2 + d * 16 * 15 * 2
    cur = lwe
    for _ in range(2):
        cur = _keyswitch(ksk, _bootstrap(dk, cur, d), d)
        for j in range(m):
            err = ((O.lwe_phase(cur[j], s_lwe) - int(mus[j]) * (O.P // 2) + O.P // 2) % O.P) - O.P // 2
            assert abs(err) <= bound, (j, err)


def _lwe_bits(seed, s, mus, B):
    """LWE ciphertexts of bits mus encoded as mu * 2 * floor(p/8) under s."""
    g = np.random.Generator(np.random.PCG64(seed))
    n = len(s)
    out = np.zeros((len(mus), n + 1), np.uint64)
    out[:, :n] = g.integers(0, O.P, size=(len(mus), n), dtype=np.uint64)
    on = [i for i in range(n) if s[i]]
    for j, mu in enumerate(mus):
        e = int(g.integers(-B, B + 1))
        out[j, n] = (sum(int(out[j, i]) for i in on) + int(mu) * 2 * (O.P // 8) + e) % O.P
    return out


def _decode_q4(c, s):
    ph = O.lwe_phase(c, s)
    return 1 if abs(((ph - 2 * (O.P // 8) + O.P // 2) % O.P) - O.P // 2) < O.P // 8 else 0


class _GateKeys:
    def __init__(self, d, n, seed):
        g = np.random.Generator(np.random.PCG64(seed))
        self.d, self.n = d, n
        self.s = g.integers(0, 2, size=n)
        dk = WL.ring_draws(seed + 1, n, d, O.ROWS, O.P, bits=self.s.astype(np.uint8))
        self.bk, self.bkt = _prepared_key(dk, d)
        self.ksk = _ksk(seed + 2, dk.s, self.s, 2)
        self.ksk_d = _dev(self.ksk)

    def gate(self, g, x, y):
        m = x.shape[0]
        xd, yd = _dev(x), _dev(y)
        out = torch.zeros((m, self.n + 1), dtype=torch.int64, device="cuda")
        ws_b = S.sfft_ring_gate_bootstrap_workspace_bytes(self.d, self.n, m)
        ws = torch.empty(ws_b // 8 + 1, dtype=torch.int64, device="cuda")
        S.sfft_ring_gate_bootstrap(self.d, g, self.bkt.data_ptr(), self.n, self.ksk_d.data_ptr(), xd.data_ptr(),
                                   yd.data_ptr(), m, out.data_ptr(), ws.data_ptr(), ws_b, _stream())
        torch.cuda.synchronize()
        return _host(out)


@pytest.mark.parametrize("d,n", [(16, 5), (1024, 4)])
def test_bootstrapped_gates_match_oracle(d, n):
    """AND, XOR, OR, NAND on all four input pairs (errors up to p/64), bit for
    bit against the oracle, and decoding to the truth tables."""
    say("ring bootstrapped gates d=%d n=%d" % (d, n))
    K = _GateKeys(d, n, 1200 + d)
    xs, ys = [0, 0, 1, 1], [0, 1, 0, 1]
    x = _lwe_bits(1210 + d, K.s, xs, O.P // 64)
    y = _lwe_bits(1220 + d, K.s, ys, O.P // 64)
    for g, fn in ((4, lambda a, b: a & b), (5, lambda a, b: a ^ b), (6, lambda a, b: a | b),
                  (8, lambda a, b: 1 - (a & b))):
        got = K.gate(g, x, y)
        assert np.array_equal(got, O.gate_bootstrap(g, _host(K.bk), K.ksk, x, y)), g
        assert [_decode_q4(got[j], K.s) for j in range(4)] == [fn(a, b) for a, b in zip(xs, ys)], g


def test_bootstrapped_ripple_adder_d1024():
    """An 8-bit ripple-carry adder of bootstrapped gates at d = 1024 (depth 17
    gates on the carry chain, far beyond what an unrefreshed ring product
    survives), on 16 random operand pairs at once: every sum bit decodes."""
    d, n, m, w = 1024, 16, 16, 8
    say("ring bootstrapped ripple adder d=%d n=%d m=%d" % (d, n, m))
    K = _GateKeys(d, n, 1300)
    g = np.random.Generator(np.random.PCG64(1301))
    a = g.integers(0, 1 << w, size=m)
    b = g.integers(0, 1 << w, size=m)
    A = [_lwe_bits(1310 + i, K.s, (a >> i) & 1, 2) for i in range(w)]
    Bv = [_lwe_bits(1330 + i, K.s, (b >> i) & 1, 2) for i in range(w)]
    carry = None
    bits = []
    for i in range(w):
        if carry is None:
            bits.append(K.gate(5, A[i], Bv[i]))
            carry = K.gate(4, A[i], Bv[i])
        else:
            t = K.gate(5, A[i], Bv[i])
            bits.append(K.gate(5, t, carry))
            carry = K.gate(6, K.gate(4, A[i], Bv[i]), K.gate(4, t, carry))
    bits.append(carry)
    for j in range(m):
        got = sum(_decode_q4(bits[i][j], K.s) << i for i in range(w + 1))
        assert got == int(a[j] + b[j]), j


def test_fft_circuit_on_bootstrapped_gates_d1024():
    """An encrypted FFT with no depth limit: the N=4 complex Q(8,4) circuit
    evaluated gate by gate on the library's bootstrapped gates at d = 1024
    (one batched call per level and gate kind); the decrypted outputs equal
    the Boolean simulation and the fixed-point emulation."""
    from oracle import fixedpoint as fx
    from oracle import netlist as N
    from tests import ring_fft_driver as RF
    d, n = 1024, 16
    say("ring bootstrapped FFT N=4 d=%d n=%d" % (d, n))
    K = _GateKeys(d, n, 1400)
    cn = N.Compact(N.build_fft_netlist(1, 4, 8, 4, True))
    sig = WL.uniform_pm1(1401, 4, 8, 4, True)
    re, im = fx.quantize(np.asarray(sig.re), 8, 4), fx.quantize(np.asarray(sig.im), 8, 4)
    words = np.stack([re, im], 1).ravel()
    bits = fx.words_to_bits(words, 8)
    cts = _lwe_bits(1402, K.s, bits, 2)
    import time
    t0 = time.perf_counter()
    out, levels, calls = RF.evaluate(cn, cts, n, K.gate)
    t_eval = time.perf_counter() - t0
    got = [_decode_q4(c, K.s) for c in out]
    assert got == N.simulate(cn, [int(b) for b in bits], 1)
    er, ei = fx.fft1d_fixed(re[None], im[None], 8, 4)
    want = np.stack([er[0], ei[0]], 1).ravel()
    vals = []
    for v in range(len(want)):
        u = sum(got[v * 8 + i] << i for i in range(8))
        vals.append(u - 256 if u & 128 else u)
    assert vals == want.tolist()
    print("[gpu-case] %d levels, %d gate calls, %d gates, %.3f s (host copies included)" % (
        levels, calls, sum(1 for t in cn.t if t in N.BINARY), t_eval), flush=True)


@pytest.mark.parametrize("dims,L,F,f,cplx", [(1, 4, 8, 4, True), (1, 8, 8, 4, False), (1, 64, 16, 8, True)])
def test_ring_fft_plan_matches_emulation(dims, L, F, f, cplx):
    """The native executor of FFT plans on bootstrapped gates
    (sfft_ring_fft_execute) at d = 1024 with a 16-bit LWE key: decrypted
    outputs equal the integer fixed-point emulation -- up to the N=64 complex
    Q(16,8) circuit (289k bootstrapped gates, 157 levels)."""
    from oracle import fixedpoint as fx
    d, n = 1024, 16
    say("ring FFT plan N=%d F=%d cplx=%d d=%d n=%d" % (L, F, cplx, d, n))
    K = _GateKeys(d, n, 1500 + L)
    shp = S.shape(dims, L, F, f, cplx)
    info = S.sfft_ring_plan_analyze(shp, d, n)
    plan = S.sfft_ring_plan_create(shp, d, n)
    try:
        sig = WL.uniform_pm1(1501 + L, L, F, f, cplx)
        re = fx.quantize(np.asarray(sig.re), F, f)
        im = fx.quantize(np.asarray(sig.im), F, f) if cplx else np.zeros(L, np.int64)
        words = np.stack([re, im], 1).ravel() if cplx else re
        bits = fx.words_to_bits(words, F)
        assert len(bits) == info.n_inputs
        cts = _dev(_lwe_bits(1502 + L, K.s, bits, 2))
        out = torch.zeros((info.n_outputs, n + 1), dtype=torch.int64, device="cuda")
        ws = torch.empty(info.ws_bytes // 8 + 1, dtype=torch.int64, device="cuda")
        S.sfft_ring_fft_execute(plan, K.bkt.data_ptr(), K.ksk_d.data_ptr(), cts.data_ptr(), out.data_ptr(),
                                ws.data_ptr(), info.ws_bytes, _stream())
        torch.cuda.synchronize()
        got = [_decode_q4(c, K.s) for c in _host(out)]
        er, ei = fx.fft1d_fixed(re[None], im[None], F, f)
        want = np.stack([er[0], ei[0]], 1).ravel()
        vals = []
        for v in range(len(want)):
            u = sum(got[v * F + i] << i for i in range(F))
            vals.append(u - (1 << F) if u >> (F - 1) & 1 else u)
        assert vals == want.tolist()
        print("[gpu-case] %d gates, %d levels, %d calls" % (info.gates, info.levels, info.calls), flush=True)
    finally:
        S.sfft_ring_plan_destroy(plan)
