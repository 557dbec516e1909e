"""Pins of the ring-GSW oracle against what the mathematics fixes (no GPU).

* the negacyclic product against a plain full convolution folded with
  X^d = -1 (Python integers), monomial closed forms, and d = 1 (scalars);
* the gadget identities: G^-1(G) is the identity matrix, so G (the
  noiseless encryption of 1) is a two-sided unit of the product, and the
  zero matrix annihilates it;
* the exact phase of a fresh encryption, row by row;
* gate truth tables, the noise bound of one product, and a depth-3 circuit;
* blind rotation: with a noiseless key it is exactly the rotation by
  X^(sum r_i s_i) (coefficients moved by hand); with a real key it decrypts
  to the rotated test polynomial within n * 2*ell*d * B;
* gate bootstrapping: exact output phase mu * 2 * floor(p/4) under a
  noiseless key and noiseless inputs, within the bound under a real key;
* key switching keeps the phase exactly under a noiseless key; bootstrapping
  plus key switching refreshes LWE ciphertexts twice in a row.
"""
import numpy as np
import pytest

from oracle import rgsw as R
from paper_1611_08769_amd import workloads as WL


def _fold_reference(a, b, p):
    d = len(a)
    full = [0] * (2 * d - 1)
    for i in range(d):
        for j in range(d):
            full[i + j] += int(a[i]) * int(b[j])
    return [(full[k] - (full[k + d] if k + d < 2 * d - 1 else 0)) % p for k in range(d)]


@pytest.mark.parametrize("d", [1, 2, 8, 32])
def test_negmul_matches_folded_convolution(d):
    g = np.random.Generator(np.random.PCG64(d))
    for _ in range(3):
        a = g.integers(0, R.P, size=d, dtype=np.uint64)
        b = g.integers(0, R.P, size=d, dtype=np.uint64)
        assert R.negmul(a, b).tolist() == _fold_reference(a, b, R.P)


def test_negmul_monomials_and_scalars():
    d = 16
    for i in range(d):
        for j in range(d):
            xi = np.zeros(d, np.uint64)
            xj = np.zeros(d, np.uint64)
            xi[i] = 1
            xj[j] = 1
            want = np.zeros(d, np.uint64)
            if i + j < d:
                want[i + j] = 1
            else:
                want[i + j - d] = R.P - 1          # X^d = -1
            assert R.negmul(xi, xj).tolist() == want.tolist()
    a, b = 0x3ABCDEF012345678, 0x1234567890ABCDE
    assert int(R.negmul([a], [b])[0]) == a * b % R.P


def _gadget(d, n=1):
    """Noiseless encryption of 1: G, as (n, ROWS, 2, d)."""
    G = np.zeros((n, R.ROWS, 2, d), np.uint64)
    for r in range(R.ROWS):
        G[:, r, r // R.ELL, 0] = (1 << (r % R.ELL)) % R.P
    return G


def test_gadget_is_a_unit_of_the_product():
    d = 8
    dr = WL.ring_draws(1, 2, d, R.ROWS, R.P)
    L = R.encrypt(dr)
    G = _gadget(d, 2)
    # G^-1(L) * G = L  (the decomposition recomposes)
    assert np.array_equal(R.gate(R.AND, L, G), L)
    # G^-1(G) = I, so G^-1(G) * L = L
    assert np.array_equal(R.gate(R.AND, G, L), L)
    # zero annihilates
    Z = np.zeros_like(L)
    assert not R.gate(R.AND, L, Z).any() and not R.gate(R.AND, Z, L).any()
    # NAND(L, G) = G - L = NOT(L); XOR(L, 0) = L; OR(L, 0) = L
    assert np.array_equal(R.gate(R.NAND, L, G), R.gate(R.NOT, L))
    assert np.array_equal(R.gate(R.XOR, L, Z), L)
    assert np.array_equal(R.gate(R.OR, L, Z), L)
    assert np.array_equal(R.gate(R.NOT, R.gate(R.NOT, L)), L)


def test_fresh_phase_is_exact():
    d = 16
    dr = WL.ring_draws(7, 2, d, R.ROWS, R.P, bits=[0, 1])
    ct = R.encrypt(dr)
    s = dr.s
    for c in range(2):
        m = int(dr.bits[c])
        for r in (0, 1, R.ELL - 1, R.ELL, 2 * R.ELL - 1):
            got = R.centred(R.phase(ct[c], r, s))
            want = [int(x) for x in dr.e[c, r]]
            if r < R.ELL:
                want[0] += m << r
            else:
                # the gadget on column 1 contributes -m * 2^(r-ell) * s
                want = [w - m * (1 << (r - R.ELL)) * int(sv) for w, sv in zip(want, s)]
            want = [((w + R.P // 2) % R.P) - R.P // 2 if abs(w) > R.P // 2 else w for w in want]
            assert list(got) == want, (c, r)


@pytest.mark.parametrize("op,fn", [(R.AND, lambda x, y: x & y), (R.XOR, lambda x, y: x ^ y),
                                   (R.OR, lambda x, y: x | y), (R.NAND, lambda x, y: 1 - (x & y))])
def test_truth_tables(op, fn):
    d = 16
    xs = np.array([0, 0, 1, 1], np.uint8)
    ys = np.array([0, 1, 0, 1], np.uint8)
    dx = WL.ring_draws(11, 4, d, R.ROWS, R.P, bits=xs)
    dy = WL.ring_draws(12, 4, d, R.ROWS, R.P, bits=ys)
    dy.s = dx.s                                   # one key
    X, Y = R.encrypt(dx), R.encrypt(dy)
    assert R.decrypt(X, dx.s).tolist() == xs.tolist()
    out = R.gate(op, X, Y)
    assert R.decrypt(out, dx.s).tolist() == [fn(int(a), int(b)) for a, b in zip(xs, ys)]


def test_product_noise_within_bound():
    """After AND the error of the decrypting row is m2*e1 + (G^-1(L)*e2)_row,
    whose coefficients are at most B*(1 + 2*ell*d) in magnitude."""
    d, B = 32, 2
    xs, ys = np.array([1, 1, 0, 1], np.uint8), np.array([1, 0, 1, 1], np.uint8)
    dx = WL.ring_draws(21, 4, d, R.ROWS, R.P, B, bits=xs)
    dy = WL.ring_draws(22, 4, d, R.ROWS, R.P, B, bits=ys)
    dy.s = dx.s
    out = R.gate(R.AND, R.encrypt(dx), R.encrypt(dy))
    for c in range(4):
        ph = R.centred(R.phase(out[c], R.ELL - 1, dx.s))
        m = int(xs[c] & ys[c])
        ph[0] -= m << (R.ELL - 1)
        ph = [((int(v) + R.P // 2) % R.P) - R.P // 2 for v in ph]
        assert max(abs(v) for v in ph) <= B * (1 + 2 * R.ELL * d)
        assert max(abs(v) for v in ph) > 0


def test_depth_three_circuit():
    """((a AND b) XOR c) OR (NOT d) ... evaluated to depth 3 on 8 random inputs."""
    d = 32
    n = 8
    ds = [WL.ring_draws(30 + i, n, d, R.ROWS, R.P) for i in range(4)]
    for x in ds[1:]:
        x.s = ds[0].s
    a, b, c, e = (R.encrypt(x) for x in ds)
    t1 = R.gate(R.AND, a, b)
    t2 = R.gate(R.XOR, t1, c)
    t3 = R.gate(R.OR, t2, R.gate(R.NOT, e))
    bits = [x.bits.astype(int) for x in ds]
    want = ((bits[0] & bits[1]) ^ bits[2]) | (1 - bits[3])
    assert R.decrypt(t3, ds[0].s).tolist() == want.tolist()


def _rotate(a, r, d):
    """X^r * a in Z_p[X]/(X^d + 1), by moving coefficients (r taken mod 2d)."""
    out = [0] * d
    r %= 2 * d
    for u in range(d):
        e = u + r
        sign = 1
        while e >= d:
            e -= d
            sign = -sign
        out[e] = (out[e] + sign * int(a[u])) % R.P
    return out


def test_blind_rotation_with_noiseless_key_is_an_exact_rotation():
    """With bk[i] = s_i * G (no error), each CMux step is exact: the result is
    X^(sum r_i s_i) * acc, coefficient for coefficient."""
    d, n, m = 16, 5, 3
    g = np.random.Generator(np.random.PCG64(8))
    bits = g.integers(0, 2, size=n)
    bk = np.zeros((n, R.ROWS, 2, d), np.uint64)
    for i in range(n):
        if bits[i]:
            bk[i] = _gadget(d)[0]
    rot = g.integers(0, 2 * d, size=(m, n)).astype(np.int32)
    acc = g.integers(0, R.P, size=(m, 2, d), dtype=np.uint64)
    out = R.blind_rotate(bk, rot, acc)
    for j in range(m):
        k = int(sum(int(rot[j, i]) * int(bits[i]) for i in range(n)))
        for col in range(2):
            assert out[j, col].tolist() == _rotate(acc[j, col], k, d), (j, col)


def test_blind_rotation_decrypts_to_the_rotated_test_polynomial():
    """Noisy key (fresh encryptions of s_i), trivial accumulator (TV, 0) with
    TV = 2^61 * t for a 0/1 pattern t: the phase of the result is
    X^(sum r_i s_i) * TV plus an error of at most n * (2*ell*d) * B."""
    d, n, m, B = 32, 4, 2, 2
    dk = WL.ring_draws(60, n, d, R.ROWS, R.P, B)
    bk = R.encrypt(dk)
    g = np.random.Generator(np.random.PCG64(61))
    t = g.integers(0, 2, size=d)
    acc = np.zeros((m, 2, d), np.uint64)
    acc[:, 0, :] = (t.astype(np.uint64) << np.uint64(61)) % np.uint64(R.P)
    rot = g.integers(0, 2 * d, size=(m, n)).astype(np.int32)
    out = R.blind_rotate(bk, rot, acc)
    bound = n * 2 * R.ELL * d * B
    for j in range(m):
        k = int(sum(int(rot[j, i]) * int(dk.bits[i]) for i in range(n)))
        want = _rotate(acc[j, 0], k, d)
        ph = R.rlwe_phase(out[j], dk.s)
        err = [((int(a) - int(b) + R.P // 2) % R.P) - R.P // 2 for a, b in zip(ph, want)]
        assert max(abs(x) for x in err) <= bound
        got_bits = [1 if min(int(v), R.P - int(v)) > R.P // 4 else 0 for v in ph]
        assert got_bits == [1 if min(int(v), R.P - int(v)) > R.P // 4 else 0 for v in want]


def _lwe_inputs(seed, m, n, mus, B=3):
    """LWE ciphertexts mod p of bits mus under a binary secret (test-side
    encryption with Python integers): b = <a, s> + mu*floor(p/2) + e."""
    g = np.random.Generator(np.random.PCG64(seed))
    s = g.integers(0, 2, size=n)
    lwe = np.zeros((m, n + 1), np.uint64)
    for j in range(m):
        a = g.integers(0, R.P, size=n, dtype=np.uint64)
        e = int(g.integers(-B, B + 1))
        b = (sum(int(x) * int(y) for x, y in zip(a, s)) + int(mus[j]) * (R.P // 2) + e) % R.P
        lwe[j, :n] = a
        lwe[j, n] = b
    return s, lwe


def test_bootstrap_refreshes_bits():
    """Gate bootstrapping: the output LWE ciphertexts (under the ring secret)
    decrypt to the input bits, with a phase within the blind rotation's error
    bound of mu * 2 * floor(p/4) -- whatever the inputs' error was."""
    d, n, m, B = 32, 6, 8, 2
    mus = np.array([0, 1, 1, 0, 1, 0, 0, 1])
    s_lwe, lwe = _lwe_inputs(70, m, n, mus)
    dk = WL.ring_draws(71, n, d, R.ROWS, R.P, B, bits=s_lwe.astype(np.uint8))
    out = R.bootstrap(R.encrypt(dk), lwe)
    delta = R.P // 4
    bound = n * 2 * R.ELL * d * B
    for j in range(m):
        ph = R.lwe_phase(out[j], dk.s)
        err = ((ph - int(mus[j]) * 2 * delta + R.P // 2) % R.P) - R.P // 2
        assert abs(err) <= bound, (j, err)


def test_bootstrap_with_noiseless_key_hits_the_encoding_exactly():
    """With a noiseless key (bk[i] = s_i * G) and noiseless inputs, the output
    phase is exactly mu * 2 * floor(p/4)."""
    d, n, m = 16, 4, 6
    mus = np.array([1, 0, 1, 1, 0, 0])
    s_lwe, lwe = _lwe_inputs(80, m, n, mus, B=0)
    bk = np.zeros((n, R.ROWS, 2, d), np.uint64)
    for i in range(n):
        if s_lwe[i]:
            bk[i] = _gadget(d)[0]
    out = R.bootstrap(bk, lwe)
    zero = np.zeros(d, np.int64)   # the ring secret of a noiseless trivial key: its phase is b' itself
    for j in range(m):
        assert R.lwe_phase(out[j], zero) == int(mus[j]) * 2 * (R.P // 4) % R.P, j


def _ksk(seed, s_ring, s_lwe, B):
    """Key-switching key (test-side encryption with Python integers): entry
    [t][k] encrypts s_ring[t] * 16^k under s_lwe, errors in [-B, B]."""
    g = np.random.Generator(np.random.PCG64(seed))
    d, n = len(s_ring), len(s_lwe)
    ksk = np.zeros((d, 16, n + 1), np.uint64)
    ksk[:, :, :n] = g.integers(0, R.P, size=(d, 16, n), dtype=np.uint64)
    e = g.integers(-B, B + 1, size=(d, 16)) if B else np.zeros((d, 16), np.int64)
    sl = [int(x) for x in s_lwe]
    for t in range(d):
        for k in range(16):
            dot = sum(int(x) * y for x, y in zip(ksk[t, k, :n], sl) if y)
            ksk[t, k, n] = (dot + int(s_ring[t]) * (16 ** k) + int(e[t, k])) % R.P
    return ksk


def test_keyswitch_with_noiseless_key_keeps_the_phase():
    """Under a noiseless key-switching key the phase under the new secret
    equals the phase under the old one, exactly."""
    d, n, m = 16, 5, 4
    g = np.random.Generator(np.random.PCG64(90))
    s_ring = g.integers(-1, 2, size=d)
    s_lwe = g.integers(0, 2, size=n)
    ksk = _ksk(91, s_ring, s_lwe, 0)
    lwe = g.integers(0, R.P, size=(m, d + 1), dtype=np.uint64)
    out = R.keyswitch(ksk, lwe)
    for j in range(m):
        assert R.lwe_phase(out[j], s_lwe) == R.lwe_phase(lwe[j], s_ring), j


def test_refresh_round_trip():
    """Bootstrapping then key switching maps LWE ciphertexts under s_lwe back
    to LWE ciphertexts under s_lwe, with errors reset: inputs with errors up
    to p/16 come out with errors below the bound of the two steps, twice in
    a row (2*floor(p/4) = floor(p/2) for this p, so the output encoding is
    the input's)."""
    d, n, m, B = 32, 6, 6, 2
    mus = np.array([1, 0, 0, 1, 1, 0])
    s_lwe, lwe = _lwe_inputs(95, m, n, mus, B=R.P // 16)
    dk = WL.ring_draws(96, n, d, R.ROWS, R.P, B, bits=s_lwe.astype(np.uint8))
    bk = R.encrypt(dk)
    ksk = _ksk(97, dk.s, s_lwe, B)
    bound = n * 2 * R.ELL * d * B + d * 16 * 15 * B
    cur = lwe
    for _ in range(2):
        cur = R.keyswitch(ksk, R.bootstrap(bk, cur))
        assert cur.shape == lwe.shape
        for j in range(m):
            err = ((R.lwe_phase(cur[j], s_lwe) - int(mus[j]) * 2 * (R.P // 4) + R.P // 2) % R.P) - R.P // 2
            assert abs(err) <= bound, (j, err)


def _lwe_bits(seed, s, mus, B):
    """LWE ciphertexts of bits mus encoded as mu * 2 * floor(p/8) under s."""
    g = np.random.Generator(np.random.PCG64(seed))
    n = len(s)
    out = np.zeros((len(mus), n + 1), np.uint64)
    out[:, :n] = g.integers(0, R.P, size=(len(mus), n), dtype=np.uint64)
    for j, mu in enumerate(mus):
        e = int(g.integers(-B, B + 1))
        out[j, n] = (sum(int(out[j, i]) for i in range(n) if s[i]) + int(mu) * 2 * (R.P // 8) + e) % R.P
    return out


def _decode_q4(c, s):
    ph = R.lwe_phase(c, s)
    return 1 if abs(((ph - 2 * (R.P // 8) + R.P // 2) % R.P) - R.P // 2) < R.P // 8 else 0


def _gate_keys(d, n, seed, B=2):
    g = np.random.Generator(np.random.PCG64(seed))
    s_lwe = g.integers(0, 2, size=n)
    dk = WL.ring_draws(seed + 1, n, d, R.ROWS, R.P, B, bits=s_lwe.astype(np.uint8))
    return s_lwe, R.encrypt(dk), _ksk(seed + 2, dk.s, s_lwe, B)


@pytest.mark.parametrize("gate,fn", [(4, lambda a, b: a & b), (6, lambda a, b: a | b),
                                     (8, lambda a, b: 1 - (a & b)), (5, lambda a, b: a ^ b)])
def test_bootstrapped_gate_truth_tables(gate, fn):
    d, n = 16, 6
    s_lwe, bk, ksk = _gate_keys(d, n, 300 + gate)
    xs, ys = [0, 0, 1, 1], [0, 1, 0, 1]
    x = _lwe_bits(310 + gate, s_lwe, xs, R.P // 64)
    y = _lwe_bits(320 + gate, s_lwe, ys, R.P // 64)
    out = R.gate_bootstrap(gate, bk, ksk, x, y)
    assert [_decode_q4(out[j], s_lwe) for j in range(4)] == [fn(a, b) for a, b in zip(xs, ys)]


def test_bootstrapped_gates_compose():
    """A full adder from bootstrapped gates, twice chained (carry into the
    next), on all 8 input triples: outputs decode exactly, errors stay fresh."""
    d, n = 16, 6
    s_lwe, bk, ksk = _gate_keys(d, n, 400)
    trip = [(a, b, c) for a in (0, 1) for b in (0, 1) for c in (0, 1)]
    A = _lwe_bits(401, s_lwe, [t[0] for t in trip], 2)
    Bc = _lwe_bits(402, s_lwe, [t[1] for t in trip], 2)
    C = _lwe_bits(403, s_lwe, [t[2] for t in trip], 2)
    axb = R.gate_bootstrap(5, bk, ksk, A, Bc)
    s_ = R.gate_bootstrap(5, bk, ksk, axb, C)
    carry = R.gate_bootstrap(6, bk, ksk, R.gate_bootstrap(4, bk, ksk, A, Bc), R.gate_bootstrap(4, bk, ksk, axb, C))
    for j, (a, b, c) in enumerate(trip):
        assert _decode_q4(s_[j], s_lwe) == a ^ b ^ c
        assert _decode_q4(carry[j], s_lwe) == (a & b) | (c & (a ^ b))


def test_fft_circuit_on_bootstrapped_gates():
    """The N=4 complex Q(8,4) FFT circuit evaluated gate by gate on the
    oracle's bootstrapped gates (d = 16): every output bit equals the Boolean
    simulation of the same circuit, whatever its depth."""
    from oracle import netlist as N
    from tests import ring_fft_driver as RF
    d, n = 16, 4
    s_lwe, bk, ksk = _gate_keys(d, n, 500)
    cn = N.Compact(N.build_fft_netlist(1, 4, 8, 4, True))
    g = np.random.Generator(np.random.PCG64(501))
    bits = g.integers(0, 2, size=cn.n_inputs)
    cts = _lwe_bits(502, s_lwe, bits, 2)
    out, levels, calls = RF.evaluate(cn, cts, n, lambda gt, x, y: R.gate_bootstrap(gt, bk, ksk, x, y))
    want = N.simulate(cn, [int(b) for b in bits], 1)
    assert levels > 10
    assert [_decode_q4(c, s_lwe) for c in out] == want
