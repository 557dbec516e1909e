"""Pins of the CPU oracle against facts it does not derive itself: published
reference outputs, closed-form integer arithmetic, brute-force truth tables,
the textbook GSW13 form, numpy's float64 FFT within the paper's bound, and
the paper's own Table 1 (in distribution)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import fixedpoint as fx
from oracle import gsw, literal_gsw, prng
from oracle import netlist as N

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------------------
# SplitMix64
# ---------------------------------------------------------------------------
def test_splitmix64_reference_outputs():
    """Reference outputs of SplitMix64 (Steele-Lea-Flood / Vigna's
    splitmix64.c): state 0 and state 1234567."""
    s0 = [prng.mix((i + 1) * prng.GAMMA) for i in range(3)]
    assert s0 == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    s1 = [prng.mix(1234567 + (i + 1) * prng.GAMMA) for i in range(3)]
    assert s1 == [6457827717110365317, 3203168211198807973, 9817491932198370423]
    # the C core implements the same counter generator
    lib = gsw.lib()
    for seed, dom, i in [(0, 0, 0), (5, 4, 123456789), (2**63 + 11, 3, 7)]:
        assert lib.or_word(seed, dom, i) == prng.word(seed, dom, i)


def test_ternary_distribution():
    vals = [prng.ternary(9, 3, j) for j in range(20000)]
    c = {v: vals.count(v) / len(vals) for v in (-1, 0, 1)}
    assert set(vals) <= {-1, 0, 1}
    assert abs(c[0] - 0.5) < 0.02 and abs(c[1] - 0.25) < 0.02 and abs(c[-1] - 0.25) < 0.02


# ---------------------------------------------------------------------------
# fixed-point arithmetic: closed forms and exhaustive enumeration at F = 8
# ---------------------------------------------------------------------------
def _bits_of(vals, F):
    """Bit-parallel simulator inputs: input word w, bit i -> int over samples."""
    vals = [int(v) & ((1 << F) - 1) for v in vals]
    return [sum(((v >> i) & 1) << s for s, v in enumerate(vals)) for i in range(F)]


def _words_from_sim(outs, F, nsamp):
    res = []
    for s in range(nsamp):
        u = sum(((outs[i] >> s) & 1) << i for i in range(F))
        res.append(u - (1 << F) if u >= 1 << (F - 1) else u)
    return np.array(res)


@pytest.mark.parametrize("op", ["add", "sub"])
def test_adder_subtractor_exhaustive_F8(op):
    F = 8
    nl = N.Netlist()
    x = [nl.inp() for _ in range(F)]
    y = [nl.inp() for _ in range(F)]
    nl.outputs = nl.add(x, y) if op == "add" else nl.sub(x, y)
    cn = N.Compact(nl)
    a = np.repeat(np.arange(-128, 128), 256)
    b = np.tile(np.arange(-128, 128), 256)
    outs = N.simulate(cn, _bits_of(a, F) + _bits_of(b, F), len(a))
    got = _words_from_sim(outs, F, len(a))
    want = fx.wrap(a + b if op == "add" else a - b, F)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("f", [0, 3, 4, 8])
def test_constant_multiplier_exhaustive_F8(f):
    """Wallace multiplier + middle-bit slice == floor(x*c/2^f) mod 2^8 for
    every x and every constant c in the signed 8-bit range."""
    F = 8
    xs = np.arange(-128, 128)
    for c in range(-128, 128):
        nl = N.Netlist()
        x = [nl.inp() for _ in range(F)]
        nl.outputs = nl.mul_const(x, c, f)
        cn = N.Compact(nl)
        got = _words_from_sim(N.simulate(cn, _bits_of(xs, F), 256), F, 256)
        want = np.array([((int(v) * c) >> f) for v in xs])
        assert np.array_equal(got, fx.wrap(want, F)), c


def test_emulated_multiply_matches_integer_floor():
    rng = np.random.default_rng(5)
    for F, f in [(12, 6), (16, 8), (24, 12), (32, 16)]:
        x = rng.integers(-(1 << (F - 1)), 1 << (F - 1), 2000)
        c = rng.integers(-(1 << f), (1 << f) + 1, 2000)
        got = np.array([fx.fx_mul(xi, ci, F, f) for xi, ci in zip(x, c)])
        want = [((int(a) * int(b)) // (1 << f)) for a, b in zip(x, c)]
        want = [((w + (1 << (F - 1))) % (1 << F)) - (1 << (F - 1)) for w in want]
        assert got.tolist() == want


def test_half_and_full_adder_truth_tables_plain():
    for mode in (N.RIPPLE, N.CSA):
        nl = N.Netlist()
        a, b, c = nl.inp(), nl.inp(), nl.inp()
        s, cy = nl.FA(a, b, c, mode)
        hs, hc = nl.HA(a, b)
        nl.outputs = [s, cy, hs, hc]
        cn = N.Compact(nl)
        samples = [(i >> 0 & 1, i >> 1 & 1, i >> 2 & 1) for i in range(8)]
        ins = [sum(t[j] << s_ for s_, t in enumerate(samples)) for j in range(3)]
        outs = N.simulate(cn, ins, 8)
        for s_, (x, y, z) in enumerate(samples):
            got = [(o >> s_) & 1 for o in outs]
            assert got == [(x + y + z) & 1, (x + y + z) >> 1, (x + y) & 1, (x + y) >> 1]


def test_full_adder_constant_folding_cases():
    """Every constant pattern of the full adder still adds."""
    for pattern in range(27):
        kinds = [(pattern // 3 ** i) % 3 for i in range(3)]  # 0 -> const 0, 1 -> const 1, 2 -> input
        nl = N.Netlist()
        wires = []
        for kd in kinds:
            wires.append(nl.inp() if kd == 2 else kd)
        s, cy = nl.FA(*wires, N.RIPPLE)
        nl.outputs = [s, cy]
        cn = N.Compact(nl)
        nin = cn.n_inputs
        for v in range(1 << nin):
            ins = [(v >> i) & 1 for i in range(nin)]
            outs = N.simulate(cn, ins, 1)
            it = iter(ins)
            vals = [next(it) if kd == 2 else kd for kd in kinds]
            assert outs == [sum(vals) & 1, sum(vals) >> 1]


# ---------------------------------------------------------------------------
# the FFT: exactness on tiny sizes, float64 within the paper's bound,
# and Table 1 in distribution
# ---------------------------------------------------------------------------
def test_fixed_fft_is_exact_dft_for_N_le_4():
    """With twiddles in {1, -i} (N <= 4) no multiply rounds: the fixed-point
    FFT equals the integer DFT sum_n x_n (-i)^(kn) mod 2^F."""
    rng = np.random.default_rng(2)
    F, f = 12, 6
    for Nn in (2, 4):
        re = rng.integers(-300, 300, (50, Nn))
        im = rng.integers(-300, 300, (50, Nn))
        yr, yi = fx.fft1d_fixed(re, im, F, f)
        for s in range(50):
            for k in range(Nn):
                acc = 0
                for n in range(Nn):
                    w = [1, -1j, -1, 1j][(k * n * (4 // Nn)) % 4]
                    acc += (int(re[s, n]) + 1j * int(im[s, n])) * w
                assert yr[s, k] == fx.wrap(int(round(acc.real)), F)
                assert yi[s, k] == fx.wrap(int(round(acc.imag)), F)


@pytest.mark.parametrize("Nn,F,f", [(8, 16, 8), (32, 16, 8), (64, 16, 8), (128, 24, 12), (128, 32, 16)])
def test_fixed_fft_within_theorem_bound(Nn, F, f):
    """Theorem 2: error <= 2^-f (N/2)(log2 N + X_b + 1) against numpy's
    float64 FFT of the unquantised signal (inputs in [-1, 1), X_b = 1)."""
    rng = np.random.default_rng(Nn + F)
    xr = rng.uniform(-1, 1, (64, Nn)) * (0.999 if F == 16 else 1.0)
    xi = rng.uniform(-1, 1, (64, Nn))
    yr, yi = fx.fft1d_fixed(fx.quantize(xr, F, f), fx.quantize(xi, F, f), F, f)
    ex = np.fft.fft(xr + 1j * xi, axis=-1)
    err = np.maximum(fx.wrapped_error(yr, ex.real, F, f), fx.wrapped_error(yi, ex.imag, F, f))
    assert err.max() <= fx.error_bound(Nn, f, 1.0)


def test_fixed_fft2d_within_bound():
    rng = np.random.default_rng(11)
    S, F, f = 16, 16, 8
    x = np.floor(256 * rng.uniform(0, 1, (8, S, S))) / 256
    yr, yi = fx.fft2d_fixed(fx.quantize(x, F, f), np.zeros((8, S, S), np.int64), F, f)
    ex = np.fft.fft2(x)
    err = np.maximum(fx.wrapped_error(yr, ex.real, F, f), fx.wrapped_error(yi, ex.imag, F, f))
    assert err.max() <= fx.error_bound(S * S, f, 1.0)


def test_table1_error_statistics_in_distribution():
    """Paper Table 1 (Q(32,16), random complex signals in [0,1], ~100
    signals): our emulation's mean and sd of the absolute error land within
    a factor 3 of each printed row (the signals themselves are unpublished)."""
    ref = json.load(open(os.path.join(GOLDEN, "table1_errors.json")))
    rng = np.random.default_rng(0)
    for Nn, (total, mean, var, sd) in ref["rows_1d"].items():
        Nn = int(Nn)
        xr, xi = rng.uniform(0, 1, (100, Nn)), rng.uniform(0, 1, (100, Nn))
        yr, yi = fx.fft1d_fixed(fx.quantize(xr, 32, 16), fx.quantize(xi, 32, 16), 32, 16)
        ex = np.fft.fft(xr + 1j * xi, axis=-1)
        st = fx.error_stats(np.concatenate([fx.wrapped_error(yr, ex.real, 32, 16),
                                            fx.wrapped_error(yi, ex.imag, 32, 16)], axis=1))
        assert mean / 3 < st["mean"] < mean * 3, (Nn, st, mean)
        assert sd / 3 < st["sd"] < sd * 3, (Nn, st, sd)
        assert abs(st["var"] - st["sd"] ** 2) < 1e-12  # population variance: sd = sqrt(var)
        assert math.isclose(math.sqrt(var), sd, rel_tol=0.02)  # the table's own columns agree


def test_twiddle_tie_guard():
    """No twiddle sits within 1e-9 of a rounding tie for f <= 16, m <= 256,
    so float64 cos/sin from any libm round to the same integers."""
    worst = min(fx.twiddle_tie_margin(1 << s, f) for s in range(1, 9) for f in range(2, 17))
    assert worst > 1e-9


@pytest.mark.parametrize("dims,L,F,f,cplx", [(1, 8, 8, 4, False), (1, 16, 12, 6, True),
                                             (1, 32, 16, 8, True), (2, 4, 12, 6, False),
                                             (2, 8, 16, 8, False)])
def test_netlist_computes_fixed_point_fft(dims, L, F, f, cplx):
    """Boolean simulation of the gate netlist equals the integer emulation
    bit for bit on random inputs."""
    nl = N.build_fft_netlist(dims, L, F, f, cplx)
    cn = N.Compact(nl)
    rng = np.random.default_rng(L * F)
    S = 40
    shape = (S, L) if dims == 1 else (S, L, L)
    re = rng.integers(-(1 << (F - 1)), 1 << (F - 1), shape)
    im = rng.integers(-(1 << (F - 1)), 1 << (F - 1), shape) if cplx else np.zeros(shape, np.int64)
    # input index (v*C + comp)*F + bit
    C = 2 if cplx else 1
    npts = L if dims == 1 else L * L
    ins = [0] * (npts * C * F)
    for s in range(S):
        rv = re[s].ravel()
        iv = im[s].ravel()
        for v in range(npts):
            for comp, val in enumerate([rv[v], iv[v]][:C]):
                u = int(val) & ((1 << F) - 1)
                for bit in range(F):
                    ins[(v * C + comp) * F + bit] |= ((u >> bit) & 1) << s
    outs = N.simulate(cn, ins, S)
    yr, yi = fx.fft_fixed(dims, re, im, F, f)
    for s in range(S):
        vals = []
        for v in range(npts):
            for comp in range(2):
                u = sum((((outs[(v * 2 + comp) * F + bit]) >> s) & 1) << bit for bit in range(F))
                vals.append(u - (1 << F) if u >= 1 << (F - 1) else u)
        want = np.stack([yr[s].ravel(), yi[s].ravel()], 1).ravel()
        assert vals == want.tolist()


def test_netlist_shape_numbers():
    """Counts of the canonical netlist (products = distinct ordered operand
    pairs of AND/XOR/OR; depth = longest chain of products)."""
    cn = N.Compact(N.build_fft_netlist(1, 8, 8, 4, False))
    st = cn.stats()
    assert (st["products"], st["depth"], st["max_width"]) == (941, 25, 77)
    assert N.choose_k(cn, 1) == 192 and N.least_k(cn, 1) == 179


# ---------------------------------------------------------------------------
# GSW13: textbook form, truth tables, noise
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def small():
    p = gsw.Params(1, 32)
    keys = gsw.keygen(p, 21)
    lit = literal_gsw.LiteralGSW(1, 32, 21)
    return p, keys, lit


def _packed_equal(ct, packed_rows, p):
    return all(gsw.from_limbs(ct[r, b]) == packed_rows[r][b] for r in range(p.nct) for b in range(p.n1))


def test_public_key_relation(small):
    p, keys, lit = small
    for j in range(p.m):
        As = sum(gsw.from_limbs(keys.A[j, b]) * keys.s[b] for b in range(p.n1)) % p.q
        assert gsw.centered(As, p.q) == keys.e[j]


def test_literal_gsw_equals_packed(small):
    """Textbook GSW13 (explicit Flatten of N x N matrices) and the packed
    C' = C G representation agree on encryption, every gate and decryption."""
    p, keys, lit = small
    mus = [0, 1, 1, 0]
    cts = gsw.encrypt(keys, mus, seed=21, first_ct_id=0)
    lits = [lit.enc(mu, i) for i, mu in enumerate(mus)]
    for c, C, mu in zip(cts, lits, mus):
        assert _packed_equal(c, lit.packed(C), p)
        assert lit.dec(C) == mu == gsw.decrypt(keys, c)
        assert np.array_equal(np.unpackbits(c.view(np.uint8), bitorder="little").reshape(p.nct, p.nct),
                              np.array(C, dtype=np.uint8))
    pairs = [(0, 1), (1, 2), (2, 3), (1, 1)]
    for code, fn in [(4, lit.AND), (5, lit.XOR), (6, lit.OR), (7, lit.XADD)]:
        for i, j in pairs:
            if code == 7 and mus[i] & mus[j]:
                continue
            X = gsw.gate(p, code, cts[i], cts[j])
            Cl = fn(lits[i], lits[j])
            assert _packed_equal(X, lit.packed(Cl), p), (code, i, j)
    X = gsw.gate(p, 3, cts[1])
    assert _packed_equal(X, lit.packed(lit.NOT(lits[1])), p)
    # NAND as the paper's primitive: Flatten(I - C1 C2) == NOT(AND)
    nand = lit.nand(lits[1], lits[2])
    assert _packed_equal(gsw.gate(p, 3, gsw.gate(p, 4, cts[1], cts[2])), lit.packed(nand), p)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_gate_truth_tables_encrypted(seed):
    """Every gate decrypts to its truth table; measured noise within the
    propagated bound."""
    p = gsw.Params(1, 64)
    keys = gsw.keygen(p, seed)
    cts = gsw.encrypt(keys, [0, 1], seed=seed)
    nct = p.nct
    for code, fn in [(4, lambda a, b: a & b), (5, lambda a, b: a ^ b), (6, lambda a, b: a | b)]:
        for a in (0, 1):
            for b in (0, 1):
                X = gsw.gate(p, code, cts[a], cts[b])
                assert gsw.decrypt(keys, X) == fn(a, b)
                bound = nct + (2 * nct - 1 if code == 5 else nct) * nct
                assert gsw.max_noise(keys, X, fn(a, b)) <= bound
    for a in (0, 1):
        assert gsw.decrypt(keys, gsw.gate(p, 3, cts[a])) == 1 - a
    X = gsw.gate(p, 7, cts[0], cts[1])
    assert gsw.decrypt(keys, X) == 1 and gsw.max_noise(keys, X, 1) <= 2 * nct


def test_fresh_noise_bound():
    p = gsw.Params(1, 32)
    keys = gsw.keygen(p, 4)
    cts = gsw.encrypt(keys, [0, 1] * 4, seed=4)
    for i, c in enumerate(cts):
        assert gsw.max_noise(keys, c, i & 1) <= p.m


def test_encrypted_adders_and_noise_invariant():
    """Encrypted half/full adders over all inputs: decryptions are the
    truth table and every output's measured noise (all rows) is within its
    propagated bound."""
    p = gsw.Params(1, 96)
    keys = gsw.keygen(p, 8)
    for mode in (N.RIPPLE, N.CSA):
        nl = N.Netlist()
        a, b, c = nl.inp(), nl.inp(), nl.inp()
        s, cy = nl.FA(a, b, c, mode)
        hs, hc = nl.HA(a, b)
        nl.outputs = [s, cy, hs, hc]
        cn = N.Compact(nl)
        B = N.noise_bounds(cn, p.nct)
        for v in range(8):
            bits = [(v >> i) & 1 for i in range(3)]
            cts = gsw.encrypt(keys, bits, seed=8, first_ct_id=3 * v)
            out = gsw.evaluate(p, cn, cts)
            x, y, z = bits
            want = [(x + y + z) & 1, (x + y + z) >> 1, (x + y) & 1, (x + y) >> 1]
            assert gsw.decrypt_many(keys, out) == want
            for o, w, node in zip(out, want, cn.outputs):
                assert gsw.max_noise(keys, o, w) <= B[node]


def test_encrypted_fft_cfg_small_end_to_end():
    """N=8 real Q(8,4), n=1, k from the noise rule: the oracle's encrypted
    FFT decrypts exactly to the integer emulation and every output's noise is
    within its bound, which is below q/8."""
    nl = N.build_fft_netlist(1, 8, 8, 4, False)
    cn = N.Compact(nl)
    k = N.choose_k(cn, 1)
    p = gsw.Params(1, k)
    rng = np.random.default_rng(3)
    q = fx.quantize(rng.uniform(-1, 1, 8), 8, 4)
    keys = gsw.keygen(p, 3)
    cts = gsw.encrypt(keys, fx.words_to_bits(q, 8), seed=3)
    out = gsw.evaluate(p, cn, cts)
    dec = gsw.decrypt_many(keys, out)
    er, ei = fx.fft1d_fixed(q[None], np.zeros((1, 8), np.int64), 8, 4)
    assert fx.bits_to_words(dec, 8).tolist() == np.stack([er[0], ei[0]], 1).ravel().tolist()
    B = N.noise_bounds(cn, p.nct)
    for i in range(0, len(out), 7):  # a spread of outputs (all rows each)
        assert gsw.max_noise(keys, out[i], dec[i]) <= B[cn.outputs[i]] < p.q // 8


# ---------------------------------------------------------------------------
# paper-literal NAND-only circuits (Lemma "binary gates", Lemma "full adder")
# ---------------------------------------------------------------------------
def test_nand_only_gates_adders_truth_tables():
    """NOT/AND/OR/XOR built from NANDs, and full adders whose carry is the OR
    of two half-adder carries, over every input and constant pattern; no
    node of the NAND-only netlist is anything but an input or a NAND."""
    for pattern in range(27):
        kinds = [(pattern // 3 ** i) % 3 for i in range(3)]
        nl = N.Netlist(nand_only=True)
        wires = [nl.inp() if kd == 2 else kd for kd in kinds]
        s, cy = nl.FA(*wires, N.RIPPLE)
        x, y = wires[0], wires[1]
        nl.outputs = [s, cy, nl.NOT(x), nl.AND(x, y), nl.OR(x, y), nl.XOR(x, y)]
        cn = N.Compact(nl)
        assert set(cn.t[2:]) <= {N.IN, N.NAND}
        for v in range(1 << cn.n_inputs):
            ins = [(v >> i) & 1 for i in range(cn.n_inputs)]
            outs = N.simulate(cn, ins, 1)
            it = iter(ins)
            a, b, c = [next(it) if kd == 2 else kd for kd in kinds]
            assert outs == [(a + b + c) & 1, (a + b + c) >> 1, 1 - a, a & b, a | b, a ^ b], (kinds, v)


@pytest.mark.parametrize("op", ["add", "sub", "mul"])
def test_nand_only_words_exhaustive_F6(op):
    F = 6
    lo, hi = -(1 << (F - 1)), 1 << (F - 1)
    if op == "mul":
        xs = np.arange(lo, hi)
        for c in (-31, -17, 5, 22, 31):
            nl = N.Netlist(nand_only=True)
            x = [nl.inp() for _ in range(F)]
            nl.outputs = nl.mul_const(x, c, 3)
            cn = N.Compact(nl)
            got = _words_from_sim(N.simulate(cn, _bits_of(xs, F), len(xs)), F, len(xs))
            assert np.array_equal(got, fx.wrap(np.array([(int(v) * c) >> 3 for v in xs]), F)), c
        return
    nl = N.Netlist(nand_only=True)
    x = [nl.inp() for _ in range(F)]
    y = [nl.inp() for _ in range(F)]
    nl.outputs = nl.add(x, y) if op == "add" else nl.sub(x, y)
    cn = N.Compact(nl)
    a = np.repeat(np.arange(lo, hi), hi - lo)
    b = np.tile(np.arange(lo, hi), hi - lo)
    got = _words_from_sim(N.simulate(cn, _bits_of(a, F) + _bits_of(b, F), len(a)), F, len(a))
    assert np.array_equal(got, fx.wrap(a + b if op == "add" else a - b, F))


def test_nand_only_fft_netlist_and_encrypted_run():
    """The NAND-only FFT netlist simulates to the integer emulation, and an
    encrypted N=4 transform through the packed-GSW oracle decrypts to it."""
    dims, L, F, f, cplx = 1, 4, 6, 3, True
    cn = N.Compact(N.build_fft_netlist(dims, L, F, f, cplx, nand_only=True))
    assert N.Compact(N.build_fft_netlist(dims, L, F, f, cplx)).hash() != cn.hash()
    rng = np.random.default_rng(9)
    re = rng.integers(-32, 32, (1, L))
    im = rng.integers(-32, 32, (1, L))
    words = np.stack([re[0], im[0]], 1).ravel()
    bits = fx.words_to_bits(words, F)
    yr, yi = fx.fft_fixed(1, re, im, F, f)
    want = np.stack([yr.ravel(), yi.ravel()], 1).ravel()
    sim = N.simulate(cn, [int(b) for b in bits], 1)
    assert fx.bits_to_words(np.array(sim), F).tolist() == want.tolist()
    k = N.choose_k(cn, 1)
    keys = gsw.keygen(gsw.Params(1, k), 4)
    out = gsw.evaluate(keys.params, cn, gsw.encrypt(keys, bits, seed=4))
    assert fx.bits_to_words(np.array(gsw.decrypt_many(keys, out)), F).tolist() == want.tolist()
