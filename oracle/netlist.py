"""Oracle: canonical gate netlist of the encrypted FFT, its Boolean simulator and
its noise bound.  TEST INFRASTRUCTURE ONLY -- the product path never imports it.

What is built (paper, section "FFT in FHE"):
  * gates NOT / AND / OR / XOR on encrypted bits (Lemma "binary gates"),
  * half adder = (XOR, AND) and full adder (Lemmas "half adder" / "full adder"),
  * ripple-carry F-bit addition, and subtraction as addition of the inverted
    operand with carry-in 1 (Lemma "add/subtract", the 8-bit adder figure),
  * two's-complement sign extension and a Wallace-tree multiplier by a
    plaintext constant whose zero bits select no partial product, followed by
    the middle-bit slice that implements the fixed-point scaling
    (Lemmas "integer multiplication" / "fixed multiplication"),
  * the radix-2 decimation-in-time butterfly network with plaintext twiddles
    and a plaintext bit-reversal (Lemma "evaluation", Theorem 1), and the
    row-column 2D transform used for images (section "Experimental Results").

The paper gives gates only as NAND compositions and defers the Wallace tree to
Wallace (1964).  The construction below fixes one canonical reading of those
steps (operand order, column rule, constant folding) so that two independent
implementations produce the same directed graph; every reading is listed in
the design notes of the repository.

Node ids 0 and 1 are the constants 0 and 1 and are never materialised.
"""
from __future__ import annotations

import hashlib
import math
import struct

# node types (serialised in the netlist hash with these codes)
IN, CONST0, CONST1, NOT, AND, XOR, OR, XADD, NAND = range(9)
TYPE_NAMES = ["IN", "CONST0", "CONST1", "NOT", "AND", "XOR", "OR", "XADD", "NAND"]
BINARY = (AND, XOR, OR, XADD, NAND)   # node types with two operands
PRODUCT = (AND, XOR, OR, NAND)        # node types evaluated through the product of their operands
ZERO, ONE = 0, 1
RIPPLE, CSA = 0, 1


def is_const(v: int) -> bool:
    return v == ZERO or v == ONE


class Netlist:
    """Gate graph in construction order.  Every gate call creates a new node
    (no structural sharing), so the graph mirrors the circuit as drawn: each
    adder and each Wallace tree owns its gates.

    With nand_only the circuit is the paper's literal one (Lemma "binary
    gates": every gate a NAND; Lemma "full adder": two half adders and an
    OR): NOT x = NAND(x, x), AND = NOT NAND, OR(l, r) = NAND(NOT l, NOT r),
    XOR(l, r) = NAND(NAND(l, t), NAND(r, t)) with t = NAND(l, r), and a full
    adder's carry is OR of the two half-adder carries."""

    def __init__(self, nand_only: bool = False):
        self.nand_only = nand_only
        self.t = [CONST0, CONST1]
        self.a = [-1, -1]
        self.b = [-1, -1]
        self.n_inputs = 0
        self.outputs: list[int] = []

    # -- node creation -------------------------------------------------
    def _node(self, t, a=-1, b=-1):
        i = len(self.t)
        self.t.append(t)
        self.a.append(a)
        self.b.append(b)
        return i

    def inp(self) -> int:
        """Fresh encrypted input bit; `a` holds the input ciphertext index."""
        i = len(self.t)
        self.t.append(IN)
        self.a.append(self.n_inputs)
        self.b.append(-1)
        self.n_inputs += 1
        return i

    # -- gates with constant folding ------------------------------------
    def NAND(self, l, r):
        if l == ZERO or r == ZERO:
            return ONE
        if l == ONE and r == ONE:
            return ZERO
        if l == ONE:
            return self.NOT(r)
        if r == ONE:
            return self.NOT(l)
        return self._node(NAND, l, r)

    def NOT(self, x):
        if x == ZERO:
            return ONE
        if x == ONE:
            return ZERO
        if self.nand_only:
            return self._node(NAND, x, x)
        return self._node(NOT, x)

    def AND(self, l, r):
        if l == ZERO or r == ZERO:
            return ZERO
        if l == ONE:
            return r
        if r == ONE:
            return l
        if self.nand_only:
            t = self._node(NAND, l, r)
            return self._node(NAND, t, t)
        return self._node(AND, l, r)

    def XOR(self, l, r):
        if l == ZERO:
            return r
        if r == ZERO:
            return l
        if l == ONE:
            return self.NOT(r)
        if r == ONE:
            return self.NOT(l)
        if self.nand_only:
            t = self._node(NAND, l, r)
            return self._node(NAND, self._node(NAND, l, t), self._node(NAND, r, t))
        return self._node(XOR, l, r)

    def OR(self, l, r):
        if l == ONE or r == ONE:
            return ONE
        if l == ZERO:
            return r
        if r == ZERO:
            return l
        if self.nand_only:
            return self._node(NAND, self._node(NAND, l, l), self._node(NAND, r, r))
        return self._node(OR, l, r)

    def XADD(self, x, y):
        """Sum of two bits known never to be 1 together (a full adder's two
        partial carries): plain ciphertext addition."""
        if x == ZERO:
            return y
        if y == ZERO:
            return x
        if x == ONE or y == ONE:
            raise ValueError("XADD of a constant 1 with a non-constant bit")
        return self._node(XADD, x, y)

    # -- adders -----------------------------------------------------------
    def HA(self, a, b):
        s = self.XOR(a, b)
        c = self.AND(a, b)
        return s, c

    def FA(self, a, b, c, mode):
        ins = (a, b, c)
        if any(is_const(v) for v in ins):
            nc = [v for v in ins if not is_const(v)]
            K = sum(1 for v in ins if v == ONE)
            if len(nc) == 2:
                x, y = nc
                if K == 0:
                    return self.HA(x, y)
                s = self.NOT(self.XOR(x, y))
                return s, self.OR(x, y)
            if len(nc) == 1:
                x = nc[0]
                if K == 0:
                    return x, ZERO
                if K == 1:
                    return self.NOT(x), x
                return x, ONE
            return (ONE if K & 1 else ZERO), (ONE if K >> 1 else ZERO)
        A = self.AND(a, b)
        X = self.XOR(a, b)
        if mode == RIPPLE:
            P = self.AND(c, X)
            S = self.XOR(c, X)
        else:
            P = self.AND(X, c)
            S = self.XOR(X, c)
        if self.nand_only:
            return S, self.OR(A, P)
        return S, self.XADD(A, P)

    # -- fixed-point words (lists of bit node ids, LSB first) -----------------
    def add(self, x, y):
        carry = ZERO
        out = []
        for i in range(len(x)):
            s, carry = self.FA(x[i], y[i], carry, RIPPLE)
            out.append(s)
        return out

    def sub(self, x, y):
        carry = ONE
        out = []
        for i in range(len(x)):
            nb = self.NOT(y[i])
            s, carry = self.FA(x[i], nb, carry, RIPPLE)
            out.append(s)
        return out

    def mul_const(self, x, c, f):
        """floor(x*c / 2^f) mod 2^F for an encrypted word x and plaintext c."""
        F = len(x)
        W = f + F
        cols = [[] for _ in range(W)]
        cu = c % (1 << (2 * F))
        for i in range(2 * F):
            if (cu >> i) & 1:
                for j in range(W - i):
                    cols[i + j].append(x[min(j, F - 1)])
        while any(len(col) > 2 for col in cols):
            new = [[] for _ in range(W)]
            for w in range(W):
                col = cols[w]
                p = 0
                while len(col) - p >= 3:
                    s, cy = self.FA(col[p], col[p + 1], col[p + 2], CSA)
                    p += 3
                    new[w].append(s)
                    if w + 1 < W:
                        new[w + 1].append(cy)
                if len(col) - p == 2:
                    s, cy = self.HA(col[p], col[p + 1])
                    new[w].append(s)
                    if w + 1 < W:
                        new[w + 1].append(cy)
                elif len(col) - p == 1:
                    new[w].append(col[p])
            cols = new
        carry = ZERO
        out = []
        for w in range(W):
            a = cols[w][0] if len(cols[w]) > 0 else ZERO
            b = cols[w][1] if len(cols[w]) > 1 else ZERO
            s, carry = self.FA(a, b, carry, RIPPLE)
            out.append(s)
        return out[f:f + F]

    # -- FFT ----------------------------------------------------------------
    def fft1d(self, xs, f):
        """Radix-2 DIT over a list of complex words (re_bits, im_bits) in
        natural order; returns natural-order outputs."""
        N = len(xs)
        lg = N.bit_length() - 1
        x = [xs[bitrev(i, lg)] for i in range(N)]
        one = 1 << f
        for s in range(1, lg + 1):
            m = 1 << s
            h = m // 2
            for g in range(0, N, m):
                for j in range(h):
                    cr, ci = twiddle(j, m, f)
                    a = x[g + j]
                    b = x[g + j + h]
                    if (cr, ci) == (one, 0):
                        xi = (self.add(a[0], b[0]), self.add(a[1], b[1]))
                        xj = (self.sub(a[0], b[0]), self.sub(a[1], b[1]))
                    elif (cr, ci) == (0, -one):
                        xi = (self.add(a[0], b[1]), self.sub(a[1], b[0]))
                        xj = (self.sub(a[0], b[1]), self.add(a[1], b[0]))
                    else:
                        m_rr = self.mul_const(b[0], cr, f)
                        m_ii = self.mul_const(b[1], ci, f)
                        tr = self.sub(m_rr, m_ii)
                        m_ir = self.mul_const(b[1], cr, f)
                        m_ri = self.mul_const(b[0], ci, f)
                        ti = self.add(m_ir, m_ri)
                        xi = (self.add(a[0], tr), self.add(a[1], ti))
                        xj = (self.sub(a[0], tr), self.sub(a[1], ti))
                    x[g + j] = xi
                    x[g + j + h] = xj
        return x


def bitrev(i: int, lg: int) -> int:
    r = 0
    for _ in range(lg):
        r = (r << 1) | (i & 1)
        i >>= 1
    return r


def round_half_away(v: float) -> int:
    a = math.floor(abs(v) + 0.5)
    return int(a) if v >= 0 else -int(a)


def twiddle(j: int, m: int, f: int):
    """Plaintext twiddle W_m^j = exp(-2 pi i j / m) in Q(., f): each part
    rounded half away from zero from float64."""
    ang = 2.0 * math.pi * j / m
    return (round_half_away(math.cos(ang) * (1 << f)),
            round_half_away(-math.sin(ang) * (1 << f)))


# ---------------------------------------------------------------------------
# whole-transform netlists
# ---------------------------------------------------------------------------
def build_fft_netlist(dims: int, length: int, F: int, f: int, is_complex: bool, nand_only: bool = False):
    """Canonical netlist of a 1D (dims=1, `length` points) or 2D (dims=2,
    length x length image, rows then columns) forward FFT.

    Input ciphertext index = (v*C + comp)*F + bit (v = point index, row-major
    for images; C = 2 for complex input, 1 for real; comp 0 = Re, 1 = Im).
    Output index = (v*2 + comp)*F + bit in natural order.  nand_only builds
    every gate from NANDs (see Netlist)."""
    nl = Netlist(nand_only)
    npts = length if dims == 1 else length * length
    C = 2 if is_complex else 1
    words = []
    for v in range(npts):
        re = [nl.inp() for _ in range(F)]
        im = [nl.inp() for _ in range(F)] if is_complex else [ZERO] * F
        words.append((re, im))
    if dims == 1:
        out = nl.fft1d(words, f)
    else:
        S = length
        rows = []
        for r in range(S):
            rows.append(nl.fft1d(words[r * S:(r + 1) * S], f))
        out = [None] * npts
        for c in range(S):
            col = nl.fft1d([rows[r][c] for r in range(S)], f)
            for r in range(S):
                out[r * S + c] = col[r]
    outs = []
    for v in range(npts):
        outs.extend(out[v][0])
        outs.extend(out[v][1])
    nl.outputs = outs
    assert nl.n_inputs == npts * C * F
    return nl


# ---------------------------------------------------------------------------
# dead-code elimination, statistics, hash
# ---------------------------------------------------------------------------
class Compact:
    """Nodes reachable from the outputs, renumbered densely in construction
    order (constants keep ids 0 and 1)."""

    def __init__(self, nl: Netlist):
        n = len(nl.t)
        live = bytearray(n)
        live[0] = live[1] = 1
        stack = list(nl.outputs)
        while stack:
            v = stack.pop()
            if live[v]:
                continue
            live[v] = 1
            t = nl.t[v]
            if t in (NOT,):
                stack.append(nl.a[v])
            elif t in BINARY:
                stack.append(nl.a[v])
                stack.append(nl.b[v])
        # inputs are kept even when unused so that input indices stay valid
        for v in range(n):
            if nl.t[v] == IN:
                live[v] = 1
        remap = [-1] * n
        self.t, self.a, self.b = [], [], []
        for v in range(n):
            if not live[v]:
                continue
            remap[v] = len(self.t)
            t = nl.t[v]
            self.t.append(t)
            if t == IN:
                self.a.append(nl.a[v])
                self.b.append(-1)
            elif t == NOT:
                self.a.append(remap[nl.a[v]])
                self.b.append(-1)
            elif t in BINARY:
                self.a.append(remap[nl.a[v]])
                self.b.append(remap[nl.b[v]])
            else:
                self.a.append(-1)
                self.b.append(-1)
        self.outputs = [remap[v] for v in nl.outputs]
        self.n_inputs = nl.n_inputs

    def __len__(self):
        return len(self.t)

    def products(self):
        """Distinct ordered operand pairs of AND/XOR/OR/NAND nodes, in order
        of first appearance."""
        seen = {}
        for v, t in enumerate(self.t):
            if t in PRODUCT:
                key = (self.a[v], self.b[v])
                if key not in seen:
                    seen[key] = len(seen)
        return list(seen.keys())

    def stats(self):
        cnt = [0] * 9
        for t in self.t:
            cnt[t] += 1
        level = [0] * len(self.t)
        for v, t in enumerate(self.t):
            if t == NOT:
                level[v] = level[self.a[v]]
            elif t == XADD:
                level[v] = max(level[self.a[v]], level[self.b[v]])
            elif t in PRODUCT:
                level[v] = 1 + max(level[self.a[v]], level[self.b[v]])
        prods = self.products()
        plev = [1 + max(level[a], level[b]) for a, b in prods]
        depth = max(plev) if plev else 0
        width = [0] * (depth + 1)
        for L in plev:
            width[L] += 1
        return dict(
            nodes=len(self.t),
            products=len(prods),
            gates=cnt[AND] + cnt[XOR] + cnt[OR] + cnt[XADD] + cnt[NAND],
            nots=cnt[NOT],
            depth=depth,
            max_width=max(width) if prods else 0,
            avg_width=(len(prods) / depth) if depth else 0.0,
        )

    def hash(self) -> str:
        """SHA-256 over: per node (type:u8, a:i32, b:i32) little-endian in
        construction order, then the output count (u32) and the output ids
        (i32 each)."""
        h = hashlib.sha256()
        buf = bytearray()
        for v in range(len(self.t)):
            buf += struct.pack("<Bii", self.t[v], self.a[v], self.b[v])
            if len(buf) > (1 << 20):
                h.update(bytes(buf))
                buf.clear()
        buf += struct.pack("<I", len(self.outputs))
        for o in self.outputs:
            buf += struct.pack("<i", o)
        h.update(bytes(buf))
        return h.hexdigest()


# ---------------------------------------------------------------------------
# Boolean simulation (bit-parallel: each wire is a Python int holding one bit
# per sample)
# ---------------------------------------------------------------------------
def simulate(cn: Compact, inputs: list[int], nsamples: int) -> list[int]:
    mask = (1 << nsamples) - 1
    val = [0] * len(cn.t)
    val[1] = mask
    for v, t in enumerate(cn.t):
        if t == IN:
            val[v] = inputs[cn.a[v]]
        elif t == NOT:
            val[v] = val[cn.a[v]] ^ mask
        elif t == AND:
            val[v] = val[cn.a[v]] & val[cn.b[v]]
        elif t == XOR:
            val[v] = val[cn.a[v]] ^ val[cn.b[v]]
        elif t == OR:
            val[v] = val[cn.a[v]] | val[cn.b[v]]
        elif t == XADD:
            x, y = val[cn.a[v]], val[cn.b[v]]
            if x & y:
                raise AssertionError("XADD operands are both 1 for some sample")
            val[v] = x | y
        elif t == NAND:
            val[v] = (val[cn.a[v]] & val[cn.b[v]]) ^ mask
    return [val[o] for o in cn.outputs]


# ---------------------------------------------------------------------------
# noise bound and the parameter rule
# ---------------------------------------------------------------------------
def noise_bounds(cn: Compact, nct: int) -> list[int]:
    """Worst-case |noise| of every node for ciphertext dimension nct.

    A fresh encryption R*A has noise R*e with R binary (nct x m, m = nct) and
    e in {-1,0,1}: at most m.  For a gate of the form alpha*L + beta*R +
    gamma*P with P = BitDecomp(L')*R', the noise is
    (alpha + gamma*mu_R)*e_L + (beta*I + gamma*C_L)*e_R, whose row sums bound
    AND (gamma=1), XOR (1,1,-2) and OR (1,1,-1) as below; NAND = G - P adds
    no noise to P's."""
    B = [0] * len(cn.t)
    for v, t in enumerate(cn.t):
        if t == IN:
            B[v] = nct
        elif t == NOT:
            B[v] = B[cn.a[v]]
        elif t == AND or t == OR or t == NAND:
            B[v] = B[cn.a[v]] + nct * B[cn.b[v]]
        elif t == XOR:
            B[v] = B[cn.a[v]] + (2 * nct - 1) * B[cn.b[v]]
        elif t == XADD:
            B[v] = B[cn.a[v]] + B[cn.b[v]]
    return B


def bound_bits(cn: Compact, nct: int) -> int:
    B = noise_bounds(cn, nct)
    bmax = max((B[o] for o in cn.outputs), default=0)
    return bmax.bit_length() + 3


def choose_k(cn: Compact, n_lwe: int, step: int = 32) -> int:
    """Least k (a multiple of `step`) with bitlen(Bmax(Nct=(n+1)k)) + 3 <= k,
    so that every output's noise stays below q/8 and decryption (which needs
    |noise| < q/4) has a bit of margin."""
    k = step
    while True:
        g = bound_bits(cn, (n_lwe + 1) * k)
        if g <= k:
            return k
        k = -(-g // step) * step


def least_k(cn: Compact, n_lwe: int) -> int:
    """Least integer k (no rounding) satisfying the same rule."""
    lo = choose_k(cn, n_lwe, 32) - 32
    for k in range(max(lo, 1), lo + 33):
        if bound_bits(cn, (n_lwe + 1) * k) <= k:
            return k
    raise AssertionError
