"""Test helper: evaluate a gate netlist on bootstrapped ring-LWE gates.

Every Boolean gate of the circuit is one bootstrapped gate (a refresh), so the
FFT circuit's depth needs no modulus sized for it.  The helper levelises the
netlist (a NOT is free and takes its operand's level), runs each level's
gates of one kind as one batched call of `gate_fn(gate, x, y)` on stacked
LWE ciphertexts, and returns the output ciphertexts.  Bits are encoded as
mu * 2 * floor(p/8); constants are the trivial ciphertexts.  The caller
chooses whether gate_fn runs on the GPU (the library) or the CPU (the
oracle).
"""
import numpy as np

from oracle import netlist as N
from oracle import rgsw as O

GATE_CODE = {N.AND: 4, N.XOR: 5, N.OR: 6, N.NAND: 8, N.XADD: 5}   # XADD's operands are never both 1


def _not(c):
    out = (np.uint64(O.P) - c) % np.uint64(O.P)
    out[-1] = (2 * (O.P // 8) + O.P - int(c[-1])) % O.P
    return out


def evaluate(cn, input_cts, n, gate_fn):
    """cn: oracle Compact netlist; input_cts: (n_inputs, n+1) uint64 LWE
    ciphertexts of the input bits; returns (n_outputs, n+1)."""
    depth = [0] * len(cn.t)
    for v, t in enumerate(cn.t):
        if t == N.NOT:
            depth[v] = depth[cn.a[v]]
        elif t in N.BINARY:
            depth[v] = max(depth[cn.a[v]], depth[cn.b[v]]) + 1
    ct = [None] * len(cn.t)
    zero = np.zeros(n + 1, np.uint64)
    one = zero.copy()
    one[n] = 2 * (O.P // 8)
    ct[0], ct[1] = zero, one
    for v, t in enumerate(cn.t):
        if t == N.IN:
            ct[v] = input_cts[cn.a[v]]
    levels = max(depth) if depth else 0
    calls = 0
    for lev in range(levels + 1):
        if lev > 0:
            for t, g in GATE_CODE.items():
                nodes = [v for v in range(len(cn.t)) if depth[v] == lev and cn.t[v] == t]
                if not nodes:
                    continue
                x = np.stack([ct[cn.a[v]] for v in nodes])
                y = np.stack([ct[cn.b[v]] for v in nodes])
                out = gate_fn(g, x, y)
                calls += 1
                for i, v in enumerate(nodes):
                    ct[v] = out[i]
        for v in range(len(cn.t)):   # construction order: operands first
            if cn.t[v] == N.NOT and depth[v] == lev:
                ct[v] = _not(ct[cn.a[v]])
    return np.stack([ct[o] for o in cn.outputs]), levels, calls
