#!/usr/bin/env python3
"""Generate aes_sbox_circuit.hpp: the AES S-box and inverse S-box as networks
of 3-input lookup tables (one v_bitop3_b32 each) for the bitsliced kernel.

Derivation (S-box = GF(2^8) inverse followed by the affine map, section 3.2.2
Def. 4; the paper gives no construction, so this one is ours):

1. The AES field GF(2)[x]/(x^8+x^4+x^3+x+1) is rewritten as a tower
   GF(((2^2)^2)^2): GF(4) = GF(2)[w]/(w^2+w+1), GF(16) = GF(4)[z]/(z^2+z+N),
   GF(256) = GF(16)[y]/(y^2+y+L).  A root beta of the AES polynomial in the
   tower gives the change of basis x^i -> beta^i (an 8x8 bit matrix X).
2. In the tower, a = ah*y + al has inverse (ah*di)*y + (ah+al)*di with
   d = L*ah^2 + ah*al + al^2 and di = d^-1 in GF(16); GF(16) inverses and
   products reduce the same way to GF(4), whose products take 3 ANDs.  This
   gives a netlist of 2-input AND/XOR gates; linear maps are XOR trees.
3. The S-box netlist is: tower bits = X * input, inversion, output =
   affine(X^-1 * result).  The inverse S-box: tower bits =
   X * A^-1 * (input ^ 0x63), inversion, output = X^-1 * result.
4. Linear maps share common pairs of terms (Paar's greedy heuristic, a few
   fixed tie-breaking orders).  Common gates are merged, then the netlist is
   covered by 3-input cuts
   (area-flow cut selection with a few rounds of exact-area recovery); each
   cut becomes one LUT whose 8-bit truth table is the bitop3 immediate.
   Constant terms (0x63) are folded into the truth tables.
5. Every candidate tower (all N, L, beta) is built and mapped; the smallest
   network is kept, after checking it on all 256 inputs.

Run from anywhere:  python3 gen_sbox_circuit.py  (writes the header beside it)
"""
from __future__ import annotations

import os
import random

# ------------------------------------------------------------ AES field
AES_POLY = 0x11B


def gmul(a: int, b: int) -> int:
    r = 0
    while b:
        if b & 1:
            r ^= a
        a <<= 1
        if a & 0x100:
            a ^= AES_POLY
        b >>= 1
    return r


def ginv(a: int) -> int:
    if a == 0:
        return 0
    r, e, base = 1, 254, a
    while e:
        if e & 1:
            r = gmul(r, base)
        base = gmul(base, base)
        e >>= 1
    return r


def affine(b: int) -> int:
    """The affine map without its constant: bit i = b_i ^ b_{i+4} ^ b_{i+5} ^ b_{i+6} ^ b_{i+7}."""
    out = 0
    for i in range(8):
        v = 0
        for k in (0, 4, 5, 6, 7):
            v ^= (b >> ((i + k) % 8)) & 1
        out |= v << i
    return out


SBOX = [affine(ginv(x)) ^ 0x63 for x in range(256)]
INV_SBOX = [0] * 256
for _x, _s in enumerate(SBOX):
    INV_SBOX[_s] = _x


# --------------------------------------------------------- bit matrices
def mat_apply(cols, v: int) -> int:
    """cols[i] = image of unit vector i."""
    r = 0
    for i in range(8):
        if (v >> i) & 1:
            r ^= cols[i]
    return r


def mat_inverse(cols):
    img = {mat_apply(cols, v): v for v in range(256)}
    if len(img) != 256:
        return None
    return [img[1 << i] for i in range(8)]


AFFINE_COLS = [affine(1 << i) for i in range(8)]
AFFINE_INV_COLS = mat_inverse(AFFINE_COLS)


# ------------------------------------------------------- tower arithmetic
def m4(a, b):
    a1, a0, b1, b0 = a >> 1, a & 1, b >> 1, b & 1
    p, q = a1 & b1, a0 & b0
    t = (a1 ^ a0) & (b1 ^ b0)
    return ((t ^ q) << 1) | (p ^ q)


def make_m16(n):
    def m16(a, b):
        a1, a0, b1, b0 = a >> 2, a & 3, b >> 2, b & 3
        p, q = m4(a1, b1), m4(a0, b0)
        t = m4(a1 ^ a0, b1 ^ b0)
        return ((t ^ q) << 2) | (m4(n, p) ^ q)
    return m16


def make_m256(n, l):
    m16 = make_m16(n)

    def m256(a, b):
        a1, a0, b1, b0 = a >> 4, a & 15, b >> 4, b & 15
        p, q = m16(a1, b1), m16(a0, b0)
        t = m16(a1 ^ a0, b1 ^ b0)
        return ((t ^ q) << 4) | (m16(l, p) ^ q)
    return m16, m256


def towers():
    """Yield (N, L, X): X[i] = beta^i in tower bits, for every valid tower and root."""
    for n in range(1, 4):
        if not all(m4(z, z) ^ z ^ n for z in range(4)):
            continue
        m16 = make_m16(n)
        for l in range(1, 16):
            if not all(m16(y, y) ^ y ^ l for y in range(16)):
                continue
            _, m256 = make_m256(n, l)
            for beta in range(2, 256):
                pw = [1]
                for _ in range(8):
                    pw.append(m256(pw[-1], beta))
                if pw[8] ^ pw[4] ^ pw[3] ^ pw[1] ^ pw[0] == 0 and mat_inverse(pw[:8]) is not None:
                    yield n, l, pw[:8]


# ------------------------------------------------------------- netlist
class Net:
    """Gates over wires; wires 0..7 are the inputs; 'x' = XOR, 'a' = AND (two
    inputs), 'n' = NOT (one input, stored as (op, a, a)); constant terms such as
    0x63 enter as NOT gates, which the LUT mapping absorbs into truth tables."""

    def __init__(self):
        self.gates = []          # (op, a, b)
        self.memo = {}

    def g(self, op, a, b):
        if a > b:
            a, b = b, a
        key = (op, a, b)
        if key in self.memo:
            return self.memo[key]
        self.gates.append(key)
        w = 8 + len(self.gates) - 1
        self.memo[key] = w
        return w

    def xor_all(self, ws):
        ws = sorted(ws)
        if not ws:
            return None
        acc = ws[0]
        for w in ws[1:]:
            acc = self.g("x", acc, w)
        return acc


def linear(net, cols, ins, rng=None):
    """Output bit j = XOR of ins[i] with bit j of cols[i]; None for an all-zero
    row.  Pairs of wires shared by several rows are XORed once (Paar's greedy
    heuristic: repeatedly take the pair that occurs in most rows; ties and the
    order of the remaining chains are broken by rng, or by wire number)."""
    rows = [set(ins[i] for i in range(8) if (cols[i] >> j) & 1) for j in range(8)]
    while True:
        count = {}
        for r in rows:
            rl = sorted(r)
            for a in range(len(rl)):
                for b in range(a + 1, len(rl)):
                    count[(rl[a], rl[b])] = count.get((rl[a], rl[b]), 0) + 1
        top = max(count.values()) if count else 0
        if top < 2:
            break
        cands = sorted(k for k, v in count.items() if v == top)
        a, b = rng.choice(cands) if rng is not None else cands[0]
        w = net.g("x", a, b)
        for r in rows:
            if a in r and b in r:
                r.discard(a)
                r.discard(b)
                r.add(w)
    out = []
    for r in rows:
        rl = sorted(r)
        if rng is not None:
            rng.shuffle(rl)
        out.append(net.xor_all(rl) if rl else None)
    return out


def xor_opt(net, a, b):
    if a is None:
        return b
    if b is None:
        return a
    return net.g("x", a, b)


def build_inversion(net, n, l, t):
    """t: 8 tower-bit wires (bit 0 first) -> 8 tower-bit wires of the inverse."""
    m16 = make_m16(n)

    def g4mul(a, b):
        (a1, a0), (b1, b0) = a, b
        p = net.g("a", a1, b1)
        q = net.g("a", a0, b0)
        tt = net.g("a", net.g("x", a1, a0), net.g("x", b1, b0))
        return (net.g("x", tt, q), net.g("x", p, q))

    def g4add(a, b):
        return (xor_opt(net, a[0], b[0]), xor_opt(net, a[1], b[1]))

    def g4scale(c, a):
        a1, a0 = a
        if c == 1:
            return a
        if c == 2:
            return (net.g("x", a1, a0), a1)
        return (a0, net.g("x", a1, a0))

    def g4sq(a):
        return (a[0], net.g("x", a[0], a[1]))

    def g16mul(a, b):
        (a1, a0), (b1, b0) = a, b
        p, q = g4mul(a1, b1), g4mul(a0, b0)
        tt = g4mul(g4add(a1, a0), g4add(b1, b0))
        return (g4add(tt, q), g4add(g4scale(n, p), q))

    def lin4(bits, f):
        """GF(2)-linear map f on the 4 bits (bit0..bit3) -> 4 wires as ((b3, b2), (b1, b0))."""
        outs = []
        for j in range(4):
            outs.append(net.xor_all([bits[i] for i in range(4) if (f(1 << i) >> j) & 1]))
        return ((outs[3], outs[2]), (outs[1], outs[0]))

    def g16inv(a):
        a1, a0 = a
        d1 = g4mul(a1, a0)

        def f4(v):
            h, lo = v >> 2, v & 3
            return m4(m4(h, h), n) ^ m4(lo, lo)
        bits = [a0[1], a0[0], a1[1], a1[0]]
        lp = []
        for j in range(2):
            lp.append(net.xor_all([bits[i] for i in range(4) if (f4(1 << i) >> j) & 1]))
        delta = g4add(d1, (lp[1], lp[0]))
        dinv = g4sq(delta)
        return (g4mul(a1, dinv), g4mul(g4add(a1, a0), dinv))

    ah = ((t[7], t[6]), (t[5], t[4]))
    al = ((t[3], t[2]), (t[1], t[0]))
    d1 = g16mul(ah, al)

    def fsq(v):
        h, lo = v >> 4, v & 15
        return m16(m16(h, h), l) ^ m16(lo, lo)
    outs = [net.xor_all([t[i] for i in range(8) if (fsq(1 << i) >> j) & 1]) for j in range(4)]
    d = g4add(d1[0], (outs[3], outs[2])), g4add(d1[1], (outs[1], outs[0]))
    di = g16inv(d)
    oh = g16mul(ah, di)
    ol = g16mul((g4add(ah[0], al[0]), g4add(ah[1], al[1])), di)
    return [ol[1][1], ol[1][0], ol[0][1], ol[0][0], oh[1][1], oh[1][0], oh[0][1], oh[0][0]]


def build(n, l, x_cols, inverse: bool, rng=None):
    """Netlist of the S-box (or inverse S-box) in tower (n, l, X); returns
    (net, outputs), inputs being the 8 bits of the byte."""
    net = Net()
    x_inv = mat_inverse(x_cols)
    ins = list(range(8))
    if not inverse:
        t = linear(net, x_cols, ins, rng)
        r = build_inversion(net, n, l, t)
        cols = [affine(x_inv[i]) for i in range(8)]      # tower -> aes basis -> affine
        out = linear(net, cols, r, rng)
        out = [net.g("n", o, o) if (0x63 >> j) & 1 else o for j, o in enumerate(out)]
        return net, out
    cols_in = [mat_apply(x_cols, AFFINE_INV_COLS[i]) for i in range(8)]
    t = linear(net, cols_in, ins, rng)
    in_const = mat_apply(x_cols, mat_apply(AFFINE_INV_COLS, 0x63))
    t = [net.g("n", w, w) if (in_const >> j) & 1 else w for j, w in enumerate(t)]
    r = build_inversion(net, n, l, t)
    out = linear(net, x_inv, r, rng)
    return net, out


# --------------------------------------------------------------- mapping
def lut_map(net, outs):
    """Cover the netlist with 3-input cuts; returns the LUTs (out_wire, leaves,
    truth table) in topological order."""
    n_in = 8
    nw = n_in + len(net.gates)
    fan = [0] * nw
    for op, a, b in net.gates:
        fan[a] += 1
        if op != "n":
            fan[b] += 1
    for o in outs:
        fan[o] += 1

    # all cuts of size <= 3
    cuts = [None] * nw
    for w in range(n_in):
        cuts[w] = [frozenset([w])]
    for k, (op, a, b) in enumerate(net.gates):
        w = n_in + k
        cs = {frozenset([w])}
        if op == "n":
            cs.update(cuts[a])
        for ca in cuts[a]:
            for cb in (cuts[b] if op != "n" else [frozenset()]):
                u = ca | cb
                if len(u) <= 3:
                    cs.add(u)
        cuts[w] = list(cs)

    def func(w, leaves):
        """truth table (as a function of the leaves' values, constants included)
        of wire w over the given leaves."""
        leaves = list(leaves)
        table = 0
        for idx in range(1 << len(leaves)):
            val = {}
            for j, lf in enumerate(leaves):
                val[lf] = (idx >> (len(leaves) - 1 - j)) & 1

            def ev(x):
                if x in val:
                    return val[x]
                op, a, b = net.gates[x - n_in]
                if op == "n":
                    return 1 - ev(a)
                va, vb = ev(a), ev(b)
                return (va ^ vb) if op == "x" else (va & vb)
            table |= ev(w) << idx
        return table

    # area-flow selection, then exact-area recovery
    est = [max(f, 1) for f in fan]
    best = [None] * nw
    for it in range(6):
        af = [0.0] * nw
        for k in range(len(net.gates)):
            w = n_in + k
            choice, score = None, None
            for c in cuts[w]:
                if c == frozenset([w]):
                    continue
                s = 1.0 + sum(af[x] / est[x] for x in c if x >= n_in)
                key = (s, len(c))
                if score is None or key < score:
                    choice, score = c, key
            best[w] = choice
            af[w] = score[0]
        # cover
        refs = [0] * nw
        need = list(outs)
        used = set()
        while need:
            w = need.pop()
            if w < n_in or w in used:
                continue
            used.add(w)
            for x in best[w]:
                refs[x] += 1
                need.append(x)
        for w in range(nw):
            est[w] = max(refs[w] + (1 if w in outs else 0), 1)
    # final cover in topological order
    used = set()
    need = list(outs)
    while need:
        w = need.pop()
        if w < n_in or w in used:
            continue
        used.add(w)
        need.extend(best[w])
    luts = []
    for w in sorted(used):
        leaves = sorted(best[w])
        luts.append((w, leaves, func(w, leaves)))
    return luts


def eval_luts(luts, outs, x):
    """Evaluate the LUT network on byte x (inputs are the raw byte bits)."""
    val = {i: (x >> i) & 1 for i in range(8)}
    for w, leaves, table in luts:
        idx = 0
        for lf in leaves:
            idx = (idx << 1) | val[lf]
        val[w] = (table >> idx) & 1
    y = 0
    for j, o in enumerate(outs):
        y |= val[o] << j
    return y


def map_sbox(n, l, x_cols, inverse, rng=None):
    net, outs = build(n, l, x_cols, inverse, rng)
    luts = lut_map(net, outs)
    want = INV_SBOX if inverse else SBOX
    for x in range(256):
        if eval_luts(luts, outs, x) != want[x]:
            raise AssertionError("circuit mismatch at %d (inverse=%s)" % (x, inverse))
    return luts, outs


SEEDS = range(6)  # tie-breaking orders tried for the linear layers (fixed, so the output is reproducible)


def best_circuit(inverse):
    best = None
    for seed in SEEDS:
        rng = random.Random(seed)
        for n, l, x_cols in towers():
            r = map_sbox(n, l, x_cols, inverse, rng)
            if best is None or len(r[0]) < len(best[0]):
                best = r
    return best


# ---------------------------------------------------------------- output
def bitop3_imm(leaves, table):
    """bitop3 immediate for src0..src2 = leaves (padded by repeating the last)."""
    k = len(leaves)
    imm = 0
    for idx in range(8):
        s0, s1, s2 = (idx >> 2) & 1, (idx >> 1) & 1, idx & 1
        vals = [s0, s1, s2][:k]
        # the leaf tuple is read with leaves[0] as the most significant index bit
        sub = 0
        for v in vals:
            sub = (sub << 1) | v
        # when padding, the extra operands repeat the last leaf: only consistent
        # assignments matter, the rest are don't-cares (set from the leaf values)
        imm |= ((table >> sub) & 1) << idx
    return imm


def emit_function(name, luts, outs):
    lines = ["__device__ __forceinline__ void %s(const uint32_t x[8], uint32_t y[8])" % name, "{"]
    names = {i: "x[%d]" % i for i in range(8)}
    for w, leaves, table in luts:
        v = "t%d" % w
        names[w] = v
        ops = [names[lf] for lf in leaves]
        while len(ops) < 3:
            ops.append(ops[-1])
        imm = bitop3_imm(leaves, table)
        if len(leaves) < 3:
            # unused index bits: make the table independent of the padded operands
            imm = pad_imm(len(leaves), table)
        lines.append("    const uint32_t %s = __builtin_amdgcn_bitop3_b32(%s, %s, %s, 0x%02x);" % (v, ops[0], ops[1], ops[2], imm))
    for j, o in enumerate(outs):
        lines.append("    y[%d] = %s;" % (j, names[o]))
    lines.append("}")
    return "\n".join(lines)


def pad_imm(k, table):
    """Immediate for a k-input table (k < 3) when the operands are (l0, .., l_{k-1}, l_{k-1}, ...)."""
    imm = 0
    for idx in range(8):
        bits = [(idx >> 2) & 1, (idx >> 1) & 1, idx & 1]
        sub = 0
        for v in bits[:k]:
            sub = (sub << 1) | v
        imm |= ((table >> sub) & 1) << idx
    return imm


def main():
    fwd = best_circuit(False)
    inv = best_circuit(True)
    here = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(here, "aes_sbox_circuit.hpp")
    text = [
        "// aes_sbox_circuit.hpp -- generated by gen_sbox_circuit.py; do not edit.",
        "//",
        "// The AES S-box (%d three-input LUTs) and inverse S-box (%d) on bit slices:" % (len(fwd[0]), len(inv[0])),
        "// x[i] holds bit i of 32 independent bytes (one per bit position of the",
        "// word), y[i] receives bit i of their images.  Each LUT is one",
        "// v_bitop3_b32 whose immediate is the truth table, indexed by",
        "// (src0 << 2) | (src1 << 1) | src2.  The networks come from a tower-field",
        "// form of the GF(2^8) inverse followed by the affine map (see the",
        "// generator) and were checked on all 256 inputs when generated.",
        "#pragma once",
        "#include <hip/hip_runtime.h>",
        "#include <cstdint>",
        "",
        "namespace aesgpu {",
        "",
        emit_function("sbox_slices", *fwd),
        "",
        emit_function("inv_sbox_slices", *inv),
        "",
        "}  // namespace aesgpu",
        "",
    ]
    with open(path, "w") as f:
        f.write("\n".join(text))
    print("wrote %s: S-box %d LUTs, inverse %d LUTs" % (path, len(fwd[0]), len(inv[0])))


if __name__ == "__main__":
    main()
