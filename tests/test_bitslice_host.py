"""CPU checks of the bitsliced path's generated code and slice algebra.

The S-box networks in csrc/aes_sbox_circuit.hpp are parsed from the header
text and evaluated here with the documented v_bitop3_b32 semantics (result
bit = immediate bit ((src0 << 2) | (src1 << 1) | src2)) on 32-bit words that
each carry 32 bytes, one per bit position, and compared with the oracle's
S-box and inverse S-box on all 256 inputs."""
import os
import re

import numpy as np

from paper_1902_05234_amd import inputs

HEADER = os.path.join(os.path.dirname(__file__), "..", "paper_1902_05234_amd", "csrc", "aes_sbox_circuit.hpp")


def bitop3(a, b, c, imm):
    out = np.zeros_like(a)
    for idx in range(8):
        if (imm >> idx) & 1:
            ma = a if (idx >> 2) & 1 else ~a
            mb = b if (idx >> 1) & 1 else ~b
            mc = c if idx & 1 else ~c
            out |= ma & mb & mc
    return out


def parse(name):
    text = open(HEADER).read()
    body = text[text.index("void %s(" % name):]
    body = body[:body.index("\n}")]
    stmts = []
    for m in re.finditer(r"const uint32_t (t\d+) = __builtin_amdgcn_bitop3_b32\(([^,]+), ([^,]+), ([^,]+), 0x([0-9a-f]+)\);", body):
        stmts.append((m.group(1), m.group(2).strip(), m.group(3).strip(), m.group(4).strip(), int(m.group(5), 16)))
    outs = dict((int(j), e.strip()) for j, e in re.findall(r"y\[(\d+)\] = ([^;]+);", body))
    return stmts, outs


def run(name, xs):
    """Evaluate the parsed network on 256 bytes packed as 8 groups of 32."""
    stmts, outs = parse(name)
    xs = np.asarray(xs, dtype=np.uint32).reshape(8, 32)
    # bit-slice: slice i of group g = bit i of the 32 bytes of group g
    weights = (np.uint32(1) << np.arange(32, dtype=np.uint32))
    res = np.zeros((8, 32), dtype=np.uint32)
    for g in range(8):
        env = {"x[%d]" % i: np.array([(((xs[g] >> i) & 1) * weights).sum()], dtype=np.uint32) for i in range(8)}
        for t, a, b, c, imm in stmts:
            env[t] = bitop3(env[a], env[b], env[c], imm)
        for j in range(8):
            word = env[outs[j]][0]
            res[g] |= ((word >> np.arange(32, dtype=np.uint32)) & 1).astype(np.uint32) << np.uint32(j)
    return res.reshape(-1)


def test_generated_sbox_network_matches_oracle(oracle_lib):
    assert os.path.exists(HEADER)
    got = run("sbox_slices", np.arange(256))
    assert np.array_equal(got.astype(np.uint8), oracle_lib.sbox())


def test_generated_inverse_sbox_network_matches_oracle(oracle_lib):
    got = run("inv_sbox_slices", np.arange(256))
    assert np.array_equal(got.astype(np.uint8), oracle_lib.inv_sbox())


def test_networks_are_small():
    # one v_bitop3_b32 per LUT; the kernel's cost model assumes about 100 per S-box
    for name in ("sbox_slices", "inv_sbox_slices"):
        stmts, outs = parse(name)
        assert len(stmts) <= 120 and len(outs) == 8
