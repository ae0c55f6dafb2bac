"""Pins that tie the CPU oracle to something other than itself.

Each ``pin_*`` takes an ``oracle.Oracle`` and raises ``AssertionError`` when
the oracle disagrees with what the paper (Wang & Chu, arXiv:1902.05234), the
mathematics or an independent implementation fixes.  The suite is run
against the real oracle (test_oracle_pins.py) and against deliberately broken
copies of it (test_oracle_mutants.py), which must each fail at least one pin.
"""
from __future__ import annotations

import os
import shutil
import subprocess

import numpy as np

from paper_1902_05234_amd import inputs

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden_rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line.split()


# ------------------------------------------------------------------ helpers
def clmul(a: int, b: int) -> int:
    """Carry-less product of two polynomials over GF(2) (no reduction)."""
    acc = 0
    while b:
        if b & 1:
            acc ^= a
        a <<= 1
        b >>= 1
    return acc


def poly_mod(p: int, m: int = 0x11B) -> int:
    """Remainder of polynomial long division over GF(2)."""
    dm = m.bit_length()
    while p.bit_length() >= dm:
        p ^= m << (p.bit_length() - dm)
    return p


def openssl_available() -> bool:
    return shutil.which("openssl") is not None


def openssl_ecb(key: bytes, data: bytes, decrypt: bool) -> bytes:
    """AES-ECB through the OpenSSL command-line tool (an independent implementation)."""
    cmd = ["openssl", "enc", "-aes-%d-ecb" % (8 * len(key)), "-nopad", "-K", key.hex()]
    if decrypt:
        cmd.insert(2, "-d")
    r = subprocess.run(cmd, input=data, capture_output=True, check=True)
    return r.stdout


def openssl_ctr(key: bytes, iv: bytes, data: bytes) -> bytes:
    """AES-CTR through the OpenSSL command-line tool (128-bit big-endian counter)."""
    cmd = ["openssl", "enc", "-aes-%d-ctr" % (8 * len(key)), "-K", key.hex(), "-iv", iv.hex()]
    r = subprocess.run(cmd, input=data, capture_output=True, check=True)
    return r.stdout


def openssl_cbc(key: bytes, iv: bytes, data: bytes, decrypt: bool) -> bytes:
    """AES-CBC through the OpenSSL command-line tool, no padding."""
    cmd = ["openssl", "enc", "-aes-%d-cbc" % (8 * len(key)), "-nopad", "-K", key.hex(), "-iv", iv.hex()]
    if decrypt:
        cmd.insert(2, "-d")
    r = subprocess.run(cmd, input=data, capture_output=True, check=True)
    return r.stdout


def counter_blocks(iv: bytes, offset: int, n: int) -> np.ndarray:
    """n successive 128-bit big-endian counters from iv + offset, by Python integers."""
    c0 = int.from_bytes(iv, "big") + offset
    out = b"".join(((c0 + j) % (1 << 128)).to_bytes(16, "big") for j in range(n))
    return np.frombuffer(out, dtype=np.uint8).copy()


# ---------------------------------------------------------------- the pins
def pin_paper_field_examples(o):
    """Section 3.2.1 worked examples (Defs. 1-3, eqs 7-17)."""
    for op, a, b, want, src in _golden_rows("paper_gf_examples.txt"):
        a = int(a, 16)
        want = int(want, 16)
        if op == "add":
            # addition is coefficient-wise, i.e. the oracle's XOR; check the
            # product table is linear in the sum the paper gives
            b = int(b, 16)
            assert a ^ b == want, src
            m = o.gf_mul_table()
            assert np.array_equal(m[a ^ b], m[a] ^ m[b]), src
        elif op == "xtime":
            assert o.xtime(a) == want, src
            assert o.gf_mul(a, 0x02) == want, src
        elif op == "clmul":
            b = int(b, 16)
            assert clmul(a, b) == want, src           # pins the test's own helper
            assert o.gf_mul(a, b) == poly_mod(want), src
        elif op == "mul":
            b = int(b, 16)
            assert o.gf_mul(a, b) == want, src
            assert o.gf_mul(b, a) == want, src
        else:  # pragma: no cover
            raise AssertionError("unknown op " + op)


def pin_field_matches_polynomial_arithmetic(o):
    """Every product equals carry-less multiplication reduced mod m(x) (eq 8),
    computed here by long division -- a different algorithm from the oracle's
    repeated xtime."""
    m = o.gf_mul_table()
    want = np.array([[poly_mod(clmul(a, b)) for b in range(256)] for a in range(256)], dtype=np.uint8)
    assert np.array_equal(m, want)


def pin_field_axioms(o):
    """GF(2^8) is a field: exhaustive commutativity, associativity,
    distributivity, identity, inverses; {03} generates the multiplicative group."""
    m = o.gf_mul_table()
    a = np.arange(256)
    assert np.array_equal(m, m.T)
    assert np.array_equal(m[1], a) and not m[0].any()
    # associativity (a*b)*c == a*(b*c) over all 2^24 triples
    left = m[m[:, :, None], a[None, None, :]]      # [a, b, c] -> (a*b)*c
    right = m[a[:, None, None], m[None, :, :]]     # [a, b, c] -> a*(b*c)
    assert np.array_equal(left, right)
    # distributivity a*(b^c) == a*b ^ a*c over all 2^24 triples
    x = a[:, None] ^ a[None, :]
    assert np.array_equal(m[:, x], m[:, :, None] ^ m[:, None, :])
    inv = np.array([o.gf_inv(v) for v in range(256)])
    assert inv[0] == 0
    assert all(m[v, inv[v]] == 1 for v in range(1, 256))
    p, seen = 1, set()
    for _ in range(255):
        seen.add(p)
        p = int(m[p, 3])
    assert p == 1 and len(seen) == 255


def pin_sbox_structure(o):
    """SubBytes table (Def. 4, eq 18): a permutation; equal to an affine map of
    the field inverse (the map x -> S(inv(x)) ^ S(0) is GF(2)-linear and
    commutes with a one-bit rotation); no fixed or opposite-fixed points;
    differential uniformity 4 and nonlinearity 112 (those of inversion)."""
    s = o.sbox().astype(np.int64)
    si = o.inv_sbox().astype(np.int64)
    assert sorted(s.tolist()) == list(range(256))
    assert np.array_equal(si[s], np.arange(256)) and np.array_equal(s[si], np.arange(256))
    inv = np.array([o.gf_inv(v) for v in range(256)])
    lin = s[inv] ^ s[0]
    xs = np.arange(256)
    assert np.array_equal(lin[xs[:, None] ^ xs[None, :]], lin[:, None] ^ lin[None, :])
    rot = lambda v: ((v << 1) | (v >> 7)) & 0xFF
    assert np.array_equal(lin[rot(xs)], rot(lin))
    assert not np.any(s == xs) and not np.any(s == (xs ^ 0xFF))
    ddt = np.zeros((256, 256), dtype=np.int64)
    for dx in range(1, 256):
        np.add.at(ddt[dx], s ^ s[xs ^ dx], 1)
    assert ddt[1:].max() == 4
    # Walsh spectrum: max |sum (-1)^(a.x ^ b.S(x))| = 32  <=>  nonlinearity 112
    par = np.array([bin(v).count("1") & 1 for v in range(256)])
    sign_x = 1 - 2 * par[xs[:, None] & xs[None, :]]       # [a, x]
    sign_s = 1 - 2 * par[xs[:, None] & s[None, :]]        # [b, x]
    walsh = sign_x @ sign_s.T                               # [a, b]
    assert np.abs(walsh[:, 1:]).max() == 32


def pin_mix_columns(o):
    """MixColumns (Def. 6, eq 20): the matrix is the paper's; A * A^-1 = I over
    GF(2^8); the step function agrees with the matrix; a constant column is a
    fixed point (02^03^01^01 = 01); InvMixColumns undoes it."""
    want = np.array([[int(v, 16) for v in row] for row in _golden_rows("paper_mix_matrix.txt")], dtype=np.uint8)
    a = o.mix_matrix()
    assert np.array_equal(a, want)
    ai = o.inv_mix_matrix()
    m = o.gf_mul_table()
    prod = np.zeros((4, 4), dtype=np.uint8)
    for r in range(4):
        for c in range(4):
            acc = 0
            for k in range(4):
                acc ^= int(m[a[r, k], ai[k, c]])
            prod[r, c] = acc
    assert np.array_equal(prod, np.eye(4, dtype=np.uint8))
    g = inputs.rng(101)
    for _ in range(64):
        blk = g.integers(0, 256, 16, dtype=np.uint8)
        out = np.frombuffer(o.mix_columns(blk.tobytes()), dtype=np.uint8)
        for c in range(4):
            col = blk[4 * c: 4 * c + 4]
            for r in range(4):
                acc = 0
                for k in range(4):
                    acc ^= int(m[want[r, k], col[k]])
                assert out[4 * c + r] == acc
        assert o.inv_mix_columns(out.tobytes()) == blk.tobytes()
    for v in range(256):
        assert o.mix_columns(bytes([v]) * 16) == bytes([v]) * 16


def pin_shift_rows(o):
    """ShiftRows (Def. 5, eq 19) with the standard's byte <-> state map
    (byte r + 4c is row r, column c): row r moves left by r; the inverse
    undoes it."""
    blk = bytes(range(16))
    out = o.shift_rows(blk)
    for r in range(4):
        for c in range(4):
            assert out[r + 4 * c] == blk[r + 4 * ((r + c) % 4)]
    assert o.inv_shift_rows(out) == blk
    assert o.sub_bytes(o.inv_sub_bytes(blk)) == blk


def pin_add_round_key(o):
    """AddRoundKey (Def. 7, eq 21) is a byte-wise XOR in input byte order."""
    g = inputs.rng(102)
    for _ in range(16):
        b = g.integers(0, 256, 16, dtype=np.uint8)
        k = g.integers(0, 256, 16, dtype=np.uint8)
        assert o.add_round_key(b.tobytes(), k.tobytes()) == (b ^ k).tobytes()


def pin_key_schedule_shape(o):
    """Section 3.2.2: Nb*(Nr+1) words; the first Nk words are the key itself."""
    for keybits, rounds, sched_bits in _golden_rows("paper_key_schedule.txt"):
        keybits, rounds, sched_bits = int(keybits), int(rounds), int(sched_bits)
        key = inputs.random_key(7, keybits)
        w, nr = o.expand_key(key)
        assert nr == rounds
        assert 8 * len(w) == sched_bits
        assert w[: len(key)] == key
    for bad in (0, 64, 100, 512):
        try:
            o.expand_key(b"\0" * 16, bad)
        except ValueError:
            continue
        raise AssertionError("accepted keybits=%d" % bad)


def pin_openssl_known_answers(o, per_size: int = 3, nbytes: int = 4096):
    """Full cipher against the OpenSSL command-line tool, an implementation
    independent of the oracle, for all three key sizes, both directions:
    seeded random keys and data, plus the counting-pattern key and plaintext
    of FIPS-197 Appendix C (expected values come from OpenSSL at test time)."""
    if not openssl_available():
        raise AssertionError("openssl command-line tool not found")
    for keybits in (128, 192, 256):
        cases = [(bytes(range(keybits // 8)), bytes.fromhex("00112233445566778899aabbccddeeff"))]
        for s in range(per_size):
            cases.append((inputs.random_key(1000 + s, keybits), inputs.random_bytes(2000 + 10 * s + keybits, nbytes).tobytes()))
        for key, data in cases:
            assert o.ecb_encrypt(key, data).tobytes() == openssl_ecb(key, data, False), (keybits, key.hex())
            assert o.ecb_decrypt(key, data).tobytes() == openssl_ecb(key, data, True), (keybits, key.hex())


def pin_round_trip(o):
    """Decryption inverts encryption for every key size."""
    for keybits in (128, 192, 256):
        key = inputs.random_key(3, keybits)
        x = inputs.random_bytes(4, 16 * 257)
        y = o.ecb_encrypt(key, x)
        assert not np.array_equal(x, y)
        assert np.array_equal(o.ecb_decrypt(key, y), x)


def pin_ecb_structure(o):
    """ECB (section 3.1.1, eq 1): block i of the output depends on block i of
    the input only; equal blocks give equal results; thread count is
    irrelevant."""
    key = inputs.random_key(5, 128)
    x = inputs.random_bytes(6, 16 * 64).reshape(64, 16)
    x[10] = x[3]
    y = o.ecb_encrypt(key, x, nthreads=1).reshape(64, 16)
    assert np.array_equal(y[10], y[3])
    perm = inputs.rng(103).permutation(64)
    yp = o.ecb_encrypt(key, x[perm], nthreads=5).reshape(64, 16)
    assert np.array_equal(yp, y[perm])


# counters whose increments carry within the low half, across the two 64-bit
# halves, and wrap at 2^128
CTR_EDGE_IVS = [
    bytes(15) + b"\xfe",
    bytes(8) + b"\xff" * 8,
    bytes(7) + b"\x05" + b"\xff" * 8,
    b"\xff" * 16,
]


def pin_ctr_openssl(o):
    """CTR (section 3.1.5, eq 5) against the OpenSSL command-line tool: all
    key sizes, seeded keys and counters, lengths with a partial last block,
    and counters that carry across the 64-bit halves or wrap at 2^128."""
    if not openssl_available():
        raise AssertionError("openssl command-line tool not found")
    for keybits in (128, 192, 256):
        key = inputs.random_key(3000 + keybits, keybits)
        ivs = [inputs.random_bytes(3100 + keybits, 16).tobytes()] + CTR_EDGE_IVS
        for i, iv in enumerate(ivs):
            for n in (1, 15, 16, 17, 16 * 37 + 5):
                data = inputs.random_bytes(3200 + 7 * i + n, n).tobytes()
                assert o.ctr_crypt(key, iv, data).tobytes() == openssl_ctr(key, iv, data), (keybits, iv.hex(), n)


def pin_ctr_structure(o):
    """CTR (eq 5): the key stream is the cipher of successive counters and does
    not depend on the data; applying it twice restores the data; a start
    offset of k blocks continues the same stream; a prefix of the data gets
    the prefix of the result; the thread count is irrelevant."""
    for keybits in (128, 192, 256):
        key = inputs.random_key(3300 + keybits, keybits)
        for iv in [inputs.random_bytes(3301, 16).tobytes()] + CTR_EDGE_IVS:
            nblk = 19
            zeros = np.zeros(16 * nblk, dtype=np.uint8)
            stream = o.ctr_crypt(key, iv, zeros, nthreads=3)
            assert np.array_equal(stream, o.ecb_encrypt(key, counter_blocks(iv, 0, nblk))), iv.hex()
            stream7 = o.ctr_crypt(key, iv, zeros[: 16 * (nblk - 7)], offset=7, nthreads=2)
            assert np.array_equal(stream7, stream[16 * 7:]), iv.hex()
            x = inputs.random_bytes(3302 + keybits, 16 * nblk - 9)
            y = o.ctr_crypt(key, iv, x, nthreads=1)
            assert np.array_equal(y ^ x, stream[: x.size])
            assert np.array_equal(o.ctr_crypt(key, iv, y, nthreads=4), x)
            assert np.array_equal(o.ctr_crypt(key, iv, x[:33]), y[:33])
    # a start offset past 2^64 blocks still adds as a 128-bit integer
    key = inputs.random_key(3400, 128)
    iv = b"\x00" * 7 + b"\x01" + b"\xff" * 8
    off = (1 << 64) - 3
    got = o.ctr_crypt(key, iv, np.zeros(16 * 6, dtype=np.uint8), offset=off)
    assert np.array_equal(got, o.ecb_encrypt(key, counter_blocks(iv, off, 6)))


def pin_cbc_openssl(o):
    """CBC (section 3.1.2, eq 2 read with the block cipher) against the
    OpenSSL command-line tool, both directions, all key sizes."""
    if not openssl_available():
        raise AssertionError("openssl command-line tool not found")
    for keybits in (128, 192, 256):
        key = inputs.random_key(3500 + keybits, keybits)
        iv = inputs.random_bytes(3501 + keybits, 16).tobytes()
        for nblk in (1, 2, 37):
            data = inputs.random_bytes(3502 + nblk, 16 * nblk).tobytes()
            assert o.cbc_encrypt(key, iv, data).tobytes() == openssl_cbc(key, iv, data, False), (keybits, nblk)
            assert o.cbc_decrypt(key, iv, data, nthreads=3).tobytes() == openssl_cbc(key, iv, data, True), (keybits, nblk)


def pin_cbc_structure(o):
    """CBC (eq 2): decryption inverts encryption; plaintext block i is the
    ECB decryption of ciphertext block i XOR ciphertext block i-1 (the
    initialisation vector for i = 1); the first ciphertext block is the ECB
    encryption of P_1 XOR IV; changing ciphertext block i changes plaintext
    blocks i and i+1 only; the thread count is irrelevant."""
    for keybits in (128, 192, 256):
        key = inputs.random_key(3600 + keybits, keybits)
        iv = inputs.random_bytes(3601 + keybits, 16).tobytes()
        ivn = np.frombuffer(iv, dtype=np.uint8)
        x = inputs.random_bytes(3602 + keybits, 16 * 29)
        c = o.cbc_encrypt(key, iv, x)
        assert np.array_equal(o.cbc_decrypt(key, iv, c, nthreads=4), x)
        assert np.array_equal(c[:16], o.ecb_encrypt(key, x[:16] ^ ivn))
        prev = np.concatenate([ivn, c[:-16]])
        assert np.array_equal(o.cbc_decrypt(key, iv, c, nthreads=1), o.ecb_decrypt(key, c) ^ prev)
        c2 = c.copy()
        c2[16 * 7 + 3] ^= 0x40
        d2 = o.cbc_decrypt(key, iv, c2, nthreads=2).reshape(-1, 16)
        changed = [i for i in range(29) if not np.array_equal(d2[i], x.reshape(-1, 16)[i])]
        assert changed == [7, 8], changed


ALL_PINS = [
    pin_paper_field_examples,
    pin_field_matches_polynomial_arithmetic,
    pin_field_axioms,
    pin_sbox_structure,
    pin_mix_columns,
    pin_shift_rows,
    pin_add_round_key,
    pin_key_schedule_shape,
    pin_round_trip,
    pin_ecb_structure,
    pin_openssl_known_answers,
    pin_ctr_structure,
    pin_ctr_openssl,
    pin_cbc_structure,
    pin_cbc_openssl,
]

# pins that need the openssl command-line tool
OPENSSL_PINS = (pin_openssl_known_answers, pin_ctr_openssl, pin_cbc_openssl)
