"""CPU checks of the counter-mode kernel's two departures from the plain
round structure, before any GPU run: (1) the split of a CTR launch into
counter-aligned units (the cached whole units and the two edge units)
covers every block exactly once; (2) the shared/lane split of rounds 1-2
(the 27 lookups a unit shares, the 1 + 4 each lane does) gives the same
key stream as the whole cipher, emulated in numpy with the library's
T-table and checked against the CPU oracle's CTR."""
import numpy as np
import pytest

from paper_1902_05234_amd import aes, inputs

M32 = 0xFFFFFFFF


def units(c0_lo, nbytes, span, waves):
    """Blocks each wave handles, as ctr_kernel splits them (counter of data
    block b is c0 + b; unit u holds counter offsets u*span + i from c0 - d)."""
    nfull, nblocks = nbytes // 16, (nbytes + 15) // 16
    d = c0_lo & (span - 1)
    first_full = 1 if d else 0
    end_full = (nfull + d) // span
    n_units = (nblocks + d + span - 1) // span
    seen = []
    for w in range(waves):
        u = first_full + w
        while u < end_full:
            seen += [("full", u * span - d + i) for i in range(span)]
            u += waves
    edge = []
    if d:
        edge.append(0)
    back = max(first_full, end_full)
    if back < n_units and not (d and back == 0):
        edge.append(back)
    for u in edge:
        for i in range(span):
            off = u * span + i
            if off >= d and off - d < nblocks:
                seen.append(("edge", off - d))
    return seen, nfull, nblocks


@pytest.mark.parametrize("span", [64, 128, 256])
def test_ctr_units_cover_every_block_once(span):
    g = inputs.rng(70, span)
    cases = [(0, 16 * span * 3), (5, 16), (255, 16 * 1000 + 7), (span - 1, 16 * (span + 1)), (1, 1)]
    cases += [(int(g.integers(0, 2**63)), int(g.integers(1, 16 * 5 * span))) for _ in range(200)]
    for c0_lo, nbytes in cases:
        for waves in (1, 2, 7):
            seen, nfull, nblocks = units(c0_lo, nbytes, span, waves)
            blocks = sorted(b for _, b in seen)
            assert blocks == list(range(nblocks)), (c0_lo, nbytes, waves)
            # a cached (whole) unit never holds the partial last block, and its
            # counters share bytes 0..14: no carry out of the low byte inside it
            d = c0_lo & (span - 1)
            for kind, b in seen:
                if kind == "full":
                    assert b < nfull
                    assert ((c0_lo - d) + (b + d) // span * span) % 256 + span <= 256


def ks_words(block_ints):
    """State words of 128-bit big-endian counters (word c = bytes 4c..4c+3, LE)."""
    be = b"".join(x.to_bytes(16, "big") for x in block_ints)
    return np.frombuffer(be, dtype="<u4").reshape(-1, 4).astype(np.uint64)


def cached_keystream(ks, c0, nblocks, span):
    """Key stream of counters c0 .. c0+nblocks-1 with rounds 1-2 split as in
    ctr_kernel: per unit, 27 shared lookups; per lane, 1 + 4."""
    _, _, te0, _ = aes.aes_host_tables()
    te0 = te0.astype(np.uint64)
    T = [((te0 << (8 * k)) | (te0 >> (32 - 8 * k))) & M32 if k else te0 for k in range(4)]
    rk = ks.rk_enc.astype(np.uint64)
    b = lambda x, t: ((np.asarray(x) >> np.uint64(8 * t)) & np.uint64(0xFF)).astype(np.intp)
    out = []
    d = c0 % span
    for u in range((nblocks + d + span - 1) // span):
        base = (c0 - d + u * span) % 2**128
        w = ks_words([base])[0]
        x = [np.uint64(w[c] ^ rk[c]) for c in range(4)]
        u0 = T[0][b(x[0], 0)] ^ T[1][b(x[1], 1)] ^ T[2][b(x[2], 2)] ^ rk[4]
        u1 = T[0][b(x[1], 0)] ^ T[1][b(x[2], 1)] ^ T[2][b(x[3], 2)] ^ T[3][b(x[0], 3)] ^ rk[5]
        u2 = T[0][b(x[2], 0)] ^ T[1][b(x[3], 1)] ^ T[2][b(x[0], 2)] ^ T[3][b(x[1], 3)] ^ rk[6]
        u3 = T[0][b(x[3], 0)] ^ T[1][b(x[0], 1)] ^ T[2][b(x[1], 2)] ^ T[3][b(x[2], 3)] ^ rk[7]
        v0 = T[1][b(u1, 1)] ^ T[2][b(u2, 2)] ^ T[3][b(u3, 3)] ^ rk[8]
        v1 = T[0][b(u1, 0)] ^ T[1][b(u2, 1)] ^ T[2][b(u3, 2)] ^ rk[9]
        v2 = T[0][b(u2, 0)] ^ T[1][b(u3, 1)] ^ T[3][b(u1, 3)] ^ rk[10]
        v3 = T[0][b(u3, 0)] ^ T[2][b(u1, 2)] ^ T[3][b(u2, 3)] ^ rk[11]
        lanes = np.arange(span, dtype=np.uint64)
        w3 = (np.uint64(w[3]) + (lanes << np.uint64(24))) & np.uint64(M32)   # only byte 15 moves
        a = u0 ^ T[3][b(w3 ^ rk[3], 3)]
        s = np.stack([v0 ^ T[0][b(a, 0)], v1 ^ T[3][b(a, 3)], v2 ^ T[2][b(a, 2)], v3 ^ T[1][b(a, 1)]], axis=1)
        for r in range(3, ks.nr):
            s = np.stack([T[0][b(s[:, j], 0)] ^ T[1][b(s[:, (j + 1) % 4], 1)] ^ T[2][b(s[:, (j + 2) % 4], 2)]
                          ^ T[3][b(s[:, (j + 3) % 4], 3)] ^ rk[4 * r + j] for j in range(4)], axis=1)
        sbox = aes.aes_host_tables()[0].astype(np.uint64)
        fin = np.stack([(sbox[b(s[:, j], 0)] | (sbox[b(s[:, (j + 1) % 4], 1)] << np.uint64(8))
                         | (sbox[b(s[:, (j + 2) % 4], 2)] << np.uint64(16))
                         | (sbox[b(s[:, (j + 3) % 4], 3)] << np.uint64(24))) ^ rk[4 * ks.nr + j] for j in range(4)],
                       axis=1)
        blocks = fin.astype("<u4").view(np.uint8).reshape(-1, 16)
        for i in range(span):
            if u * span + i >= d and u * span + i - d < nblocks:
                out.append(blocks[i])
    return np.concatenate(out)


@pytest.mark.parametrize("keybits", [128, 192, 256])
@pytest.mark.parametrize("span", [64, 256])
def test_shared_and_lane_lookups_give_the_cipher(oracle_lib, keybits, span):
    key = inputs.random_key(71, keybits)
    ks = aes.aes_expand_key(key)
    # counters whose low 64 bits end near a byte wrap and a 2^64 carry, and one near 2^128
    for c0 in (0x0102030405060708090A0B0C0D0E0FF1, 0x00000000000000FFFFFFFFFFFFFFFFC0, 2**128 - 70):
        n = 3 * span + 5
        want = oracle_lib.ctr_crypt(key, c0.to_bytes(16, "big"), np.zeros(16 * n, dtype=np.uint8))
        got = cached_keystream(ks, c0, n, span)
        assert np.array_equal(got, want), hex(c0)
