"""CPU tests of libaesgpu's host side: exported symbols, key schedules, the
T-tables (checked against GF(2^8) products from the oracle), a numpy
emulation of the kernels' round structure against the oracle, argument
checking, tuning table and batch planner.  No GPU is touched."""
import os
import re

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from paper_1902_05234_amd import aes, inputs

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "aesgpu.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(aes_\w+)\s*\(", text)))


def test_library_exports_every_header_symbol():
    lib = aes._lib()
    names = header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(aes.exported_symbols())


def test_header_is_plain_c(tmp_path):
    """The boundary header compiles as pedantic C99 (C callers need no C++)
    and as C++17, with no warnings."""
    import shutil
    import subprocess
    src = tmp_path / "use_header.c"
    src.write_text('#include "aesgpu.h"\n'
                   "int main(void) { aes_msg m; aes_work_item w; aes_variant v; (void)m; (void)w; (void)v;\n"
                   "  const char *(*err)(void) = aes_last_error; (void)err;\n"
                   "  return AES_MAX_ITEM_BLOCKS > 0 ? 0 : 1; }\n")
    for cc, lang, std in (("gcc", "c", "-std=c99"), ("g++", "c++", "-std=c++17")):
        if shutil.which(cc) is None:
            pytest.skip("%s not installed" % cc)
        r = subprocess.run([cc, std, "-x", lang, "-Wall", "-Wextra", "-pedantic", "-Werror",
                            "-I" + os.path.dirname(HEADER), "-c", str(src), "-o", str(tmp_path / "o.o")],
                           capture_output=True, text=True)
        assert r.returncode == 0, (cc, r.stderr[-2000:])


def le_words(b: bytes) -> np.ndarray:
    return np.frombuffer(b, dtype="<u4").astype(np.uint32)


@pytest.mark.parametrize("keybits", [128, 192, 256])
def test_encryption_schedule_matches_oracle(oracle_lib, keybits):
    for s in range(20):
        key = inputs.random_key(500 + s, keybits)
        ks = aes.aes_expand_key(key)
        w, nr = oracle_lib.expand_key(key)
        assert ks.nr == nr
        assert np.array_equal(ks.rk_enc, le_words(w))
        ks2 = aes.expand_key(key)  # the short name gives the same schedule
        assert ks2.nr == nr and np.array_equal(ks2.rk_enc, ks.rk_enc) and np.array_equal(ks2.rk_dec, ks.rk_dec)


@pytest.mark.parametrize("keybits", [128, 192, 256])
def test_decryption_schedule_structure(oracle_lib, keybits):
    key = inputs.random_key(77, keybits)
    ks = aes.aes_expand_key(key)
    nr = ks.nr
    e = ks.rk_enc.reshape(nr + 1, 4)
    d = ks.rk_dec.reshape(nr + 1, 4)
    assert np.array_equal(d[0], e[nr]) and np.array_equal(d[nr], e[0])
    for r in range(1, nr):
        want = oracle_lib.inv_mix_columns(e[nr - r].astype("<u4").tobytes())
        assert d[r].astype("<u4").tobytes() == want


def test_key_slot_layout():
    key = inputs.random_key(3, 192)
    slot = aes.aes_key_slot(key)
    ks = aes.aes_expand_key(key)
    n = 4 * (ks.nr + 1)
    assert np.array_equal(slot[:n], ks.rk_enc)
    assert np.array_equal(slot[64:64 + n], ks.rk_dec)
    assert slot[124] == ks.nr
    assert not slot[n:64].any() and not slot[64 + n:124].any()


def rotl(x, n):
    x = np.asarray(x, dtype=np.uint64)
    return (((x << n) | (x >> (32 - n))) & 0xFFFFFFFF).astype(np.uint32) if n else np.asarray(x, dtype=np.uint32)


def test_t_tables_are_the_papers_gf_products(oracle_lib):
    """Eqs 22-25: T_k column of entry w is the GF multiples of s = sbox(w)
    given in tests/golden/paper_t_tables.txt; decryption tables use the
    inverse MixColumns multipliers on InvS(w)."""
    sbox, inv, te0, td0 = aes.aes_host_tables()
    assert np.array_equal(sbox, oracle_lib.sbox())
    assert np.array_equal(inv, oracle_lib.inv_sbox())
    m = oracle_lib.gf_mul_table()
    rows = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "paper_t_tables.txt")):
        if line.strip() and not line.startswith("#"):
            name, *mult = line.split()
            rows[int(name[1])] = [int(v, 16) for v in mult]
    s = oracle_lib.sbox()
    for k in range(4):
        tk = rotl(te0, 8 * k)
        for r in range(4):
            assert np.array_equal((tk >> (8 * r)) & 0xFF, m[rows[k][r], s]), (k, r)
    ai = oracle_lib.inv_mix_matrix()
    si = oracle_lib.inv_sbox()
    for k in range(4):
        tk = rotl(td0, 8 * k)
        for r in range(4):
            assert np.array_equal((tk >> (8 * r)) & 0xFF, m[ai[r, k], si]), (k, r)


# ------------------------------------------------------- numpy kernel emulation
def emulate(ks, data: np.ndarray, decrypt: bool) -> np.ndarray:
    """The kernels' arithmetic on the CPU: eq 26 rounds with the library's
    tables and schedules, final round from T-table bytes (enc) or InvS (dec)."""
    sbox, inv, te0, td0 = aes.aes_host_tables()
    T = [rotl(td0 if decrypt else te0, 8 * k).astype(np.uint32) for k in range(4)]
    rk = (ks.rk_dec if decrypt else ks.rk_enc).astype(np.uint32)
    w = data.reshape(-1, 4).copy().view(np.uint32) if data.dtype == np.uint32 else np.frombuffer(data.tobytes(), dtype="<u4").reshape(-1, 4).astype(np.uint32)
    w = w ^ rk[0:4]
    s = 3 if decrypt else 1
    b = lambda x, t: ((x >> (8 * t)) & 0xFF).astype(np.intp)
    for r in range(1, ks.nr):
        e = np.empty_like(w)
        for j in range(4):
            e[:, j] = (T[0][b(w[:, j], 0)] ^ T[1][b(w[:, (j + s) % 4], 1)] ^ T[2][b(w[:, (j + 2 * s) % 4], 2)]
                       ^ T[3][b(w[:, (j + 3 * s) % 4], 3)] ^ rk[4 * r + j])
        w = e
    out = np.empty_like(w)
    box = inv if decrypt else sbox
    for j in range(4):
        v = np.zeros(w.shape[0], dtype=np.uint32)
        for t in range(4):
            v |= box[b(w[:, (j + t * s) % 4], t)].astype(np.uint32) << (8 * t)
        out[:, j] = v ^ rk[4 * ks.nr + j]
    return out.astype("<u4").view(np.uint8).reshape(-1)


@pytest.mark.parametrize("keybits", [128, 192, 256])
def test_table_emulation_matches_oracle(oracle_lib, keybits):
    key = inputs.random_key(11, keybits)
    ks = aes.aes_expand_key(key)
    x = inputs.random_bytes(12, 16 * 4099)
    c = emulate(ks, x, False)
    assert np.array_equal(c, oracle_lib.ecb_encrypt(key, x))
    p = emulate(ks, c, True)
    assert np.array_equal(p, x)
    assert np.array_equal(emulate(ks, x, True), oracle_lib.ecb_decrypt(key, x))


def test_single_round_identity_eq26(oracle_lib):
    """One T-table round equals SubBytes, ShiftRows, MixColumns, AddRoundKey
    for all 16 x 256 single-byte states and random states."""
    _, _, te0, _ = aes.aes_host_tables()
    T = [rotl(te0, 8 * k) for k in range(4)]
    g = inputs.rng(7)
    states = [bytes(16)]
    for pos in range(16):
        for v in range(256):
            blk = bytearray(16)
            blk[pos] = v
            states.append(bytes(blk))
    states += [g.integers(0, 256, 16, dtype=np.uint8).tobytes() for _ in range(500)]
    k = g.integers(0, 256, 16, dtype=np.uint8).tobytes()
    kw = le_words(k)
    for st_ in states:
        want = oracle_lib.add_round_key(oracle_lib.mix_columns(oracle_lib.shift_rows(oracle_lib.sub_bytes(st_))), k)
        w = le_words(st_)
        e = [int(T[0][w[j] & 0xFF] ^ T[1][(w[(j + 1) % 4] >> 8) & 0xFF] ^ T[2][(w[(j + 2) % 4] >> 16) & 0xFF]
                 ^ T[3][(w[(j + 3) % 4] >> 24) & 0xFF] ^ kw[j]) for j in range(4)]
        assert np.array(e, dtype="<u4").tobytes() == want


# ------------------------------------------------------------- error handling
class FakePtr:
    """Stands in for a tensor: only data_ptr/numel are used by the binding's checks."""


def call_raw(fn_name, *args):
    return getattr(aes._lib(), fn_name)(*args)


def test_expand_key_rejects_bad_sizes():
    lib = aes._lib()
    rk = (aes.ctypes.c_uint32 * 60)()
    key = (aes.ctypes.c_uint8 * 32)()
    for bits in (0, 64, 127, 129, 160, 224, 512, -128):
        assert lib.aes_expand_key(key, bits, rk, rk, None) == aes.AES_EINVAL
        assert "keybits" in aes.aes_last_error()
    assert lib.aes_expand_key(None, 128, rk, rk, None) == aes.AES_EINVAL
    with pytest.raises(aes.AesError):
        aes.aes_expand_key(b"\0" * 20)


def test_ecb_argument_checks_before_any_device_call():
    lib = aes._lib()
    rk = np.zeros(60, dtype=np.uint32).ctypes.data_as(aes._u32p)
    A, B = 0x10000, 0x20000  # never dereferenced: every case fails in host checks
    assert lib.aes_ecb_encrypt(rk, 11, A, B, 4, None) == aes.AES_EINVAL
    assert lib.aes_ecb_decrypt(rk, 9, A, B, 4, None) == aes.AES_EINVAL
    assert lib.aes_ecb_encrypt(None, 10, A, B, 4, None) == aes.AES_EINVAL
    assert lib.aes_ecb_encrypt(rk, 10, A, B, 0, None) == aes.AES_OK           # empty: no launch
    assert lib.aes_ecb_encrypt(rk, 10, None, B, 4, None) == aes.AES_EINVAL
    assert lib.aes_ecb_encrypt(rk, 10, A, None, 4, None) == aes.AES_EINVAL
    assert lib.aes_ecb_encrypt(rk, 10, A + 4, B, 4, None) == aes.AES_EALIGN
    assert lib.aes_ecb_encrypt(rk, 10, A, B + 8, 4, None) == aes.AES_EALIGN
    assert lib.aes_ecb_encrypt(rk, 10, A, A + 16, 4, None) == aes.AES_EINVAL  # partial overlap
    assert "overlap" in aes.aes_last_error()
    bad = [aes.Variant(bpt=3), aes.Variant(wg=100), aes.Variant(wg=2048), aes.Variant(placement=7), aes.Variant(placement=3), aes.Variant(grid=-1),
           aes.Variant(bpt=aes.AES_BPT_COLUMN, placement=aes.AES_PLACEMENT_BITSLICED)]
    for v in bad:
        cv = v._c()
        assert lib.aes_ecb_crypt_variant(rk, 10, 0, A, B, 4, aes.ctypes.byref(cv), None) == aes.AES_EINVAL, v
    assert lib.aes_ecb_crypt_variant(rk, 10, 0, A, B, 4, None, None) == aes.AES_EINVAL


def test_ctr_argument_checks_before_any_device_call():
    lib = aes._lib()
    rk = np.zeros(60, dtype=np.uint32).ctypes.data_as(aes._u32p)
    iv = (aes.ctypes.c_uint8 * 16)()
    A, B = 0x10000, 0x20000  # never dereferenced: every case fails in host checks
    assert lib.aes_ctr_crypt(rk, 11, iv, 0, A, B, 64, None) == aes.AES_EINVAL
    assert lib.aes_ctr_crypt(None, 10, iv, 0, A, B, 64, None) == aes.AES_EINVAL
    assert lib.aes_ctr_crypt(rk, 10, None, 0, A, B, 64, None) == aes.AES_EINVAL
    assert lib.aes_ctr_crypt(rk, 10, iv, 0, A, B, 0, None) == aes.AES_OK            # empty: no launch
    assert lib.aes_ctr_crypt(rk, 10, iv, 0, None, B, 5, None) == aes.AES_EINVAL
    assert lib.aes_ctr_crypt(rk, 10, iv, 0, A, None, 5, None) == aes.AES_EINVAL
    assert lib.aes_ctr_crypt(rk, 10, iv, 0, A + 1, B, 5, None) == aes.AES_EALIGN
    assert lib.aes_ctr_crypt(rk, 10, iv, 0, A, A + 16, 17, None) == aes.AES_EINVAL  # partial overlap
    assert "overlap" in aes.aes_last_error()
    for v in [aes.Variant(bpt=8), aes.Variant(wg=32), aes.Variant(placement=5), aes.Variant(grid=-2),
              aes.Variant(bpt=aes.AES_BPT_COLUMN)]:
        cv = v._c()
        assert lib.aes_ctr_crypt_variant(rk, 10, iv, 0, A, B, 64, aes.ctypes.byref(cv), None) == aes.AES_EINVAL, v
    assert lib.aes_ctr_crypt_variant(rk, 10, iv, 0, A, B, 64, None, None) == aes.AES_EINVAL


def test_cbc_argument_checks_before_any_device_call():
    lib = aes._lib()
    rk = np.zeros(60, dtype=np.uint32).ctypes.data_as(aes._u32p)
    iv = (aes.ctypes.c_uint8 * 16)()
    A, B = 0x10000, 0x20000  # never dereferenced: every case fails in host checks
    assert lib.aes_cbc_decrypt(rk, 13, iv, A, B, 4, None) == aes.AES_EINVAL
    assert lib.aes_cbc_decrypt(None, 10, iv, A, B, 4, None) == aes.AES_EINVAL
    assert lib.aes_cbc_decrypt(rk, 10, None, A, B, 4, None) == aes.AES_EINVAL
    assert lib.aes_cbc_decrypt(rk, 10, iv, A, B, 0, None) == aes.AES_OK             # empty: no launch
    assert lib.aes_cbc_decrypt(rk, 10, iv, A, A, 4, None) == aes.AES_EINVAL         # in place
    assert "in place" in aes.aes_last_error()
    assert lib.aes_cbc_decrypt(rk, 10, iv, A, A + 32, 4, None) == aes.AES_EINVAL    # partial overlap
    assert lib.aes_cbc_decrypt(rk, 10, iv, A + 8, B, 4, None) == aes.AES_EALIGN
    for v in (aes.Variant(bpt=3), aes.Variant(bpt=aes.AES_BPT_COLUMN)):
        cv = v._c()
        assert lib.aes_cbc_decrypt_variant(rk, 10, iv, A, B, 4, aes.ctypes.byref(cv), None) == aes.AES_EINVAL, v
    assert lib.aes_cbc_decrypt_variant(rk, 10, iv, A, B, 4, None, None) == aes.AES_EINVAL


def test_cbc_encrypt_msgs_argument_checks_before_any_device_call():
    lib = aes._lib()
    rk = np.zeros(60, dtype=np.uint32).ctypes.data_as(aes._u32p)
    M, A, B = 0x30000, 0x10000, 0x20000  # never dereferenced: every case fails in host checks
    enc = lib.aes_cbc_encrypt_msgs

    def var(**kw):
        return aes.ctypes.byref(aes.Variant(**kw)._c())

    assert enc(rk, 11, M, 4, A, 64, B, 64, None, None) == aes.AES_EINVAL
    assert enc(None, 10, M, 4, A, 64, B, 64, None, None) == aes.AES_EINVAL
    assert enc(rk, 10, M, 0, A, 64, B, 64, None, None) == aes.AES_OK            # no messages: no launch
    assert enc(rk, 10, None, 4, A, 64, B, 64, None, None) == aes.AES_EINVAL
    assert enc(rk, 10, M, 4, None, 64, B, 64, None, None) == aes.AES_EINVAL
    assert enc(rk, 10, M, 4, A, 64, None, 64, None, None) == aes.AES_EINVAL
    assert enc(rk, 10, M + 8, 4, A, 64, B, 64, None, None) == aes.AES_EALIGN    # message list
    assert enc(rk, 10, M, 4, A + 4, 64, B, 64, None, None) == aes.AES_EALIGN
    assert enc(rk, 10, M, 4, A, 64, B + 8, 64, None, None) == aes.AES_EALIGN
    assert enc(rk, 10, M, 4, A, 64, B, 64, 0x40002, None) == aes.AES_EALIGN    # rejected counter
    # arenas: each with its own length; only the very same arena may be shared
    assert enc(rk, 10, M, 4, A, 4096, A + 1024, 16, None, None) == aes.AES_EINVAL
    assert enc(rk, 10, M, 4, A + 1024, 16, A, 4096, None, None) == aes.AES_EINVAL
    assert "overlap" in aes.aes_last_error()
    encv = lib.aes_cbc_encrypt_msgs_variant
    for v in (dict(bpt=3), dict(bpt=16), dict(placement=aes.AES_PLACEMENT_BITSLICED, wg=256), dict(wg=96),
              dict(grid=-1)):
        assert encv(rk, 10, M, 4, A, 64, B, 64, None, var(**v), None) == aes.AES_EINVAL, v
    assert encv(rk, 10, M, 4, A, 64, B, 64, None, None, None) == aes.AES_EINVAL  # null variant


def test_cbc_decrypt_msgs_argument_checks_before_any_device_call():
    lib = aes._lib()
    rk = np.zeros(60, dtype=np.uint32).ctypes.data_as(aes._u32p)
    M, A, B = 0x30000, 0x10000, 0x20000  # never dereferenced: every case fails in host checks
    dec = lib.aes_cbc_decrypt_msgs
    assert dec(rk, 9, M, 4, A, 64, B, 64, None, None) == aes.AES_EINVAL
    assert dec(None, 10, M, 4, A, 64, B, 64, None, None) == aes.AES_EINVAL
    assert dec(rk, 10, M, 0, A, 64, B, 64, None, None) == aes.AES_OK            # no messages: no launch
    assert dec(rk, 10, None, 4, A, 64, B, 64, None, None) == aes.AES_EINVAL
    assert dec(rk, 10, M + 8, 4, A, 64, B, 64, None, None) == aes.AES_EALIGN
    assert dec(rk, 10, M, 4, A, 64, B, 64, 0x40001, None) == aes.AES_EALIGN
    assert dec(rk, 10, M, 4, A, 4096, A + 16, 1, None, None) == aes.AES_EINVAL   # arenas overlap
    decv = lib.aes_cbc_decrypt_msgs_variant
    for v in (dict(bpt=8), dict(bpt=aes.AES_BPT_COLUMN), dict(bpt=3), dict(bpt=aes.AES_BPT_WAVE_MSG + 4),
              dict(bpt=aes.AES_BPT_WAVE_MSG), dict(placement=aes.AES_PLACEMENT_BITSLICED, wg=256), dict(wg=1088)):
        assert decv(rk, 10, M, 4, A, 64, B, 64, None, aes.ctypes.byref(aes.Variant(**v)._c()), None) == \
            aes.AES_EINVAL, v
    assert decv(rk, 10, M, 4, A, 64, B, 64, None, None, None) == aes.AES_EINVAL  # null variant


def test_cbc_msg_record_layout():
    # the numpy record the binding builds is the C struct aes_cbc_msg
    assert aes.CBC_MSG_DTYPE.itemsize == 48
    assert [aes.CBC_MSG_DTYPE.fields[f][1] for f in ("in_block", "out_block", "nblocks", "reserved", "iv")] == \
        [0, 8, 16, 24, 32]


def test_pipe_config_checks_before_any_device_call():
    lib = aes._lib()
    aes._pipe_sigs(lib)
    h = aes.ctypes.c_void_p()
    A, P = 0x10000, 0x20000  # never dereferenced: every case fails in host checks

    def create(**kw):
        c = dict(dev=A, dev_bytes=1 << 20, pinned=P, pinned_bytes=1 << 20, chunk_bytes=1 << 18, nslots=4, reserved=0)
        c.update(kw)
        cfg = aes._PipeConfig(**c)
        return lib.aes_pipe_create(aes.ctypes.byref(cfg), aes.ctypes.byref(h))

    assert lib.aes_pipe_create(None, aes.ctypes.byref(h)) == aes.AES_EINVAL
    assert create(chunk_bytes=0) == aes.AES_EINVAL
    assert create(chunk_bytes=1000) == aes.AES_EINVAL
    assert create(nslots=0) == aes.AES_EINVAL
    assert create(nslots=aes.AES_PIPE_MAX_SLOTS + 1) == aes.AES_EINVAL
    assert create(dev_bytes=(1 << 20) - 16) == aes.AES_EINVAL
    assert create(chunk_bytes=1 << 62) == aes.AES_EINVAL  # 4 slots: the workspace size would wrap to 0
    assert create(dev=None) == aes.AES_EINVAL
    assert create(pinned_bytes=1 << 19) == aes.AES_EINVAL
    assert create(dev=A + 8) == aes.AES_EALIGN
    assert "16-byte" in aes.aes_last_error()
    rk = np.zeros(60, dtype=np.uint32).ctypes.data_as(aes._u32p)
    assert lib.aes_pipe_run(None, 0, rk, 10, None, A, A, 16, 0) == aes.AES_EINVAL


def test_roof_probe_checks_before_any_device_call():
    lib = aes._lib()
    w = aes.ctypes.c_uint64(0)
    assert lib.aes_roof_probe(7, 10, 0x10000, 1 << 24, aes.ctypes.byref(w), None) == aes.AES_EINVAL
    assert lib.aes_roof_probe(aes.AES_PROBE_LDS, 0, 0x10000, 1 << 24, aes.ctypes.byref(w), None) == aes.AES_EINVAL
    assert lib.aes_roof_probe(aes.AES_PROBE_VALU, (1 << 24) + 1, 0x10000, 1 << 24, None, None) == aes.AES_EINVAL
    assert lib.aes_roof_probe(aes.AES_PROBE_LDS, 10, None, 1 << 24, None, None) == aes.AES_EINVAL


def test_tuning_table_round_trip():
    for nr in (10, 12, 14):
        for dec in (False, True):
            for nb in (1, 300, 5000, 70000, 1 << 22):
                old = aes.aes_tune_get(nr, dec, nb)
                v = aes.Variant(bpt=2, wg=512)
                aes.aes_tune_set(nr, dec, nb, v)
                got = aes.aes_tune_get(nr, dec, nb)
                assert (got.bpt, got.wg, got.placement) == (2, 512, aes.AES_PLACEMENT_TTABLE4)
                aes.aes_tune_set(nr, dec, nb, old)
    assert [aes.aes_size_bucket(n) for n in (1, 256, 257, 4096, 4097, 32768, 32769, 131072, 131073, 524288, 524289,
                                             2097152, 2097153)] == [0, 0, 1, 1, 2, 2, 3, 3, 4, 4, 5, 5, 6]
    with pytest.raises(aes.AesError):
        aes.aes_tune_set(10, False, 1, aes.Variant(bpt=8))
    with pytest.raises(aes.AesError):
        aes.aes_tune_get(13, False, 1)


def test_batch_launch_checks():
    lib = aes._lib()
    cfg = aes._BatchConfig(1, 1024, 0, -1)
    assert lib.aes_ecb_batch(None, 0, 0, None, 0, None, 0, None, 0, None, None, None) == aes.AES_OK
    assert lib.aes_ecb_batch(None, 1, 0, 0x1000, 1, 0x2000, 1, 0x3000, 1, 0x4000, None, None) == aes.AES_EINVAL
    assert lib.aes_ecb_batch(0x1000, 1, 0, 0x1000, 1, 0x2008, 1, 0x3000, 1, 0x4000, None, None) == aes.AES_EALIGN
    cfg.bpt = 5
    assert lib.aes_ecb_batch(0x1000, 1, 0, 0x1000, 1, 0x2000, 1, 0x3000, 1, 0x4000, aes.ctypes.byref(cfg), None) == aes.AES_EINVAL


def test_batch_arena_overlap_uses_each_arenas_own_length():
    """An output arena inside a larger input arena (beyond the smaller
    arena's length from the start) is refused; the very same arena (in
    place) is allowed whatever the two lengths.  A bad bpt stops every
    accepted case before any device call."""
    lib = aes._lib()
    cfg = aes._BatchConfig(5, 1024, 0, -1)
    base = 0x100000
    cases = [
        (base, 1000, base + 16 * 500, 10, True),    # out lies inside in, past 10 blocks from the start
        (base + 16 * 500, 10, base, 1000, True),    # in lies inside out
        (base, 1000, base + 16 * 999, 10, True),    # overlap of one block at the end of in
        (base, 1000, base + 16 * 1000, 10, False),  # adjacent: no overlap
        (base, 1000, base, 10, False),              # the same arena, in place
    ]
    for ib, nin, ob, nout, overlap in cases:
        rc = lib.aes_ecb_batch(0x1000, 1, 0, 0x1000, 1, ib, nin, ob, nout, 0x4000, aes.ctypes.byref(cfg), None)
        assert rc == aes.AES_EINVAL
        assert ("overlap" in aes.aes_last_error()) == overlap, (ib, nin, ob, nout, aes.aes_last_error())


# --------------------------------------------------------------- batch planner
def make_msgs(nblocks, decrypt, slots=None):
    m = np.zeros(len(nblocks), dtype=aes.MSG_DTYPE)
    m["nblocks"] = nblocks
    off = np.concatenate([[0], np.cumsum(nblocks)[:-1]]) if len(nblocks) else []
    m["in_block"] = off
    m["out_block"] = np.asarray(off, dtype=np.uint64) + 7
    m["decrypt"] = decrypt
    m["key_slot"] = slots if slots is not None else np.arange(len(nblocks))
    return m


@settings(max_examples=60, deadline=None)
@given(st.lists(st.tuples(st.integers(0, 5000), st.booleans()), max_size=40), st.integers(1, 2048))
def test_batch_plan_covers_every_block_once(msgs, chunk):
    m = make_msgs([n for n, _ in msgs], [int(d) for _, d in msgs])
    items, ne, nd = aes.aes_batch_plan(m, chunk)
    assert ne + nd == len(items)
    assert (items["nblocks"] >= 1).all() and (items["nblocks"] <= chunk).all()
    for i, msg in enumerate(m):
        part = items[:ne] if not msg["decrypt"] else items[ne:]
        mine = part[part["key_slot"] == i]
        assert int(mine["nblocks"].sum()) == int(msg["nblocks"])
        if len(mine):
            assert mine["in_block"][0] == msg["in_block"]
            assert (np.diff(mine["in_block"].astype(np.int64)) == chunk).all()
            assert (mine["out_block"] - mine["in_block"] == 7).all()


def test_batch_plan_capacity_and_errors():
    lib = aes._lib()
    m = make_msgs([100, 3], [0, 1])
    ne, nd = aes.ctypes.c_size_t(), aes.ctypes.c_size_t()
    items = np.zeros(1, dtype=aes.ITEM_DTYPE)
    rc = lib.aes_batch_plan(m.ctypes.data, 2, 64, items.ctypes.data, 1, aes.ctypes.byref(ne), aes.ctypes.byref(nd))
    assert rc == aes.AES_ERANGE and (ne.value, nd.value) == (2, 1)
    assert lib.aes_batch_plan(m.ctypes.data, 2, 0, items.ctypes.data, 1, aes.ctypes.byref(ne), aes.ctypes.byref(nd)) == aes.AES_EINVAL
    assert lib.aes_batch_plan(None, 2, 8, None, 0, aes.ctypes.byref(ne), aes.ctypes.byref(nd)) == aes.AES_EINVAL
    items, ne_, nd_ = aes.aes_batch_plan(np.zeros(0, dtype=aes.MSG_DTYPE), 64)
    assert len(items) == 0 and ne_ == nd_ == 0


def test_batch_plan_rejects_block_ranges_and_item_counts_that_wrap():
    """Counting and filling agree for any message sizes: a range past 2^64 or
    more than 2^32 - 1 items fails with zero counts and leaves items untouched."""
    lib = aes._lib()
    ne, nd = aes.ctypes.c_size_t(), aes.ctypes.c_size_t()
    items = np.zeros(8, dtype=aes.ITEM_DTYPE)
    items.view(np.uint8)[:] = 0xA5
    before = items.copy()

    def plan(m, chunk):
        ne.value = nd.value = 123
        rc = lib.aes_batch_plan(m.ctypes.data, len(m), chunk, items.ctypes.data, len(items),
                                aes.ctypes.byref(ne), aes.ctypes.byref(nd))
        return rc, ne.value, nd.value

    m = make_msgs([20], [0])
    assert plan(m, aes.AES_MAX_ITEM_BLOCKS + 1) == (aes.AES_EINVAL, 0, 0)
    m["in_block"] = 2**64 - 10
    assert plan(m, 8) == (aes.AES_EINVAL, 0, 0)
    m = make_msgs([20], [1])
    m["out_block"] = 2**64 - 19
    assert plan(m, 8) == (aes.AES_EINVAL, 0, 0)
    m = make_msgs([2**64 - 1], [0])
    m["out_block"] = 0
    assert plan(m, aes.AES_MAX_ITEM_BLOCKS) == (aes.AES_ERANGE, 0, 0)
    m = make_msgs([2**39, 2**39], [0, 1])  # 2^31 items each: one more than fits
    assert plan(m, 256) == (aes.AES_ERANGE, 0, 0)
    assert (items == before).all()
    with pytest.raises(aes.AesError):
        aes.aes_batch_plan(make_msgs([2**64 - 1], [0]), 1)
    # the largest item size splits exactly
    n = 3 * aes.AES_MAX_ITEM_BLOCKS + 5
    got, ne_, nd_ = aes.aes_batch_plan(make_msgs([n], [1]), aes.AES_MAX_ITEM_BLOCKS)
    assert (ne_, nd_) == (0, 4)
    assert got["nblocks"].tolist() == [aes.AES_MAX_ITEM_BLOCKS] * 3 + [5]
    assert got["in_block"].tolist() == [k * aes.AES_MAX_ITEM_BLOCKS for k in range(4)]


def _tune_get_in_child(env_extra):
    """aes_tune_get of three (key size, direction, size) cases in a fresh
    process whose environment adds env_extra; (returncode, values, stderr)."""
    import subprocess
    import sys
    code = ("from paper_1902_05234_amd import aes\n"
            "a = aes.aes_tune_get(14, False, 268435456 // 16)\n"
            "b = aes.aes_tune_get(10, True, 4096 // 16)\n"
            "c = aes.aes_tune_get(10, False, 268435456 // 16)\n"
            "print(a.bpt, a.wg, a.placement, b.bpt, b.wg, b.placement, c.bpt, c.wg, c.placement)\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = {k: v for k, v in os.environ.items() if k not in (aes.TUNE_FILE_ENV, aes.TUNE_FORCE_ENV)}
    env.update(env_extra)
    out = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True, timeout=120)
    vals = [int(x) for x in out.stdout.split()] if out.returncode == 0 else None
    return out.returncode, vals, out.stderr


def test_tune_file_from_environment_replaces_defaults(tmp_path):
    """AESGPU_TUNE_FILE installs an autotune record when the library loads;
    a record made for other kernel sources is refused unless forced."""
    import json
    from paper_1902_05234_amd import autotune
    rec = {"source_hash": autotune.source_hash(),
           "plain": {"256/enc/268435456": {"winner": {"bpt": 1, "wg": 256, "placement": 1}},
                     "128/dec/4096": {"winner": {"bpt": 2, "wg": 128, "placement": 0}}}}
    path = tmp_path / "tune.json"
    path.write_text(json.dumps(rec))
    rc, default, err = _tune_get_in_child({})
    assert rc == 0, err
    rc, got, err = _tune_get_in_child({aes.TUNE_FILE_ENV: str(path)})
    assert rc == 0, err
    # the two covered buckets take the record's variants; AES-128 encrypt of
    # the same size keeps the compiled-in default
    assert got == [1, 256, 1, 2, 128, 0] + default[6:]
    stale = dict(rec, source_hash="0123456789abcdef")
    path.write_text(json.dumps(stale))
    rc, _, err = _tune_get_in_child({aes.TUNE_FILE_ENV: str(path)})
    assert rc != 0 and "RecordMismatch" in err and "kernel sources" in err
    rc, got, err = _tune_get_in_child({aes.TUNE_FILE_ENV: str(path), aes.TUNE_FORCE_ENV: "1"})
    assert rc == 0, err
    assert got == [1, 256, 1, 2, 128, 0] + default[6:]
