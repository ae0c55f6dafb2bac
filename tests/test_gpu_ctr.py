"""GPU parity of counter mode (section 3.1.5, eq 5) against the CPU oracle,
bit-exact: byte lengths with partial last blocks around the wave and
workgroup tiles for every key size; counters that carry across the 64-bit
halves or wrap at 2^128; a message processed in pieces with block offsets;
in place; every kernel variant; 1 GiB checked on windows that the oracle
computes by offset."""
import numpy as np
import pytest

from paper_1902_05234_amd import aes, inputs
from tests.gpu_util import cuda, first_mismatch, to_dev, to_host
from tests.pins import CTR_EDGE_IVS

pytestmark = pytest.mark.gpu

MiB = 1 << 20


def assert_same(got: np.ndarray, want: np.ndarray, what: str):
    i = first_mismatch(got, want)
    assert i is None, "%s: first differing byte %d (block %d)" % (what, i, i // 16)


def gpu_ctr(ks, iv, xd, block_offset=0):
    torch = cuda()
    out = torch.empty_like(xd)
    aes.aes_ctr_crypt(ks.rk_enc, ks.nr, iv, block_offset, xd, out)
    return out


@pytest.mark.parametrize("keybits", [128, 192, 256])
@pytest.mark.parametrize("nbytes", [1, 15, 16, 17, 64 * 16 - 1, 64 * 16 + 3, 1024 * 16 + 5, 4097 * 16 + 15,
                                    65536 * 16 + 7, 4 * MiB + 3])
def test_ctr_lengths_all_key_sizes(oracle_lib, keybits, nbytes):
    key = inputs.random_key(600 + nbytes % 89, keybits)
    iv = inputs.random_bytes(601 + keybits, 16).tobytes()
    x = inputs.random_bytes(602 + nbytes, nbytes)
    ks = aes.aes_expand_key(key)
    got = to_host(gpu_ctr(ks, iv, to_dev(x)))
    assert_same(got, oracle_lib.ctr_crypt(key, iv, x), "ctr %d-bit n=%d" % (keybits, nbytes))


@pytest.mark.parametrize("iv", CTR_EDGE_IVS, ids=lambda b: b.hex())
def test_ctr_counter_carries(oracle_lib, iv):
    key = inputs.random_key(610, 128)
    ks = aes.aes_expand_key(key)
    x = inputs.random_bytes(611, 16 * 5000 + 9)
    assert_same(to_host(gpu_ctr(ks, iv, to_dev(x))), oracle_lib.ctr_crypt(key, iv, x), "iv %s" % iv.hex())
    # offsets that cross the 64-bit boundary of the low half
    for off in (2**64 - 100, 2**64 - 1):
        got = to_host(gpu_ctr(ks, iv, to_dev(x), block_offset=off))
        assert_same(got, oracle_lib.ctr_crypt(key, iv, x, offset=off), "iv %s offset %d" % (iv.hex(), off))


def test_ctr_pieces_equal_whole_and_in_place(oracle_lib):
    torch = cuda()
    key = inputs.random_key(620, 256)
    iv = inputs.random_bytes(621, 16).tobytes()
    ks = aes.aes_expand_key(key)
    x = inputs.random_bytes(622, MiB + 5)
    want = oracle_lib.ctr_crypt(key, iv, x)
    buf = to_dev(x)
    # three pieces at block boundaries, in place, each with its block offset
    cuts = [0, 16 * 1000, 16 * 40000, x.size]
    for a, b in zip(cuts[:-1], cuts[1:]):
        piece = buf[a:b]
        aes.aes_ctr_crypt(ks.rk_enc, ks.nr, iv, a // 16, piece, piece)
    assert_same(to_host(buf), want, "pieces in place")
    # decryption is the same call
    back = torch.empty_like(buf)
    aes.aes_ctr_crypt(ks.rk_enc, ks.nr, iv, 0, buf, back)
    assert_same(to_host(back), x, "ctr(ctr(x))")


VARIANTS = [aes.Variant(bpt=b, wg=w, placement=p) for p in (0, 1, 2) for b in (1, 2, 4) for w in (64, 256, 1024)]


@pytest.mark.parametrize("variant", VARIANTS, ids=lambda v: "p%d_b%d_w%d" % (v.placement, v.bpt, v.wg))
def test_ctr_every_variant(oracle_lib, variant):
    nbytes = 16 * (2 * 4096 + 77) + 11
    x = inputs.random_bytes(630, nbytes)
    xd = to_dev(x)
    torch = cuda()
    for keybits in (128, 192, 256):
        key = inputs.random_key(631, keybits)
        iv = inputs.random_bytes(632, 16).tobytes()
        ks = aes.aes_expand_key(key)
        out = torch.empty_like(xd)
        aes.aes_ctr_crypt_variant(ks.rk_enc, ks.nr, iv, 0, xd, out, variant)
        assert_same(to_host(out), oracle_lib.ctr_crypt(key, iv, x), "%s %d-bit" % (variant, keybits))


def test_ctr_rejects_misaligned_and_short_buffers():
    torch = cuda()
    ks = aes.aes_expand_key(inputs.random_key(640, 128))
    x = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    with pytest.raises(aes.AesError) as e:
        aes.aes_ctr_crypt(ks.rk_enc, ks.nr, bytes(16), 0, x[1:1025], x[2048:3072])
    assert e.value.code == aes.AES_EALIGN
    with pytest.raises(ValueError):
        aes.aes_ctr_crypt(ks.rk_enc, ks.nr, bytes(16), 0, x[:64], x[64:96], nbytes=64)


def test_ctr_1gib_windows(oracle_lib):
    """1 GiB (the bulk size), AES-128: four 1 MiB windows (first, last, two
    seeded) against the oracle started at the window's block offset, and a
    full device round trip."""
    torch = cuda()
    n = 1 << 30
    key = inputs.random_key(650, 128)
    iv = b"\x00" * 8 + b"\xff" * 6 + b"\x00\x00"   # the low half carries after 2^16 blocks
    ks = aes.aes_expand_key(key)
    xd = inputs.device_random_bytes(651, n)
    c = gpu_ctr(ks, iv, xd)
    rng = inputs.rng(652)
    starts = [0, n - MiB] + [int(s) * 16 for s in rng.integers(0, (n - MiB) // 16, size=2)]
    for s in starts:
        xs = to_host(xd[s:s + MiB])
        assert_same(to_host(c[s:s + MiB]), oracle_lib.ctr_crypt(key, iv, xs, offset=s // 16), "window at %d" % s)
    back = torch.empty_like(xd)
    aes.aes_ctr_crypt(ks.rk_enc, ks.nr, iv, 0, c, back)
    assert torch.equal(back, xd)
    del c, back, xd
    torch.cuda.empty_cache()
