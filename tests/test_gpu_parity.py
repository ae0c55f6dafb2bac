"""GPU parity: the HIP kernels against the CPU oracle, bit-exact (tolerance 0:
AES is a permutation of 16-byte blocks, so exactly one output is correct).

Sizes: the 4 MiB AES-128 case checked in full; every key size over ragged
block counts around the wave (64 blocks) and workgroup (1024 blocks) tiles;
every plain-path variant; the 1 MiB ... 4 GiB sweep (full oracle up to
16 MiB, four 1 MiB windows plus a device round trip above that)."""
import numpy as np
import pytest

from paper_1902_05234_amd import aes, inputs
from tests.gpu_util import cuda, first_mismatch, to_dev, to_host

pytestmark = pytest.mark.gpu

MiB = 1 << 20


def gpu_enc(ks, x_dev):
    torch = cuda()
    out = torch.empty_like(x_dev)
    aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, x_dev, out)
    return out


def gpu_dec(ks, x_dev):
    torch = cuda()
    out = torch.empty_like(x_dev)
    aes.aes_ecb_decrypt(ks.rk_dec, ks.nr, x_dev, out)
    return out


def assert_same(got: np.ndarray, want: np.ndarray, what: str):
    i = first_mismatch(got, want)
    assert i is None, "%s: first differing byte %d (block %d)" % (what, i, i // 16)


def test_aes128_4mib_encrypt_then_decrypt(oracle_lib):
    """AES-128, one 4 MiB buffer (262,144 blocks), seeded key and data."""
    key = inputs.random_key(0, 128)
    x = inputs.random_bytes(0, 4 * MiB)
    ks = aes.aes_expand_key(key)
    c_dev = gpu_enc(ks, to_dev(x))
    c = to_host(c_dev)
    assert_same(c, oracle_lib.ecb_encrypt(key, x), "encrypt")
    p = to_host(gpu_dec(ks, c_dev))
    assert_same(p, x, "decrypt(encrypt(x))")
    assert_same(to_host(gpu_dec(ks, to_dev(x))), oracle_lib.ecb_decrypt(key, x), "decrypt of random data")


@pytest.mark.parametrize("keybits", [128, 192, 256])
@pytest.mark.parametrize("nblocks", [1, 2, 63, 64, 65, 1023, 1024, 1025, 4097, 65536 + 17, 262144 + 33])
def test_ragged_sizes_all_key_sizes(oracle_lib, keybits, nblocks):
    key = inputs.random_key(10 + nblocks % 97, keybits)
    x = inputs.random_bytes(20 + nblocks, 16 * nblocks)
    ks = aes.aes_expand_key(key)
    xd = to_dev(x)
    assert_same(to_host(gpu_enc(ks, xd)), oracle_lib.ecb_encrypt(key, x), "enc %d-bit n=%d" % (keybits, nblocks))
    assert_same(to_host(gpu_dec(ks, xd)), oracle_lib.ecb_decrypt(key, x), "dec %d-bit n=%d" % (keybits, nblocks))


VARIANTS = [aes.Variant(bpt=b, wg=w, placement=p, grid=g) for p in (0, 1, 2) for b in (aes.AES_BPT_COLUMN, 1, 2, 4)
            for w in (64, 128, 256, 512, 1024) for g in (0, 3)]


@pytest.mark.parametrize("variant", VARIANTS, ids=lambda v: "p%d-bpt%d-wg%d-g%d" % (v.placement, v.bpt, v.wg, v.grid))
def test_every_variant(oracle_lib, variant):
    nblocks = 2 * 4096 + 77
    x = inputs.random_bytes(31, 16 * nblocks)
    xd = to_dev(x)
    torch = cuda()
    for keybits, dec in ((128, False), (256, True), (192, False)):
        key = inputs.random_key(32, keybits)
        ks = aes.aes_expand_key(key)
        out = torch.empty_like(xd)
        rk = ks.rk_dec if dec else ks.rk_enc
        aes.aes_ecb_crypt_variant(rk, ks.nr, dec, xd, out, variant)
        want = oracle_lib.ecb_decrypt(key, x) if dec else oracle_lib.ecb_encrypt(key, x)
        assert_same(to_host(out), want, "%s %d-bit dec=%s" % (variant, keybits, dec))


@pytest.mark.parametrize("placement", [0, 1, 2])
def test_column_variant_every_key_size_and_direction(oracle_lib, placement):
    """One column per lane (four lanes per block): every key size in both
    directions, block counts around the 16-block wave unit and the quads of
    a ragged last unit, in place, and a grid of one workgroup that walks the
    whole buffer."""
    torch = cuda()
    for nblocks in (1, 3, 15, 16, 17, 63, 1000, 4096 + 5):
        x = inputs.random_bytes(700 + nblocks, 16 * nblocks)
        for keybits in (128, 192, 256):
            key = inputs.random_key(701 + keybits, keybits)
            ks = aes.aes_expand_key(key)
            for dec, wg, grid in ((False, 256, 0), (True, 1024, 0), (False, 64, 1), (True, 128, 1)):
                v = aes.Variant(bpt=aes.AES_BPT_COLUMN, wg=wg, placement=placement, grid=grid)
                xd = to_dev(x)
                out = torch.empty_like(xd)
                rk = ks.rk_dec if dec else ks.rk_enc
                aes.aes_ecb_crypt_variant(rk, ks.nr, dec, xd, out, v)
                want = oracle_lib.ecb_decrypt(key, x) if dec else oracle_lib.ecb_encrypt(key, x)
                assert_same(to_host(out), want, "%s %d-bit dec=%s %d blocks" % (v, keybits, dec, nblocks))
                aes.aes_ecb_crypt_variant(rk, ks.nr, dec, xd, xd, v)  # in place
                assert_same(to_host(xd), want, "in place %s %d-bit dec=%s %d blocks" % (v, keybits, dec, nblocks))


def test_in_place_and_prefix(oracle_lib):
    torch = cuda()
    key = inputs.random_key(40, 256)
    ks = aes.aes_expand_key(key)
    x = inputs.random_bytes(41, 16 * 5000)
    buf = to_dev(x)
    aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, buf, buf)           # in place
    assert_same(to_host(buf), oracle_lib.ecb_encrypt(key, x), "in-place encrypt")
    aes.aes_ecb_decrypt(ks.rk_dec, ks.nr, buf, buf)
    assert_same(to_host(buf), x, "in-place decrypt")
    out = torch.zeros_like(buf)
    aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, buf, out, nblocks=100)  # prefix only, rest untouched
    o = to_host(out)
    assert_same(o[:1600], oracle_lib.ecb_encrypt(key, x[:1600]), "prefix")
    assert not o[1600:].any()


def test_empty_and_rejected_inputs():
    torch = cuda()
    ks = aes.aes_expand_key(inputs.random_key(1, 128))
    x = torch.zeros(64, dtype=torch.uint8, device="cuda")
    aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, x, x, nblocks=0)
    with pytest.raises(aes.AesError) as e:
        aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, x[4:36], x[32:64])
    assert e.value.code == aes.AES_EALIGN
    with pytest.raises(aes.AesError) as e:
        aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, x[:48], x[16:64])
    assert e.value.code == aes.AES_EINVAL
    with pytest.raises(ValueError):
        aes.aes_ecb_decrypt(ks.rk_dec, ks.nr, x, x, nblocks=-1)
    with pytest.raises(ValueError):
        aes.aes_cbc_decrypt(ks.rk_dec, ks.nr, bytes(16), x[:32], x[32:], nblocks=-2)
    torch.cuda.synchronize()


def window_offsets(nbytes: int, seed: int):
    g = inputs.rng(50, seed)
    offs = {0, nbytes - MiB}
    while len(offs) < 4:
        offs.add(int(g.integers(0, (nbytes - MiB) // 16)) * 16)
    return sorted(offs)


@pytest.mark.parametrize("keybits", [128, 192, 256])
@pytest.mark.parametrize("size", [1 * MiB, 16 * MiB, 256 * MiB, 1024 * MiB, 4096 * MiB],
                         ids=["1MiB", "16MiB", "256MiB", "1GiB", "4GiB"])
def test_bulk_sweep(oracle_lib, keybits, size):
    """Plain bulk path: every key size over 1 MiB ... 4 GiB (4 GiB = 2^32
    bytes, so byte offsets need 64 bits)."""
    torch = cuda()
    key = inputs.random_key(60 + keybits, keybits)
    ks = aes.aes_expand_key(key)
    if size <= 16 * MiB:
        x = inputs.random_bytes(61 + size // MiB, size)
        xd = to_dev(x)
        c = gpu_enc(ks, xd)
        assert_same(to_host(c), oracle_lib.ecb_encrypt(key, x), "enc")
        assert_same(to_host(gpu_dec(ks, xd)), oracle_lib.ecb_decrypt(key, x), "dec")
        return
    xd = inputs.device_random_bytes(62 + size // MiB + keybits, size)
    c = gpu_enc(ks, xd)
    p = gpu_dec(ks, xd)
    torch.cuda.synchronize()
    for off in window_offsets(size, keybits):
        xw = xd[off:off + MiB].cpu().numpy()
        assert_same(c[off:off + MiB].cpu().numpy(), oracle_lib.ecb_encrypt(key, xw), "enc window @%d" % off)
        assert_same(p[off:off + MiB].cpu().numpy(), oracle_lib.ecb_decrypt(key, xw), "dec window @%d" % off)
    del p
    r = gpu_dec(ks, c)
    torch.cuda.synchronize()
    assert torch.equal(r, xd), "device round trip"
    assert not torch.equal(c[:MiB], xd[:MiB])
    del r, c, xd
    torch.cuda.empty_cache()
