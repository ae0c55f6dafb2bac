"""GPU parity of CBC decryption (section 3.1.2, eq 2 read with the block
cipher) against the CPU oracle, bit-exact: block counts around the wave and
workgroup tiles for every key size, a message decrypted in pieces (each
piece's initialisation vector is the previous piece's last ciphertext
block), every kernel variant, 1 GiB on oracle windows, and the rejected
in-place call."""
import numpy as np
import pytest

from paper_1902_05234_amd import aes, inputs
from tests.gpu_util import cuda, first_mismatch, to_dev, to_host

pytestmark = pytest.mark.gpu

MiB = 1 << 20


def assert_same(got: np.ndarray, want: np.ndarray, what: str):
    i = first_mismatch(got, want)
    assert i is None, "%s: first differing byte %d (block %d)" % (what, i, i // 16)


def gpu_cbc_dec(ks, iv, cd):
    out = cuda().empty_like(cd)
    aes.aes_cbc_decrypt(ks.rk_dec, ks.nr, iv, cd, out)
    return out


@pytest.mark.parametrize("keybits", [128, 192, 256])
@pytest.mark.parametrize("nblocks", [1, 2, 63, 64, 65, 1023, 1025, 4097, 65536 + 17])
def test_cbc_decrypt_sizes(oracle_lib, keybits, nblocks):
    key = inputs.random_key(700 + nblocks % 83, keybits)
    iv = inputs.random_bytes(701 + keybits, 16).tobytes()
    x = inputs.random_bytes(702 + nblocks, 16 * nblocks)
    c = oracle_lib.cbc_encrypt(key, iv, x)
    ks = aes.aes_expand_key(key)
    got = to_host(gpu_cbc_dec(ks, iv, to_dev(c)))
    assert_same(got, x, "cbc dec %d-bit n=%d" % (keybits, nblocks))


def test_cbc_decrypt_random_ciphertext_matches_oracle(oracle_lib):
    key = inputs.random_key(710, 256)
    iv = inputs.random_bytes(711, 16).tobytes()
    c = inputs.random_bytes(712, 16 * 70001)
    ks = aes.aes_expand_key(key)
    assert_same(to_host(gpu_cbc_dec(ks, iv, to_dev(c))), oracle_lib.cbc_decrypt(key, iv, c), "random ciphertext")


def test_cbc_decrypt_helper_allocates_output(oracle_lib):
    key = inputs.random_key(713, 192)
    iv = inputs.random_bytes(714, 16).tobytes()
    x = inputs.random_bytes(715, 16 * 3001)
    c = oracle_lib.cbc_encrypt(key, iv, x)
    ks = aes.aes_expand_key(key)
    assert_same(to_host(aes.cbc_decrypt(ks, iv, to_dev(c))), x, "cbc_decrypt helper")


def test_cbc_decrypt_in_pieces_and_rejects_in_place(oracle_lib):
    torch = cuda()
    key = inputs.random_key(720, 128)
    iv = inputs.random_bytes(721, 16).tobytes()
    x = inputs.random_bytes(722, 16 * 9000)
    c = oracle_lib.cbc_encrypt(key, iv, x)
    ks = aes.aes_expand_key(key)
    cd = to_dev(c)
    out = torch.empty_like(cd)
    cuts = [0, 16 * 1, 16 * 4000, c.size]
    for a, b in zip(cuts[:-1], cuts[1:]):
        piv = iv if a == 0 else c[a - 16:a].tobytes()
        aes.aes_cbc_decrypt(ks.rk_dec, ks.nr, piv, cd[a:b], out[a:b])
    assert_same(to_host(out), x, "pieces")
    with pytest.raises(aes.AesError) as e:
        aes.aes_cbc_decrypt(ks.rk_dec, ks.nr, iv, cd, cd)
    assert e.value.code == aes.AES_EINVAL


VARIANTS = [aes.Variant(bpt=b, wg=w, placement=p) for p in (0, 1, 2) for b in (1, 2, 4) for w in (64, 1024)]


@pytest.mark.parametrize("variant", VARIANTS, ids=lambda v: "p%d_b%d_w%d" % (v.placement, v.bpt, v.wg))
def test_cbc_every_variant(oracle_lib, variant):
    torch = cuda()
    nblocks = 2 * 4096 + 77
    for keybits in (128, 192, 256):
        key = inputs.random_key(730, keybits)
        iv = inputs.random_bytes(731, 16).tobytes()
        x = inputs.random_bytes(732, 16 * nblocks)
        c = oracle_lib.cbc_encrypt(key, iv, x)
        ks = aes.aes_expand_key(key)
        cd = to_dev(c)
        out = torch.empty_like(cd)
        aes.aes_cbc_decrypt_variant(ks.rk_dec, ks.nr, iv, cd, out, variant)
        assert_same(to_host(out), x, "%s %d-bit" % (variant, keybits))


def test_cbc_1gib_windows(oracle_lib):
    """1 GiB of random ciphertext, AES-128: four 1 MiB windows against the
    oracle, each started with the ciphertext block before the window."""
    torch = cuda()
    n = 1 << 30
    key = inputs.random_key(740, 128)
    iv = inputs.random_bytes(741, 16).tobytes()
    ks = aes.aes_expand_key(key)
    cd = inputs.device_random_bytes(742, n)
    p = gpu_cbc_dec(ks, iv, cd)
    rng = inputs.rng(743)
    starts = [0, n - MiB] + [int(s) * 16 for s in rng.integers(1, (n - MiB) // 16, size=2)]
    for s in starts:
        cs = to_host(cd[s:s + MiB])
        piv = iv if s == 0 else to_host(cd[s - 16:s]).tobytes()
        assert_same(to_host(p[s:s + MiB]), oracle_lib.cbc_decrypt(key, piv, cs), "window at %d" % s)
    del p, cd
    torch.cuda.empty_cache()
