"""GPU parity of the bitsliced placement (AES_PLACEMENT_BITSLICED: no
tables, 32 blocks per lane as 128 bit slices, the S-box as a Boolean
circuit) against the CPU oracle, bit-exact: block counts around the lane
(32 blocks), wave (2,048) and workgroup tiles with ragged tails, every key
size and both directions, every allowed workgroup size, in place, a 256 MiB
buffer on oracle windows, and the rejected combinations."""
import numpy as np
import pytest

from paper_1902_05234_amd import aes, inputs
from tests.gpu_util import cuda, first_mismatch, to_dev, to_host

pytestmark = pytest.mark.gpu

MiB = 1 << 20
BS = aes.AES_PLACEMENT_BITSLICED


def assert_same(got, want, what):
    i = first_mismatch(got, want)
    assert i is None, "%s: first differing byte %d (block %d)" % (what, i, i // 16)


def run(ks, dec, xd, wg=256):
    out = cuda().empty_like(xd)
    aes.aes_ecb_crypt_variant(ks.rk_dec if dec else ks.rk_enc, ks.nr, dec, xd, out, aes.Variant(bpt=1, wg=wg, placement=BS))
    return out


@pytest.mark.parametrize("keybits", [128, 192, 256])
@pytest.mark.parametrize("nblocks", [1, 31, 33, 63, 64, 2047, 2048, 2049, 4097, 16384 + 1, 65536 + 17])
def test_bitslice_sizes(oracle_lib, keybits, nblocks):
    key = inputs.random_key(900 + nblocks % 71, keybits)
    x = inputs.random_bytes(901 + nblocks, 16 * nblocks)
    ks = aes.aes_expand_key(key)
    xd = to_dev(x)
    assert_same(to_host(run(ks, False, xd)), oracle_lib.ecb_encrypt(key, x), "enc %d-bit n=%d" % (keybits, nblocks))
    assert_same(to_host(run(ks, True, xd)), oracle_lib.ecb_decrypt(key, x), "dec %d-bit n=%d" % (keybits, nblocks))


@pytest.mark.parametrize("wg", [64, 128, 256])
def test_bitslice_workgroup_sizes_and_in_place(oracle_lib, wg):
    key = inputs.random_key(910, 128)
    ks = aes.aes_expand_key(key)
    x = inputs.random_bytes(911, 16 * 100003)
    buf = to_dev(x)
    v = aes.Variant(bpt=1, wg=wg, placement=BS)
    aes.aes_ecb_crypt_variant(ks.rk_enc, ks.nr, False, buf, buf, v)
    assert_same(to_host(buf), oracle_lib.ecb_encrypt(key, x), "enc in place wg=%d" % wg)
    aes.aes_ecb_crypt_variant(ks.rk_dec, ks.nr, True, buf, buf, v)
    assert_same(to_host(buf), x, "dec in place wg=%d" % wg)


def test_bitslice_256mib_windows(oracle_lib):
    torch = cuda()
    n = 256 * MiB
    key = inputs.random_key(920, 256)
    ks = aes.aes_expand_key(key)
    xd = inputs.device_random_bytes(921, n)
    c = run(ks, False, xd)
    rng = inputs.rng(922)
    for s in [0, n - MiB] + [int(v) * 16 for v in rng.integers(0, (n - MiB) // 16, size=2)]:
        assert_same(to_host(c[s:s + MiB]), oracle_lib.ecb_encrypt(key, to_host(xd[s:s + MiB])), "window at %d" % s)
    assert torch.equal(run(ks, True, c), xd)
    del c, xd
    torch.cuda.empty_cache()


def test_bitslice_rejected_combinations():
    torch = cuda()
    ks = aes.aes_expand_key(inputs.random_key(930, 128))
    x = torch.zeros(4096, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(aes.AesError) as e:
        aes.aes_ecb_crypt_variant(ks.rk_enc, ks.nr, False, x, y, aes.Variant(bpt=1, wg=512, placement=BS))
    assert e.value.code == aes.AES_EINVAL
    with pytest.raises(aes.AesError):
        aes.aes_ctr_crypt_variant(ks.rk_enc, ks.nr, bytes(16), 0, x, y, aes.Variant(bpt=1, wg=256, placement=BS))
    with pytest.raises(aes.AesError):
        aes.aes_cbc_decrypt_variant(ks.rk_dec, ks.nr, bytes(16), x, y, aes.Variant(bpt=1, wg=256, placement=BS))
