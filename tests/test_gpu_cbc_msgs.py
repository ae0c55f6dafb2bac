"""GPU parity of CBC encryption across independent messages (section 3.1.2,
eq 2 read with the block cipher; one chain per message) against the CPU
oracle's sequential CBC encryption, bit-exact: ragged message sets (empty
and one-block messages, lengths that are not a multiple of a lane's load
group, gaps and a shuffled output order) for every key size, every kernel
variant with a small grid so waves take several wave units, both kernels
on every table placement for 192- and 256-bit keys, in-place messages, a
message continued across two launches, messages the kernel must skip, and
the 1 GiB set of 2^18 four-KiB messages on sampled messages; and the same
for CBC decryption of message sets against the oracle's CBC decryption
(every variant, in place with skipped records, 2^18 x 4 KiB on samples)."""
import numpy as np
import pytest

from paper_1902_05234_amd import aes, inputs
from tests.gpu_util import cuda, first_mismatch, to_dev, to_host

pytestmark = pytest.mark.gpu

SENTINEL = 0xA5


def records(ms: inputs.CbcMessageSet) -> np.ndarray:
    r = np.zeros(len(ms), dtype=aes.CBC_MSG_DTYPE)
    r["in_block"], r["out_block"], r["nblocks"], r["iv"] = ms.in_block, ms.out_block, ms.nblocks, ms.iv
    return r


def run(ks, recs, src_dev, out_dev, variant=None, rejected=None):
    torch = cuda()
    msgs = to_dev(recs.view(np.uint8))
    aes.aes_cbc_encrypt_msgs(ks.rk_enc, ks.nr, msgs, recs.size, src_dev, out_dev, rejected_dev=rejected,
                             variant=variant)
    torch.cuda.synchronize()


def check_messages(oracle_lib, key, recs, src: np.ndarray, got: np.ndarray, what: str, idx=None):
    for m in (range(recs.size) if idx is None else idx):
        r = recs[m]
        a, n, o = int(r["in_block"]) * 16, int(r["nblocks"]) * 16, int(r["out_block"]) * 16
        want = oracle_lib.cbc_encrypt(key, r["iv"].tobytes(), src[a:a + n]) if n else np.zeros(0, np.uint8)
        i = first_mismatch(got[o:o + n], want)
        assert i is None, "%s: message %d (%d blocks) first differing byte %d" % (what, m, n // 16, i)


def untouched_outside(recs, got: np.ndarray, what: str):
    covered = np.zeros(got.size, dtype=bool)
    for r in recs:
        o, n = int(r["out_block"]) * 16, int(r["nblocks"]) * 16
        covered[o:o + n] = True
    assert (got[~covered] == SENTINEL).all(), "%s: bytes outside every output range were written" % what


@pytest.mark.parametrize("keybits", [128, 192, 256])
def test_ragged_message_set_matches_oracle(oracle_lib, keybits):
    torch = cuda()
    ms = inputs.cbc_message_set(800 + keybits, 1500, 200)
    key = inputs.random_key(801, keybits)
    ks = aes.aes_expand_key(key)
    src = inputs.random_bytes(802 + keybits, 16 * ms.in_blocks)
    out = torch.full((16 * ms.out_blocks,), SENTINEL, dtype=torch.uint8, device="cuda")
    recs = records(ms)
    rej = torch.zeros(1, dtype=torch.int32, device="cuda")
    run(ks, recs, to_dev(src), out, rejected=rej)
    got = to_host(out)
    assert int(rej.item()) == 0
    check_messages(oracle_lib, key, recs, src, got, "%d-bit" % keybits)
    untouched_outside(recs, got, "%d-bit" % keybits)


VARIANTS = [aes.Variant(bpt=b, wg=w, placement=p, grid=3) for p in (0, 1, 2) for b in (aes.AES_BPT_COLUMN, 1, 2, 4, 8)
            for w in (64, 1024)]


@pytest.mark.parametrize("variant", VARIANTS, ids=lambda v: "p%d_g%d_w%d" % (v.placement, v.bpt, v.wg))
def test_every_variant_matches_oracle(oracle_lib, variant):
    torch = cuda()
    # 700 messages = 11 wave units: three workgroups of one wave each walk
    # several units, and with 1024-thread groups some waves have none
    ms = inputs.cbc_message_set(810, 700, 37)
    key = inputs.random_key(811, 128)
    ks = aes.aes_expand_key(key)
    src = inputs.random_bytes(812, 16 * ms.in_blocks)
    out = torch.full((16 * ms.out_blocks,), SENTINEL, dtype=torch.uint8, device="cuda")
    recs = records(ms)
    run(ks, recs, to_dev(src), out, variant=variant)
    got = to_host(out)
    check_messages(oracle_lib, key, recs, src, got, str(variant))
    untouched_outside(recs, got, str(variant))


@pytest.mark.parametrize("keybits", [192, 256])
@pytest.mark.parametrize("placement", [0, 1, 2])
@pytest.mark.parametrize("bpt", [aes.AES_BPT_COLUMN, 8], ids=["quads", "lanes"])
def test_both_kernels_every_placement_for_longer_keys(oracle_lib, keybits, placement, bpt):
    # the 2-table placement takes inner round keys turned right by 8 bits,
    # which the longer schedules exercise over more rounds
    torch = cuda()
    ms = inputs.cbc_message_set(880 + keybits + placement, 300, 40)
    key = inputs.random_key(881 + placement, keybits)
    ks = aes.aes_expand_key(key)
    src = inputs.random_bytes(882 + keybits, 16 * ms.in_blocks)
    out = torch.full((16 * ms.out_blocks,), SENTINEL, dtype=torch.uint8, device="cuda")
    recs = records(ms)
    v = aes.Variant(bpt=bpt, wg=256, placement=placement)
    run(ks, recs, to_dev(src), out, variant=v)
    got = to_host(out)
    check_messages(oracle_lib, key, recs, src, got, "%d-bit %s" % (keybits, v))
    untouched_outside(recs, got, "%d-bit %s" % (keybits, v))


def test_in_place_messages(oracle_lib):
    ms = inputs.cbc_message_set(820, 900, 50)
    key = inputs.random_key(821, 256)
    ks = aes.aes_expand_key(key)
    src = inputs.random_bytes(822, 16 * ms.in_blocks)
    recs = records(ms)
    recs["out_block"] = recs["in_block"]
    buf = to_dev(src)
    run(ks, recs, buf, buf)
    check_messages(oracle_lib, key, recs, src, to_host(buf), "in place")


def test_message_continued_across_launches(oracle_lib):
    torch = cuda()
    key = inputs.random_key(830, 192)
    ks = aes.aes_expand_key(key)
    n = 1000
    src = inputs.random_bytes(831, 16 * n)
    iv = inputs.random_bytes(832, 16)
    want = oracle_lib.cbc_encrypt(key, iv.tobytes(), src)
    out = torch.zeros(16 * n, dtype=torch.uint8, device="cuda")
    sd = to_dev(src)
    cut = 333
    first = np.zeros(1, dtype=aes.CBC_MSG_DTYPE)
    first["nblocks"], first["iv"] = cut, iv
    run(ks, first, sd, out)
    second = np.zeros(1, dtype=aes.CBC_MSG_DTYPE)
    second["in_block"] = second["out_block"] = cut
    second["nblocks"] = n - cut
    second["iv"] = to_host(out)[16 * cut - 16:16 * cut]  # the last ciphertext block so far
    run(ks, second, sd, out)
    assert first_mismatch(to_host(out), want) is None


def test_messages_outside_their_arena_are_skipped_and_counted(oracle_lib):
    torch = cuda()
    ms = inputs.cbc_message_set(840, 300, 20)
    key = inputs.random_key(841, 128)
    ks = aes.aes_expand_key(key)
    src = inputs.random_bytes(842, 16 * ms.in_blocks)
    recs = records(ms)
    good = np.ones(recs.size, dtype=bool)
    bad = {
        5: dict(in_block=ms.in_blocks),                           # starts at the end of the input arena
        17: dict(in_block=ms.in_blocks - 2, nblocks=3),           # runs past it
        29: dict(out_block=ms.out_blocks - 1, nblocks=2),         # runs past the output arena
        41: dict(in_block=2**64 - 2, nblocks=4),                  # a sum that would wrap
        53: dict(nblocks=2**63),
        65: dict(reserved=1),
        130: dict(out_block=2**64 - 1),
    }
    for m, fields in bad.items():
        for f, v in fields.items():
            recs[f][m] = v
        good[m] = False
    out = torch.full((16 * ms.out_blocks,), SENTINEL, dtype=torch.uint8, device="cuda")
    rej = torch.zeros(1, dtype=torch.int32, device="cuda")
    run(ks, recs, to_dev(src), out, rejected=rej)
    got = to_host(out)
    assert int(rej.item()) == len(bad)
    check_messages(oracle_lib, key, recs, src, got, "skips", idx=np.nonzero(good)[0])
    untouched_outside(recs[good], got, "skips")


def test_ciphertext_decrypts_with_the_gpu_cbc_decryption():
    torch = cuda()
    ms = inputs.cbc_equal_messages(850, 640, 24)
    key = inputs.random_key(851, 128)
    ks = aes.aes_expand_key(key)
    src = inputs.random_bytes(852, 16 * ms.in_blocks)
    out = torch.empty(16 * ms.out_blocks, dtype=torch.uint8, device="cuda")
    recs = records(ms)
    run(ks, recs, to_dev(src), out)
    back = torch.empty_like(out)
    for m in range(0, recs.size, 37):
        a, n = int(recs[m]["out_block"]) * 16, 24 * 16
        aes.aes_cbc_decrypt(ks.rk_dec, ks.nr, recs[m]["iv"].tobytes(), out[a:a + n], back[a:a + n])
        torch.cuda.synchronize()
        assert first_mismatch(to_host(back[a:a + n]), src[a:a + n]) is None, m


def test_empty_list_is_a_no_op():
    torch = cuda()
    ks = aes.aes_expand_key(inputs.random_key(860, 128))
    out = torch.full((64,), SENTINEL, dtype=torch.uint8, device="cuda")
    msgs = torch.zeros(48, dtype=torch.uint8, device="cuda")
    aes.aes_cbc_encrypt_msgs(ks.rk_enc, ks.nr, msgs, 0, torch.zeros(64, dtype=torch.uint8, device="cuda"), out)
    assert (to_host(out) == SENTINEL).all()


# ------------------------------------------------------------ decryption
def run_dec(ks, recs, src_dev, out_dev, variant=None, rejected=None):
    torch = cuda()
    msgs = to_dev(recs.view(np.uint8))
    aes.aes_cbc_decrypt_msgs(ks.rk_dec, ks.nr, msgs, recs.size, src_dev, out_dev, rejected_dev=rejected,
                             variant=variant)
    torch.cuda.synchronize()


def check_decrypted(oracle_lib, key, recs, src: np.ndarray, got: np.ndarray, what: str, idx=None):
    for m in (range(recs.size) if idx is None else idx):
        r = recs[m]
        a, n, o = int(r["in_block"]) * 16, int(r["nblocks"]) * 16, int(r["out_block"]) * 16
        want = oracle_lib.cbc_decrypt(key, r["iv"].tobytes(), src[a:a + n]) if n else np.zeros(0, np.uint8)
        i = first_mismatch(got[o:o + n], want)
        assert i is None, "%s: message %d (%d blocks) first differing byte %d" % (what, m, n // 16, i)


@pytest.mark.parametrize("keybits", [128, 192, 256])
def test_decrypt_ragged_message_set_matches_oracle(oracle_lib, keybits):
    # random bytes as ciphertext: the oracle's CBC decryption of each message
    torch = cuda()
    ms = inputs.cbc_message_set(890 + keybits, 1500, 200)
    key = inputs.random_key(891, keybits)
    ks = aes.aes_expand_key(key)
    src = inputs.random_bytes(892 + keybits, 16 * ms.in_blocks)
    out = torch.full((16 * ms.out_blocks,), SENTINEL, dtype=torch.uint8, device="cuda")
    recs = records(ms)
    rej = torch.zeros(1, dtype=torch.int32, device="cuda")
    run_dec(ks, recs, to_dev(src), out, rejected=rej)
    got = to_host(out)
    assert int(rej.item()) == 0
    check_decrypted(oracle_lib, key, recs, src, got, "%d-bit" % keybits)
    untouched_outside(recs, got, "%d-bit" % keybits)


DEC_VARIANTS = [aes.Variant(bpt=b, wg=w, placement=p, grid=3) for p in (0, 1, 2)
                for b in (1, 2, 4, aes.AES_BPT_WAVE_MSG + 1, aes.AES_BPT_WAVE_MSG + 2) for w in (64, 1024)]


@pytest.mark.parametrize("variant", DEC_VARIANTS, ids=lambda v: "p%d_g%d_w%d" % (v.placement, v.bpt, v.wg))
def test_decrypt_every_variant_matches_oracle(oracle_lib, variant):
    torch = cuda()
    ms = inputs.cbc_message_set(893, 700, 37)
    key = inputs.random_key(894, 256)
    ks = aes.aes_expand_key(key)
    src = inputs.random_bytes(895, 16 * ms.in_blocks)
    out = torch.full((16 * ms.out_blocks,), SENTINEL, dtype=torch.uint8, device="cuda")
    recs = records(ms)
    run_dec(ks, recs, to_dev(src), out, variant=variant)
    got = to_host(out)
    check_decrypted(oracle_lib, key, recs, src, got, str(variant))
    untouched_outside(recs, got, str(variant))


@pytest.mark.parametrize("keybits", [128, 256])
def test_decrypt_long_messages_one_wave_each(oracle_lib, keybits):
    # messages averaging well over 64 blocks: the default takes one wave per
    # message; lengths straddle the 64- and 128-block units, plus empty ones
    torch = cuda()
    ms = inputs.cbc_message_set(905 + keybits, 300, 700)
    key = inputs.random_key(906, keybits)
    ks = aes.aes_expand_key(key)
    src = inputs.random_bytes(907 + keybits, 16 * ms.in_blocks)
    out = torch.full((16 * ms.out_blocks,), SENTINEL, dtype=torch.uint8, device="cuda")
    recs = records(ms)
    # shorten six long messages to the unit boundaries (ranges stay disjoint)
    longs = np.nonzero(recs["nblocks"] >= 129)[0][:6]
    recs["nblocks"][longs] = [63, 64, 65, 127, 128, 129]
    assert ms.in_blocks // recs.size >= 64
    run_dec(ks, recs, to_dev(src), out)
    got = to_host(out)
    check_decrypted(oracle_lib, key, recs, src, got, "%d-bit long" % keybits)
    untouched_outside(recs, got, "%d-bit long" % keybits)
    buf = to_dev(src)                                      # in place, one wave per message
    inplace = recs.copy()
    inplace["out_block"] = inplace["in_block"]
    run_dec(ks, inplace, buf, buf, variant=aes.Variant(bpt=aes.AES_BPT_WAVE_MSG + 2, wg=256))
    check_decrypted(oracle_lib, key, inplace, src, to_host(buf), "%d-bit long in place" % keybits)


def test_decrypt_round_trip_in_place_and_skips(oracle_lib):
    # encrypt a ragged set with the GPU, decrypt it in place, and skip bad records
    torch = cuda()
    ms = inputs.cbc_message_set(896, 900, 60)
    key = inputs.random_key(897, 192)
    ks = aes.aes_expand_key(key)
    plain = inputs.random_bytes(898, 16 * ms.in_blocks)
    recs = records(ms)
    recs["out_block"] = recs["in_block"]
    buf = to_dev(plain)
    run(ks, recs, buf, buf)                               # in-place encryption
    cipher = to_host(buf)
    check_messages(oracle_lib, key, recs, plain, cipher, "encrypt in place")
    bad = recs.copy()
    bad["in_block"][7] = ms.in_blocks
    bad["reserved"][11] = 5
    rej = torch.zeros(1, dtype=torch.int32, device="cuda")
    run_dec(ks, bad, buf, buf, rejected=rej)              # in-place decryption
    assert int(rej.item()) == 2
    got = to_host(buf)
    for m in range(recs.size):
        a, n = int(recs[m]["in_block"]) * 16, int(recs[m]["nblocks"]) * 16
        want = cipher[a:a + n] if m in (7, 11) else plain[a:a + n]
        assert first_mismatch(got[a:a + n], want) is None, m


def test_decrypt_one_gib_of_four_kib_messages_on_samples(oracle_lib):
    torch = cuda()
    n, blocks = 1 << 18, 256
    ms = inputs.cbc_equal_messages(899, n, blocks)
    key = inputs.random_key(899, 128)
    ks = aes.aes_expand_key(key)
    src = inputs.device_random_bytes(899, 16 * ms.in_blocks)
    out = torch.empty_like(src)
    recs = records(ms)
    run_dec(ks, recs, src, out)
    pick = np.unique(np.concatenate([[0, n - 1], inputs.rng(899).integers(0, n, size=64)]))
    for m in pick:
        a = int(m) * blocks * 16
        s = to_host(src[a:a + blocks * 16])
        want = oracle_lib.cbc_decrypt(key, recs[m]["iv"].tobytes(), s)
        assert first_mismatch(to_host(out[a:a + blocks * 16]), want) is None, int(m)


def test_helpers_take_host_records(oracle_lib):
    # cbc_encrypt_msgs / cbc_decrypt_msgs upload a host record array themselves
    cuda()
    ms = inputs.cbc_message_set(910, 400, 90)
    key = inputs.random_key(911, 128)
    ks = aes.expand_key(key)
    src = inputs.random_bytes(912, 16 * max(ms.in_blocks, ms.out_blocks))
    recs = records(ms)
    recs["out_block"] = recs["in_block"]
    x = to_dev(src)
    c = aes.cbc_encrypt_msgs(ks, recs, x)
    cipher = to_host(c)
    check_messages(oracle_lib, key, recs, src, cipher, "helper encrypt")
    back = to_host(aes.cbc_decrypt_msgs(ks, recs, c))
    for m in range(recs.size):
        a, n = int(recs[m]["in_block"]) * 16, int(recs[m]["nblocks"]) * 16
        assert first_mismatch(back[a:a + n], src[a:a + n]) is None, m


def test_one_gib_of_four_kib_messages_on_samples(oracle_lib):
    """The benchmark's set: 2^18 messages of 256 blocks, back to back, in the
    default launch; 64 random messages plus the first and last are compared
    with the oracle."""
    torch = cuda()
    n, blocks = 1 << 18, 256
    ms = inputs.cbc_equal_messages(870, n, blocks)
    key = inputs.random_key(871, 128)
    ks = aes.aes_expand_key(key)
    src = inputs.device_random_bytes(872, 16 * ms.in_blocks)
    out = torch.empty_like(src)
    recs = records(ms)
    rej = torch.zeros(1, dtype=torch.int32, device="cuda")
    run(ks, recs, src, out, rejected=rej)
    assert int(rej.item()) == 0
    pick = np.unique(np.concatenate([[0, n - 1], inputs.rng(873).integers(0, n, size=64)]))
    for m in pick:
        a = int(m) * blocks * 16
        s = to_host(src[a:a + blocks * 16])
        want = oracle_lib.cbc_encrypt(key, recs[m]["iv"].tobytes(), s)
        assert first_mismatch(to_host(out[a:a + blocks * 16]), want) is None, int(m)
