"""GPU parity of the batched path: every message of a mixed batch (own key,
key size and direction) equals the CPU oracle and the plain kernel run on
that message alone, bit-exact; graph replays equal the eager launch; bad
work items are skipped and counted without touching other messages."""
import numpy as np
import pytest

from paper_1902_05234_amd import aes, batch, inputs
from tests.gpu_util import cuda, first_mismatch

pytestmark = pytest.mark.gpu


def build(seed, n, hi_bytes, chunk, cfg=None):
    torch = cuda()
    mix = inputs.message_mix(seed, n, hi_bytes=hi_bytes)
    keys = [inputs.random_key(int(s), int(b)) for s, b in zip(mix.key_seed, mix.keybits)]
    kt = batch.key_table(keys)
    total = mix.total_blocks
    x = inputs.random_bytes(seed, 16 * total)
    in_arena = torch.from_numpy(x).cuda()
    out_arena = torch.zeros_like(in_arena)
    msgs = batch.messages_from_mix(mix)
    b = batch.prepare(msgs, kt, in_arena, out_arena, chunk_blocks=chunk, cfg=cfg)
    return mix, keys, x, b


def check_against_oracle(oracle_lib, mix, keys, x, out):
    for i in range(len(mix)):
        lo, n = int(mix.offset[i]) * 16, int(mix.nblocks[i]) * 16
        src = x[lo:lo + n]
        want = oracle_lib.ecb_decrypt(keys[i], src) if mix.decrypt[i] else oracle_lib.ecb_encrypt(keys[i], src)
        j = first_mismatch(out[lo:lo + n], want)
        assert j is None, "message %d (%d-bit, dec=%s, %d blocks): byte %d differs" % (
            i, mix.keybits[i], bool(mix.decrypt[i]), mix.nblocks[i], j)


@pytest.mark.parametrize("chunk", [64, 100, 1024, 4096])
@pytest.mark.parametrize("bpt", [1, 2, 4])
def test_mixed_batch_matches_oracle(oracle_lib, chunk, bpt):
    torch = cuda()
    mix, keys, x, b = build(7 + chunk + bpt, 300, 256 << 10, chunk, aes.BatchConfig(bpt=bpt))
    b.launch()
    torch.cuda.synchronize()
    assert b.rejected_items() == 0
    check_against_oracle(oracle_lib, mix, keys, x, b.out_arena.cpu().numpy())
    assert not b.counters_dev[:3].any(), "claim counters must be reset by the last workgroup"


@pytest.mark.parametrize("placement", [aes.AES_PLACEMENT_TTABLE4, aes.AES_PLACEMENT_TTABLE2,
                                       aes.AES_PLACEMENT_TTABLE1])
@pytest.mark.parametrize("wg,bpt", [(256, 1), (512, 2), (1024, 4), (1024, 1)])
def test_every_batch_variant_matches_oracle(oracle_lib, placement, wg, bpt):
    """Each table placement and workgroup size of the batch kernel (the
    autotuner's axes) gives the oracle's output on a mixed batch, with items
    of a ragged size (100 blocks) and a grid small enough that workgroups
    switch direction."""
    torch = cuda()
    cfg = aes.BatchConfig(bpt=bpt, wg=wg, placement=placement, grid=5)
    mix, keys, x, b = build(31 + placement * 7 + wg + bpt, 200, 128 << 10, 100, cfg)
    b.launch()
    torch.cuda.synchronize()
    assert b.rejected_items() == 0
    check_against_oracle(oracle_lib, mix, keys, x, b.out_arena.cpu().numpy())
    assert not b.counters_dev[:3].any(), "claim counters must be reset by the last workgroup"
    # a second launch (persistent grid, as the library sizes it) gives the same output
    first = b.out_arena.clone()
    b2 = batch.prepare(b.msgs, b.key_table_dev, b.in_arena, b.out_arena, chunk_blocks=100,
                       cfg=aes.BatchConfig(bpt=bpt, wg=wg, placement=placement))
    b.out_arena.zero_()
    b2.launch()
    torch.cuda.synchronize()
    assert torch.equal(b.out_arena, first)


def test_batch_equals_plain_kernel_per_message():
    torch = cuda()
    mix, keys, x, b = build(21, 500, 1 << 20, 1024)
    b.launch()
    ref = torch.zeros_like(b.out_arena)
    scheds = [aes.aes_expand_key(k) for k in keys]
    batch.run_per_message(b.msgs, scheds, b.in_arena, ref)
    torch.cuda.synchronize()
    assert torch.equal(ref, b.out_arena)


def test_graph_replay_equals_eager():
    torch = cuda()
    mix, keys, x, b = build(22, 200, 64 << 10, 256)
    b.launch()
    torch.cuda.synchronize()
    eager = b.out_arena.clone()
    b.capture()
    for r in range(3):
        b.out_arena.zero_()
        torch.cuda.synchronize()
        b.replay()
        torch.cuda.synchronize()
        assert torch.equal(b.out_arena, eager), "replay %d differs from the eager launch" % r
        # eager work between replays
        ks = aes.aes_expand_key(keys[0])
        aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, b.in_arena[:1024], torch.empty(1024, dtype=torch.uint8, device="cuda"))
        torch.cuda.synchronize()


def test_bad_items_are_skipped_and_counted(oracle_lib):
    torch = cuda()
    key = inputs.random_key(5, 128)
    kt = batch.key_table([key])
    x = inputs.random_bytes(5, 16 * 3000)
    in_arena = torch.from_numpy(x).cuda()
    out_arena = torch.zeros_like(in_arena)
    items = np.zeros(4, dtype=aes.ITEM_DTYPE)
    items[0] = (0, 0, 1000, 0)          # good
    items[1] = (1000, 1000, 1000, 5)    # key slot out of range
    items[2] = (2500, 2500, 1000, 0)    # runs past the arenas
    items[3] = (2000, 2000, 1000, 0)    # good
    items_dev = torch.from_numpy(items.view(np.uint8).copy()).cuda()
    counters = torch.zeros(4, dtype=torch.int32, device="cuda")
    aes.aes_ecb_batch(items_dev, 4, 0, kt, in_arena, out_arena, counters)
    torch.cuda.synchronize()
    assert int(counters[3].item()) == 2
    out = out_arena.cpu().numpy()
    ref = oracle_lib.ecb_encrypt(key, x)
    assert np.array_equal(out[:16000], ref[:16000])
    assert np.array_equal(out[32000:48000], ref[32000:48000])
    assert not out[16000:32000].any()


def test_largest_item_runs_and_one_block_more_is_rejected(oracle_lib):
    """An item of AES_MAX_ITEM_BLOCKS blocks (256 MiB, walked by one wave) is
    encrypted; an item one block larger is skipped and counted."""
    torch = cuda()
    n = aes.AES_MAX_ITEM_BLOCKS
    key = inputs.random_key(7, 128)
    kt = batch.key_table([key])
    in_arena = inputs.device_random_bytes(7, 16 * (n + 1))
    out_arena = torch.zeros_like(in_arena)
    items = np.zeros(2, dtype=aes.ITEM_DTYPE)
    items[0] = (0, 0, n, 0)      # blocks [0, n): at the limit
    items[1] = (0, 0, n + 1, 0)  # blocks [0, n]: over it
    items_dev = torch.from_numpy(items.view(np.uint8).copy()).cuda()
    counters = torch.zeros(4, dtype=torch.int32, device="cuda")
    aes.aes_ecb_batch(items_dev, 2, 0, kt, in_arena, out_arena, counters)
    torch.cuda.synchronize()
    assert int(counters[3].item()) == 1
    assert not out_arena[16 * n:].any(), "the rejected item wrote its last block"
    win = 1 << 20
    for off in (0, 16 * n - win):  # the first and the last MiB of the item
        xw = in_arena[off:off + win].cpu().numpy()
        j = first_mismatch(out_arena[off:off + win].cpu().numpy(), oracle_lib.ecb_encrypt(key, xw))
        assert j is None, "window @%d: byte %d differs" % (off, j)


def test_batch_config_2_full_mix(oracle_lib):
    """The full batched workload: 20,000 messages, log-uniform 16 B - 8 MiB,
    own key and key size each, half encrypt half decrypt (about 12.7 GB)."""
    torch = cuda()
    mix = inputs.message_mix(2, 20000)
    keys = [inputs.random_key(int(s), int(b)) for s, b in zip(mix.key_seed, mix.keybits)]
    kt = batch.key_table(keys)
    total = mix.total_blocks
    in_arena = inputs.device_random_bytes(2, 16 * total)
    out_arena = torch.zeros_like(in_arena)
    b = batch.prepare(batch.messages_from_mix(mix), kt, in_arena, out_arena, chunk_blocks=1024)
    b.replay()
    torch.cuda.synchronize()
    assert b.rejected_items() == 0
    ref = torch.zeros_like(in_arena)
    scheds = [aes.aes_expand_key(k) for k in keys]
    batch.run_per_message(b.msgs, scheds, in_arena, ref)
    torch.cuda.synchronize()
    assert torch.equal(ref, out_arena), "batched output differs from per-message plain launches"
    del ref
    # oracle on a seeded sample of messages (whole if <= 64 KiB, else head, tail and a middle window)
    g = inputs.rng(80)
    for i in g.choice(len(mix), 60, replace=False):
        lo, n = int(mix.offset[i]) * 16, int(mix.nblocks[i]) * 16
        mid = n // 2 // 16 * 16
        spans = [(0, n)] if n <= 65536 else [(0, 4096), (n - 4096, n), (mid, min(n, mid + 65536))]
        for a, z in spans:
            src = in_arena[lo + a:lo + z].cpu().numpy()
            want = oracle_lib.ecb_decrypt(keys[i], src) if mix.decrypt[i] else oracle_lib.ecb_encrypt(keys[i], src)
            assert np.array_equal(out_arena[lo + a:lo + z].cpu().numpy(), want), (int(i), a)
