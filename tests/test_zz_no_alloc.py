"""The allocation-free batched launch (aes_ecb_batch_noalloc, counters in the
library's per-device scratch) gives exactly the output of aes_ecb_batch on
the same work list, on two calls in a row, the second with a smaller batch,
and the scratch's claim counters start from zero on every call."""
import numpy as np
import pytest

from paper_1902_05234_amd import aes, batch, inputs
from tests.gpu_util import cuda

pytestmark = pytest.mark.gpu


def _batch(torch, seed, n, hi_bytes, chunk, cfg):
    mix = inputs.message_mix(seed, n, hi_bytes=hi_bytes)
    keys = [inputs.random_key(int(s), int(b)) for s, b in zip(mix.key_seed, mix.keybits)]
    kt = batch.key_table(keys)
    x = inputs.random_bytes(seed, 16 * mix.total_blocks)
    in_arena = torch.from_numpy(x).cuda()
    out_arena = torch.zeros_like(in_arena)
    return batch.prepare(batch.messages_from_mix(mix), kt, in_arena, out_arena, chunk_blocks=chunk, cfg=cfg)


@pytest.mark.parametrize("placement", [aes.AES_PLACEMENT_TTABLE4, aes.AES_PLACEMENT_TTABLE2])
def test_noalloc_batch_equals_batch_twice_then_smaller(placement):
    torch = cuda()
    cfg = aes.BatchConfig(bpt=2, wg=1024, placement=placement)
    for seed, n, hi in ((61, 400, 512 << 10), (62, 60, 32 << 10)):  # the second call is smaller
        b = _batch(torch, seed + placement, n, hi, 256, cfg)
        b.launch()
        torch.cuda.synchronize()
        want = b.out_arena.clone()
        assert b.rejected_items() == 0
        for rep in range(2):
            b.out_arena.zero_()
            torch.cuda.synchronize()
            aes.aes_ecb_batch_noalloc(b.items_dev, b.n_enc, b.n_dec, b.key_table_dev, b.in_arena, b.out_arena, b.cfg)
            torch.cuda.synchronize()
            if not torch.equal(b.out_arena, want):
                diff = (b.out_arena != want).nonzero()
                raise AssertionError("seed %d call %d: byte %d differs from aes_ecb_batch" % (seed, rep, int(diff[0])))


def test_noalloc_batch_runs_after_a_grid_that_stopped_early():
    """A call whose grid is smaller than the previous one still starts from
    zeroed counters: a tiny grid, then the persistent grid, then a tiny one."""
    torch = cuda()
    b = _batch(torch, 70, 120, 64 << 10, 64, aes.BatchConfig(bpt=1, wg=256, placement=aes.AES_PLACEMENT_TTABLE1))
    b.launch()
    torch.cuda.synchronize()
    want = b.out_arena.clone()
    for grid in (1, 0, 3):
        cfg = aes.BatchConfig(bpt=1, wg=256, placement=aes.AES_PLACEMENT_TTABLE1, grid=grid)
        b.out_arena.zero_()
        aes.aes_ecb_batch_noalloc(b.items_dev, b.n_enc, b.n_dec, b.key_table_dev, b.in_arena, b.out_arena, cfg)
        torch.cuda.synchronize()
        assert torch.equal(b.out_arena, want), "grid %d" % grid


def test_noalloc_batch_rejects_what_aes_ecb_batch_rejects():
    torch = cuda()
    b = _batch(torch, 71, 10, 16 << 10, 64, aes.BatchConfig())
    with pytest.raises(aes.AesError):
        aes.aes_ecb_batch_noalloc(b.items_dev, b.n_enc, b.n_dec, b.key_table_dev, b.in_arena, b.out_arena,
                                  aes.BatchConfig(bpt=3))
    with pytest.raises(aes.AesError):
        aes.aes_ecb_batch_noalloc(b.items_dev, b.n_enc, b.n_dec, b.key_table_dev, b.in_arena[16:], b.in_arena[:-16])


def test_noalloc_batch_replays_in_a_graph():
    """The callers this entry point is for capture it: a graph holding the
    counter-zeroing kernel and the batch kernel, replayed four times with
    eager work (an aes_ecb_batch launch that uses its own counters) and
    synchronisations between the replays, equals the eager output each time."""
    torch = cuda()
    b = _batch(torch, 72, 150, 256 << 10, 512, aes.BatchConfig(bpt=4, wg=1024))
    b.launch()
    torch.cuda.synchronize()
    want = b.out_arena.clone()
    # one call outside the capture: the first call on a device looks up the
    # scratch's address and the variant's occupancy, which a capture forbids
    aes.aes_ecb_batch_noalloc(b.items_dev, b.n_enc, b.n_dec, b.key_table_dev, b.in_arena, b.out_arena, b.cfg)
    torch.cuda.synchronize()
    assert torch.equal(b.out_arena, want)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            aes.aes_ecb_batch_noalloc(b.items_dev, b.n_enc, b.n_dec, b.key_table_dev, b.in_arena, b.out_arena,
                                      b.cfg)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(4):
        b.out_arena.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(b.out_arena, want), "replay %d differs from aes_ecb_batch" % rep
        b.launch()  # eager work between replays
        torch.cuda.synchronize()
    del g
