"""The native serving engine (aes_server_*): admission policy, budget, arena
and error paths in dry-run mode on the CPU; on the GPU every served result
equals the same request run alone through the plain kernel, bit-exact."""
import time

import numpy as np
import pytest

from paper_1902_05234_amd import aes, inputs


def requests(n, seed, max_blocks=3000, pool_blocks=200000, slots=8):
    g = inputs.rng(60, seed)
    r = np.zeros(n, dtype=aes.REQUEST_DTYPE)
    r["nblocks"] = g.integers(1, max_blocks, n)
    r["in_block"] = [int(g.integers(0, pool_blocks - nb)) for nb in r["nblocks"]]
    r["key_slot"] = g.integers(0, slots, n)
    r["decrypt"] = g.integers(0, 2, n)
    return r


def wait_all(srv, n, timeout=30.0):
    got = []
    t0 = time.time()
    while sum(len(x) for x in got) < n:
        got.append(srv.poll())
        if time.time() - t0 > timeout:
            raise AssertionError("requests did not finish")
        time.sleep(0.0005)
    out = np.concatenate(got)
    return out[np.argsort(out["id"])]


# ------------------------------------------------------------------ CPU part
def test_dry_run_budget_fifo_and_overlap():
    budget = 2 * 16 * 20000
    srv = aes.Server(n_slots=8, in_blocks=200000, out_blocks=60000, budget_bytes=budget, chunk_blocks=256,
                     max_batch_items=512, nslots=3, dry_run=True, dry_run_seconds=0.002, size_classes=False)
    r = requests(300, 1)
    first = srv.submit(r)
    out = wait_all(srv, 300)
    st = srv.stats()
    srv.close()
    assert first == 0 and (out["id"] == np.arange(300)).all()
    assert (out["status"] == aes.AES_SERVED_DONE).all()
    assert st["max_device_bytes_in_use"] <= budget
    assert st["arena_blocks_in_use"] == 0 and st["pending"] == 0
    assert st["batches"] >= 10
    assert (np.diff(out["admitted_s"]) >= 0).all(), "admission must follow submission order"
    assert (out["done_s"] >= out["admitted_s"]).all() and (out["admitted_s"] >= out["arrival_s"]).all()
    # requests of one batch share a batch index; batches are numbered in admission order
    assert (np.diff(out["batch"]) >= 0).all()


def test_dry_run_size_classes_keep_small_requests_out_of_large_batches():
    """With size classes every batch holds only requests of at most
    chunk_blocks blocks or only larger ones, each class is admitted in
    submission order, and everything completes; without them the same queue
    mixes the classes."""
    chunk = 256
    g = inputs.rng(60, 77)
    r = np.zeros(200, dtype=aes.REQUEST_DTYPE)
    large = g.random(200) < 0.3
    r["nblocks"] = np.where(large, g.integers(chunk + 1, 4 * chunk, 200), g.integers(1, chunk + 1, 200))
    r["in_block"] = 0
    r["key_slot"] = g.integers(0, 4, 200)
    r["decrypt"] = g.integers(0, 2, 200)
    mixed = {}
    for classes in (True, False):
        srv = aes.Server(n_slots=4, in_blocks=100000, out_blocks=200000, budget_bytes=1 << 30, chunk_blocks=chunk,
                         max_batch_items=64, nslots=2, dry_run=True, dry_run_seconds=0.001, size_classes=classes)
        srv.submit(r)
        out = wait_all(srv, 200)
        srv.close()
        assert (out["status"] == aes.AES_SERVED_DONE).all()
        big = out["nblocks"] > chunk
        mixed[classes] = sum(len(set(big[out["batch"] == b])) > 1 for b in np.unique(out["batch"]))
        for cls in (True, False):
            sel = out[big == cls]
            assert (np.diff(sel["admitted_s"]) >= 0).all(), "each class is admitted in submission order"
    assert mixed[True] == 0, "a batch mixed small and large requests"
    assert mixed[False] > 0, "the single FIFO was expected to mix the classes here"


def test_dry_run_rejects_what_can_never_run():
    srv = aes.Server(n_slots=4, in_blocks=10000, out_blocks=5000, budget_bytes=2 * 16 * 4000, chunk_blocks=64,
                     max_batch_items=256, nslots=2, dry_run=True, dry_run_seconds=0.0005)
    r = requests(40, 2, max_blocks=500, pool_blocks=10000, slots=4)
    r[3]["nblocks"] = 0                 # empty
    r[7]["nblocks"] = 4500              # over the budget
    r[11]["key_slot"] = 9               # no such key slot
    r[15]["in_block"] = 9990            # runs past the input pool
    srv.submit(r)
    out = wait_all(srv, 40)
    srv.close()
    bad = {3, 7, 11, 15}
    for i in range(40):
        assert out[i]["status"] == (aes.AES_SERVED_REJECTED if i in bad else aes.AES_SERVED_DONE), i


def test_dry_run_rejects_a_size_whose_byte_count_wraps():
    """2^59 blocks are 2^64 bytes in and out: rejected at once, not admitted as
    zero bytes and left to block the queue."""
    srv = aes.Server(n_slots=2, in_blocks=1 << 62, out_blocks=1 << 62, budget_bytes=1 << 30, chunk_blocks=256,
                     max_batch_items=64, nslots=2, dry_run=True, dry_run_seconds=0.0002)
    r = requests(3, 4, max_blocks=100, pool_blocks=100000, slots=2)
    r[1]["in_block"] = 0
    r[1]["nblocks"] = 1 << 59
    srv.submit(r)
    out = wait_all(srv, 3, timeout=10.0)
    srv.close()
    assert out["status"].tolist() == [aes.AES_SERVED_DONE, aes.AES_SERVED_REJECTED, aes.AES_SERVED_DONE]


def test_dry_run_rejects_a_request_larger_than_one_batch():
    """A request whose work items exceed max_batch_items could never be
    admitted: it is rejected at once, and the requests behind it still run."""
    srv = aes.Server(n_slots=2, in_blocks=100000, out_blocks=100000, budget_bytes=1 << 30, chunk_blocks=64,
                     max_batch_items=4, nslots=2, dry_run=True, dry_run_seconds=0.0002)
    r = requests(4, 5, max_blocks=100, pool_blocks=100000, slots=2)
    r[1]["nblocks"] = 4 * 64 + 1
    r[2]["nblocks"] = 4 * 64
    srv.submit(r)
    out = wait_all(srv, 4, timeout=10.0)
    srv.close()
    assert out["status"].tolist() == [aes.AES_SERVED_DONE, aes.AES_SERVED_REJECTED, aes.AES_SERVED_DONE,
                                      aes.AES_SERVED_DONE]


def test_dry_run_small_requests_are_counted_in_small_items():
    """A request of at most chunk_blocks blocks is split into items of
    small_item_blocks: with chunk 256 and small items of 16, a 100-block
    request needs 7 items and cannot fit a batch of 4, while a 300-block
    request (two 256-block chunks) fits."""
    srv = aes.Server(n_slots=2, in_blocks=100000, out_blocks=100000, budget_bytes=1 << 30, chunk_blocks=256,
                     small_item_blocks=16, max_batch_items=4, nslots=2, dry_run=True, dry_run_seconds=0.0002)
    r = requests(3, 6, max_blocks=60, pool_blocks=100000, slots=2)
    r[0]["nblocks"] = 64    # 4 small items: fits
    r[1]["nblocks"] = 100   # 7 small items: never fits
    r[2]["nblocks"] = 300   # 2 chunks: fits
    srv.submit(r)
    out = wait_all(srv, 3, timeout=10.0)
    srv.close()
    assert out["status"].tolist() == [aes.AES_SERVED_DONE, aes.AES_SERVED_REJECTED, aes.AES_SERVED_DONE]
    with pytest.raises(aes.AesError):
        aes.Server(n_slots=1, in_blocks=10, out_blocks=10, chunk_blocks=64, small_item_blocks=65, dry_run=True)


def test_dry_run_release_frees_only_outputs_still_held():
    """A second release of the same outputs, or a range the engine never
    handed out, is refused (AES_EINVAL) and leaves the arena intact."""
    srv = aes.Server(n_slots=2, in_blocks=100000, out_blocks=4000, budget_bytes=1 << 30, chunk_blocks=128,
                     max_batch_items=64, nslots=2, auto_release=False, dry_run=True, dry_run_seconds=0.0002)
    r = requests(10, 6, max_blocks=300, pool_blocks=100000, slots=2)
    srv.submit(r)
    out = wait_all(srv, 10)
    assert (out["status"] == aes.AES_SERVED_DONE).all()
    forged = out[:2].copy()
    forged[0]["out_block"] = 10**9        # never handed out
    forged[1]["nblocks"] += 1             # not the range that was handed out
    with pytest.raises(aes.AesError):
        srv.release(forged)
    srv.release(out)
    with pytest.raises(aes.AesError):
        srv.release(out[:3])              # released already
    t0 = time.time()
    while srv.stats()["arena_blocks_in_use"] != 0:
        assert time.time() - t0 < 5
        time.sleep(0.001)
    # every block of the arena is free again: a request as large as the arena runs
    big = requests(1, 7, max_blocks=100, pool_blocks=100000, slots=2)
    big[0]["in_block"] = 0
    big[0]["nblocks"] = 4000
    srv.submit(big)
    got = wait_all(srv, 1)
    srv.close()
    assert got[0]["status"] == aes.AES_SERVED_DONE and got[0]["out_block"] == 0


def test_dry_run_manual_release_gates_the_arena():
    srv = aes.Server(n_slots=2, in_blocks=100000, out_blocks=2000, budget_bytes=1 << 30, chunk_blocks=128,
                     max_batch_items=64, nslots=2, auto_release=False, dry_run=True, dry_run_seconds=0.0002)
    r = requests(30, 3, max_blocks=900, pool_blocks=100000, slots=2)
    srv.submit(r)
    done = []
    t0 = time.time()
    while len(done) < 30:
        got = srv.poll()
        if len(got):
            # outputs in use never exceed the arena
            assert srv.stats()["arena_blocks_in_use"] <= 2000
            done.extend(got.tolist())
            srv.release(got)
        assert time.time() - t0 < 20
        time.sleep(0.0005)
    srv.close()
    assert len(done) == 30


CLOSE_WHILE_BLOCKED = r"""
import sys, time
import numpy as np
from paper_1902_05234_amd import aes
srv = aes.Server(n_slots=2, in_blocks=100000, out_blocks=1000, budget_bytes=1 << 30, chunk_blocks=128,
                 max_batch_items=64, nslots=2, auto_release=False, dry_run=True, dry_run_seconds=0.0002)
r = np.zeros(3, dtype=aes.REQUEST_DTYPE)
r["nblocks"] = 600
r["in_block"] = [0, 1000, 2000]
srv.submit(r)
got, t0 = [], time.time()
while not got:
    got = srv.poll().tolist()
    assert time.time() - t0 < 10, "the first request did not finish"
    time.sleep(0.001)
time.sleep(0.05)
# the second request waits for output space the caller holds: the worker must sleep, not spin
c0, w0 = time.process_time(), time.time()
time.sleep(0.5)
cpu = (time.process_time() - c0) / (time.time() - w0)
st = srv.stats()
srv.close()
print("closed", cpu, st["pending"], flush=True)
"""


def test_dry_run_close_with_held_outputs_and_a_blocked_request():
    """Without auto release, a request that waits for output space the
    caller still holds neither keeps the worker busy nor stops close():
    close() finishes it as rejected and returns."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, "-c", CLOSE_WHILE_BLOCKED], cwd=root, capture_output=True, text=True,
                       timeout=60, env=dict(os.environ, PYTHONPATH=root))
    assert r.returncode == 0, r.stderr[-2000:]
    words = r.stdout.split()
    assert words[0] == "closed"
    assert float(words[1]) < 0.5, "the engine's worker spins while the queue is blocked"
    assert int(words[2]) == 2


def test_create_rejects_bad_configs():
    for kw in (dict(nslots=0), dict(nslots=17), dict(chunk_blocks=0), dict(chunk_blocks=aes.AES_MAX_ITEM_BLOCKS + 1),
               dict(bpt=3), dict(wg=100), dict(budget_bytes=0), dict(max_batch_items=0), dict(grid=-1),
               dict(placement=3), dict(completion=2)):
        args = dict(n_slots=1, in_blocks=10, out_blocks=10, dry_run=True)
        args.update(kw)
        with pytest.raises(aes.AesError):
            aes.Server(**args)


# ------------------------------------------------------------------ GPU part
@pytest.mark.gpu
@pytest.mark.parametrize("completion,placement,classes", [
    (aes.AES_SERVE_COMPLETION_AUTO, aes.AES_PLACEMENT_TTABLE4, True),
    (aes.AES_SERVE_COMPLETION_EVENTS, aes.AES_PLACEMENT_TTABLE4, True),
    (aes.AES_SERVE_COMPLETION_AUTO, aes.AES_PLACEMENT_TTABLE2, True),
    (aes.AES_SERVE_COMPLETION_AUTO, aes.AES_PLACEMENT_TTABLE4, False)])
def test_native_served_results_equal_the_request_alone(oracle_lib, completion, placement, classes):
    """Every served request equals the request run alone (and the oracle on
    samples), whichever way the worker sees batches finish (completion words
    written by the batch kernel, or events), with the 2-table batch kernel,
    and with size classes or one FIFO."""
    import torch
    from paper_1902_05234_amd import batch
    pool = inputs.key_pool(6, 32)
    kt = batch.key_table([k for _, k in pool])
    in_pool = inputs.device_random_bytes(6, 64 << 20)
    out_arena = torch.zeros(256 << 20, dtype=torch.uint8, device="cuda")
    srv = aes.Server(kt, in_pool, out_arena, budget_bytes=512 << 20, chunk_blocks=256, max_batch_items=1 << 14,
                     nslots=4, auto_release=False, completion=completion, placement=placement,
                     size_classes=classes)
    r = requests(500, 4, max_blocks=20000, pool_blocks=in_pool.numel() // 16, slots=len(pool))
    srv.submit(r[:250])
    time.sleep(0.001)
    srv.submit(r[250:])                 # arrives while the first ones run
    out = wait_all(srv, 500)
    assert (out["status"] == aes.AES_SERVED_DONE).all()
    assert srv.stats()["batches"] >= 2
    scheds = [aes.aes_expand_key(k) for _, k in pool]
    for i, q in enumerate(r):
        ks = scheds[int(q["key_slot"])]
        lo, n = int(q["in_block"]) * 16, int(q["nblocks"]) * 16
        ob = int(out[i]["out_block"]) * 16
        x = in_pool[lo:lo + n]
        alone = torch.empty_like(x)
        if q["decrypt"]:
            aes.aes_ecb_decrypt(ks.rk_dec, ks.nr, x, alone)
        else:
            aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, x, alone)
        assert torch.equal(alone, out_arena[ob:ob + n]), "request %d differs from the request alone" % i
    for i in range(0, 500, 25):
        q = r[i]
        lo, n = int(q["in_block"]) * 16, min(int(q["nblocks"]), 2048) * 16
        ob = int(out[i]["out_block"]) * 16
        key = pool[int(q["key_slot"])][1]
        x = in_pool[lo:lo + n].cpu().numpy()
        want = oracle_lib.ecb_decrypt(key, x) if q["decrypt"] else oracle_lib.ecb_encrypt(key, x)
        assert np.array_equal(out_arena[ob:ob + n].cpu().numpy(), want), i
    srv.release(out)
    srv.close()


@pytest.mark.gpu
def test_native_light_batches_read_items_from_pinned_staging(oracle_lib):
    """Batches of at most 4096 work items are launched on the work list in
    the pinned staging (no copy to the device): thirty bursts of ten small
    requests reuse the four slots many times, and every result must equal
    the request run alone."""
    import torch
    from paper_1902_05234_amd import batch
    pool = inputs.key_pool(8, 16)
    kt = batch.key_table([k for _, k in pool])
    in_pool = inputs.device_random_bytes(8, 32 << 20)
    out_arena = torch.zeros(64 << 20, dtype=torch.uint8, device="cuda")
    srv = aes.Server(kt, in_pool, out_arena, budget_bytes=256 << 20, chunk_blocks=512, nslots=4,
                     auto_release=False)
    r = requests(300, 9, max_blocks=6000, pool_blocks=in_pool.numel() // 16, slots=len(pool))
    for part in range(30):
        srv.submit(r[10 * part:10 * part + 10])
        time.sleep(0.0003)
    out = wait_all(srv, 300)
    assert (out["status"] == aes.AES_SERVED_DONE).all()
    st = srv.stats()
    assert st["batches"] >= 8
    assert st["direct_batches"] == st["batches"], "every batch here fits the direct work-list path"
    assert 0 < st["launch_ns"] < 1_000_000 * st["batches"], "launch time is counted and under 1 ms a batch"
    scheds = [aes.aes_expand_key(k) for _, k in pool]
    for i, q in enumerate(r):
        ks = scheds[int(q["key_slot"])]
        lo, n = int(q["in_block"]) * 16, int(q["nblocks"]) * 16
        ob = int(out[i]["out_block"]) * 16
        x = in_pool[lo:lo + n]
        alone = torch.empty_like(x)
        if q["decrypt"]:
            aes.aes_ecb_decrypt(ks.rk_dec, ks.nr, x, alone)
        else:
            aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, x, alone)
        assert torch.equal(alone, out_arena[ob:ob + n]), "request %d differs from the request alone" % i
    q = r[7]
    lo, n = int(q["in_block"]) * 16, int(q["nblocks"]) * 16
    ob = int(out[7]["out_block"]) * 16
    key = pool[int(q["key_slot"])][1]
    x = in_pool[lo:lo + n].cpu().numpy()
    want = oracle_lib.ecb_decrypt(key, x) if q["decrypt"] else oracle_lib.ecb_encrypt(key, x)
    assert np.array_equal(out_arena[ob:ob + n].cpu().numpy(), want)
    srv.release(out)
    srv.close()


@pytest.mark.gpu
def test_native_replay_reports_latency():
    import torch
    from paper_1902_05234_amd import batch
    pool = inputs.key_pool(7, 64)
    kt = batch.key_table([k for _, k in pool])
    in_pool = inputs.device_random_bytes(7, 256 << 20)
    out_arena = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    srv = aes.Server(kt, in_pool, out_arena, budget_bytes=1 << 30, chunk_blocks=1024, nslots=4)
    r = requests(2000, 5, max_blocks=8000, pool_blocks=in_pool.numel() // 16, slots=len(pool))
    arrival = np.cumsum(inputs.rng(61).exponential(20e-6, 2000))
    out = srv.replay(r, arrival)
    srv.close()
    assert (out["status"] == aes.AES_SERVED_DONE).all()
    lat = out["done_s"] - out["arrival_s"]
    assert (lat > 0).all() and np.percentile(lat, 99) < 1.0
