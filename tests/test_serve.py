"""Serving loop: admission/budget/arena policy on the CPU with a fake
executor (injectable delay and failure), and on the GPU every served result
equals the same request run alone through the plain kernel (bit-exact)."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

from paper_1902_05234_amd import aes, inputs
from paper_1902_05234_amd.serve import (AdmissionError, OutputArena, Request, Scheduler, requests_from_trace,
                                        run_trace)


# ------------------------------------------------------------------ CPU part
@settings(max_examples=80, deadline=None)
@given(st.lists(st.tuples(st.booleans(), st.integers(1, 300)), max_size=200))
def test_arena_first_fit_never_overlaps(ops):
    a = OutputArena(4000)
    live = {}
    nid = 0
    for do_alloc, n in ops:
        if do_alloc or not live:
            s = a.alloc(n)
            if s is not None:
                for (s2, n2) in live.values():
                    assert s + n <= s2 or s2 + n2 <= s
                assert 0 <= s and s + n <= 4000
                live[nid] = (s, n)
                nid += 1
        else:
            k = sorted(live)[n % len(live)]
            s, m = live.pop(k)
            a.release(s, m)
        assert a.used == sum(m for _, m in live.values())
        for (s1, l1), (s2, l2) in zip(a.free, a.free[1:]):
            assert s1 + l1 < s2  # sorted, disjoint, coalesced
    for s, m in list(live.values()):
        a.release(s, m)
    assert a.free == [(0, 4000)] and a.used == 0


class FakeExecutor:
    """Completes a batch `delay` seconds of fake time after launch; batches
    whose first request id is in `fail_ids` fail at launch."""

    def __init__(self, clock, nslots=2, delay=0.01, fail_ids=()):
        self.clock, self.delay, self.fail_ids = clock, delay, set(fail_ids)
        self.slots = [dict(reqs=None, t=0.0) for _ in range(nslots)]
        self.launched = []
        self.max_concurrent = 0

    def free_slot(self):
        return next((s for s in self.slots if s["reqs"] is None), None)

    def launch(self, slot, reqs):
        if reqs[0].rid in self.fail_ids:
            raise RuntimeError("injected launch failure")
        slot["reqs"], slot["t"] = reqs, self.clock() + self.delay
        self.launched.append([r.rid for r in reqs])
        self.max_concurrent = max(self.max_concurrent, sum(s["reqs"] is not None for s in self.slots))

    def poll(self):
        out = []
        for s in self.slots:
            if s["reqs"] is not None and self.clock() >= s["t"]:
                out.append((s["reqs"], True))
                s["reqs"] = None
        return out

    def busy(self):
        return any(s["reqs"] is not None for s in self.slots)


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-4   # every look at the clock advances fake time
        return self.t


def make_reqs(n, seed=0, big_every=5):
    g = inputs.rng(40, seed)
    out = []
    t = 0.0
    for i in range(n):
        t += float(g.exponential(0.002))
        nb = int(g.integers(1000, 5000)) if i % big_every == 0 else int(g.integers(1, 200))
        out.append(Request(i, int(g.integers(0, 8)), bool(g.integers(0, 2)), 0, nb, t))
    return out


def test_budget_fifo_and_completion_with_fake_executor():
    clock = FakeClock()
    budget = 2 * 16 * 8000
    sch = Scheduler(budget, arena_blocks=10000, chunk_blocks=256)
    ex = FakeExecutor(clock, nslots=3, delay=0.005)
    peak = {"in_use": 0}
    orig_admit = sch.admit

    def admit(now):
        b = orig_admit(now)
        peak["in_use"] = max(peak["in_use"], sch.in_use)
        assert sch.in_use <= budget
        return b
    sch.admit = admit
    reqs = make_reqs(300)
    stats = run_trace(sch, ex, reqs, time_fn=clock)
    assert len(stats.latencies_s) == 300 and (stats.latencies_s > 0).all()
    assert sch.in_use == 0 and sch.arena.used == 0 and not sch.pending
    order = [rid for batch in ex.launched for rid in batch]
    assert order == sorted(order), "admission must follow arrival order"
    assert peak["in_use"] <= budget
    assert ex.max_concurrent >= 2, "batches should overlap while others are in flight"


def test_oversized_request_rejected_and_failures_release_budget():
    clock = FakeClock()
    sch = Scheduler(2 * 16 * 1000, arena_blocks=5000, chunk_blocks=64)
    reqs = make_reqs(60, seed=1, big_every=1000)
    reqs[7].nblocks = 2000                   # larger than the whole budget
    ex = FakeExecutor(clock, nslots=2, delay=0.002, fail_ids={20, 40})
    stats = run_trace(sch, ex, reqs, time_fn=clock)
    status = {r.rid: r.status for r in stats.requests}
    assert status[7] == "rejected"
    assert status[20] == "failed" and status[40] == "failed"
    assert sum(s == "done" for s in status.values()) >= 50
    assert sch.in_use == 0 and sch.arena.used == 0
    with pytest.raises(AdmissionError):
        sch.submit(Request(999, 0, False, 0, 0, 0.0))
    # a request must fit one batch's work list
    small = Scheduler(1 << 30, arena_blocks=1 << 20, max_batch_items=4, chunk_blocks=64)
    small.submit(Request(1000, 0, False, 0, 4 * 64, 0.0))
    with pytest.raises(AdmissionError):
        small.submit(Request(1001, 0, False, 0, 4 * 64 + 1, 0.0))


# ------------------------------------------------------------------ GPU part
def serve_setup(n_req, seed, rate, small_max=16 << 10, large=(64 << 10, 1 << 20), pool_mib=64, nslots=4):
    import torch
    from paper_1902_05234_amd import batch
    from paper_1902_05234_amd.serve import GpuExecutor
    pool = inputs.key_pool(3, 64)
    kt = batch.key_table([k for _, k in pool])
    pool_blocks = (pool_mib << 20) // 16
    in_pool = inputs.device_random_bytes(seed, pool_blocks * 16)
    g = inputs.rng(41, seed)
    arrival = np.cumsum(g.exponential(1.0 / rate, n_req))
    small = g.random(n_req) < 0.8
    lu = lambda a, b: np.rint(np.exp(g.uniform(np.log(a), np.log(b), n_req)) / 16).astype(np.int64).clip(1)
    nblocks = np.where(small, lu(64, small_max), lu(*large))
    trace = inputs.RequestTrace(arrival, nblocks, g.integers(0, len(pool), n_req), g.random(n_req) < 0.5)
    reqs = requests_from_trace(trace, pool_blocks, seed)
    budget = 2 << 30
    out_arena = torch.zeros(budget // 2, dtype=torch.uint8, device="cuda")
    sch = Scheduler(budget, out_arena.numel() // 16, chunk_blocks=256, max_batch_items=1 << 16)
    ex = GpuExecutor(kt, in_pool, out_arena, nslots=nslots, max_items=1 << 16, chunk_blocks=256)
    return pool, in_pool, out_arena, sch, ex, reqs


@pytest.mark.gpu
def test_served_results_equal_the_request_alone(oracle_lib):
    import torch
    pool, in_pool, out_arena, sch, ex, reqs = serve_setup(400, 3, rate=20000.0)
    scheds = [aes.aes_expand_key(k) for _, k in pool]
    stats = run_trace(sch, ex, reqs, keep_outputs=True)   # outputs stay until compared
    torch.cuda.synchronize()
    checked = [(r, out_arena[r.out_block * 16:(r.out_block + r.nblocks) * 16]) for r in stats.requests]
    assert len(checked) == 400 and stats.batches >= 2
    for r, got in checked:
        ks = scheds[r.key_slot]
        x = in_pool[r.in_block * 16:(r.in_block + r.nblocks) * 16]
        alone = torch.empty_like(x)
        if r.decrypt:
            aes.aes_ecb_decrypt(ks.rk_dec, ks.nr, x, alone)
        else:
            aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, x, alone)
        assert torch.equal(alone, got), "request %d differs from the same request alone" % r.rid
    for r, got in checked[:40]:
        x = in_pool[r.in_block * 16:(r.in_block + min(r.nblocks, 4096)) * 16].cpu().numpy()
        key = pool[r.key_slot][1]
        want = oracle_lib.ecb_decrypt(key, x) if r.decrypt else oracle_lib.ecb_encrypt(key, x)
        assert np.array_equal(got[:x.size].cpu().numpy(), want), r.rid


@pytest.mark.gpu
def test_serving_reports_latency_percentiles():
    pool, in_pool, out_arena, sch, ex, reqs = serve_setup(300, 4, rate=2000.0)
    stats = run_trace(sch, ex, reqs)
    s = stats.summary()
    assert s["requests"] == 300 and 0 < s["p50_ms"] <= s["p99_ms"]
    assert sch.in_use == 0 and sch.arena.used == 0
