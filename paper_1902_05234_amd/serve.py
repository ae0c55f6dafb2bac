"""Continuous-batching request loop for ECB encryption/decryption.

Requests (key slot, direction, input blocks) arrive over time.  The loop
admits them in arrival order while the device-memory budget (input + output
bytes of every admitted, unfinished request) allows, places each output in a
first-fit output arena, and whenever one of its stream slots is free it
launches everything admitted so far as one batched kernel
(``aes_ecb_batch``).  Requests that arrive while batches run are admitted as
slots and memory free up, so batches from several streams overlap on the
device.  Completion is observed by polling HIP events; a finished request
releases its budget and its output space once the caller has taken it.

The policy (``Scheduler``, ``OutputArena``) is plain Python and runs without
a GPU; ``GpuExecutor`` is the only part that touches the device, and every
cipher step runs in the library's batch kernel.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import aes

BLOCK = 16


class AdmissionError(ValueError):
    """A request that can never be admitted (larger than the whole budget)."""


class OutputArena:
    """First-fit allocator over ``nblocks`` blocks with coalescing frees."""

    def __init__(self, nblocks: int):
        self.nblocks = int(nblocks)
        self.free = [(0, self.nblocks)]  # sorted (start, length)
        self.used = 0

    def alloc(self, n: int):
        for i, (s, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (s + n, ln - n)
                self.used += n
                return s
        return None

    def release(self, start: int, n: int):
        self.used -= n
        lst = self.free
        lo, hi = 0, len(lst)
        while lo < hi:
            mid = (lo + hi) // 2
            if lst[mid][0] < start:
                lo = mid + 1
            else:
                hi = mid
        lst.insert(lo, (start, n))
        # merge with neighbours
        if lo + 1 < len(lst) and lst[lo][0] + lst[lo][1] == lst[lo + 1][0]:
            lst[lo] = (lst[lo][0], lst[lo][1] + lst[lo + 1][1])
            lst.pop(lo + 1)
        if lo > 0 and lst[lo - 1][0] + lst[lo - 1][1] == lst[lo][0]:
            lst[lo - 1] = (lst[lo - 1][0], lst[lo - 1][1] + lst[lo][1])
            lst.pop(lo)


@dataclass
class Request:
    rid: int
    key_slot: int
    decrypt: bool
    in_block: int
    nblocks: int
    arrival: float
    out_block: int = -1
    admitted: float = 0.0
    done: float = 0.0
    status: str = "pending"   # pending -> admitted -> done | failed

    @property
    def nbytes(self) -> int:
        return self.nblocks * BLOCK

    @property
    def latency(self) -> float:
        return self.done - self.arrival


class Scheduler:
    """Admission by device-memory budget, FIFO, into batches."""

    def __init__(self, budget_bytes: int, arena_blocks: int, max_batch_items: int = 1 << 20, chunk_blocks: int = 1024):
        self.budget = int(budget_bytes)
        self.in_use = 0
        self.arena = OutputArena(arena_blocks)
        self.pending = collections.deque()
        self.max_items = int(max_batch_items)
        self.chunk = int(chunk_blocks)

    def submit(self, req: Request):
        if 2 * req.nbytes > self.budget or req.nblocks > self.arena.nblocks:
            raise AdmissionError("request %d (%d bytes) exceeds the device budget" % (req.rid, req.nbytes))
        if req.nblocks <= 0:
            raise AdmissionError("request %d has no blocks" % req.rid)
        if -(-req.nblocks // self.chunk) > self.max_items:
            raise AdmissionError("request %d needs more work items than one batch holds" % req.rid)
        self.pending.append(req)

    def admit(self, now: float):
        """Admit pending requests in arrival order until the budget, the
        output arena or the batch size stops the head of the queue."""
        batch, items = [], 0
        while self.pending:
            r = self.pending[0]
            need_items = -(-r.nblocks // self.chunk)  # submit(): at most max_items
            if items + need_items > self.max_items:
                break
            if self.in_use + 2 * r.nbytes > self.budget:
                break
            start = self.arena.alloc(r.nblocks)
            if start is None:
                break
            self.pending.popleft()
            r.out_block = start
            r.admitted = now
            r.status = "admitted"
            self.in_use += 2 * r.nbytes
            items += need_items
            batch.append(r)
        return batch

    def finish(self, reqs, now: float, ok: bool = True):
        for r in reqs:
            r.done = now
            r.status = "done" if ok else "failed"
            self.in_use -= 2 * r.nbytes

    def release_output(self, r: Request):
        self.arena.release(r.out_block, r.nblocks)


def batch_messages(reqs) -> np.ndarray:
    m = np.zeros(len(reqs), dtype=aes.MSG_DTYPE)
    for i, r in enumerate(reqs):
        m[i] = (r.in_block, r.out_block, r.nblocks, r.key_slot, int(r.decrypt))
    return m


class GpuExecutor:
    """Runs batches on ``nslots`` streams; one batch per slot at a time."""

    def __init__(self, key_table_dev, in_pool, out_arena, nslots: int = 4, max_items: int = 1 << 20,
                 chunk_blocks: int = 1024, cfg: aes.BatchConfig | None = None):
        import torch
        self.torch = torch
        self.key_table = key_table_dev
        self.in_pool = in_pool
        self.out_arena = out_arena
        self.chunk = int(chunk_blocks)
        self.cfg = cfg or aes.BatchConfig()
        self.grid = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
        self.slots = []
        for _ in range(nslots):
            self.slots.append({
                "stream": torch.cuda.Stream(),
                "items_host": torch.empty(max_items * aes.ITEM_DTYPE.itemsize, dtype=torch.uint8, pin_memory=True),
                "items_dev": torch.empty(max_items * aes.ITEM_DTYPE.itemsize, dtype=torch.uint8, device="cuda"),
                "counters": torch.zeros(4, dtype=torch.int32, device="cuda"),
                "event": None, "reqs": None,
            })
        self.max_items = int(max_items)

    def free_slot(self):
        for s in self.slots:
            if s["reqs"] is None:
                return s
        return None

    def launch(self, slot, reqs):
        torch = self.torch
        items, ne, nd = aes.aes_batch_plan(batch_messages(reqs), self.chunk)
        n = ne + nd
        if n > self.max_items:
            raise RuntimeError("batch of %d items exceeds the slot capacity" % n)
        nb = n * aes.ITEM_DTYPE.itemsize
        slot["items_host"].numpy()[:nb] = items.view(np.uint8)
        enc_b = int(items["nblocks"][:ne].sum())
        tot = max(1, int(items["nblocks"].sum()))
        enc_groups = (max(1, round(self.grid * enc_b / tot)) if ne else 0) if nd else self.grid
        cfg = aes.BatchConfig(self.cfg.bpt, self.cfg.wg, self.cfg.grid, min(enc_groups, self.grid))
        with torch.cuda.stream(slot["stream"]):
            slot["items_dev"][:nb].copy_(slot["items_host"][:nb], non_blocking=True)
            aes.aes_ecb_batch(slot["items_dev"], ne, nd, self.key_table, self.in_pool, self.out_arena,
                              slot["counters"], cfg, slot["stream"])
            ev = torch.cuda.Event()
            ev.record(slot["stream"])
        slot["event"] = ev
        slot["reqs"] = reqs

    def poll(self):
        """Finished batches as (requests, ok) pairs."""
        done = []
        for s in self.slots:
            if s["reqs"] is not None and s["event"].query():
                done.append((s["reqs"], True))
                s["reqs"] = None
                s["event"] = None
        return done

    def busy(self) -> bool:
        return any(s["reqs"] is not None for s in self.slots)


@dataclass
class ServeStats:
    latencies_s: np.ndarray
    bytes: int
    wall_s: float
    batches: int
    max_in_use: int
    requests: list = field(repr=False, default_factory=list)

    def summary(self) -> dict:
        lat = np.sort(self.latencies_s) * 1e3
        pick = lambda q: float(lat[min(len(lat) - 1, int(q * len(lat)))]) if len(lat) else float("nan")
        return {"requests": int(len(lat)), "p50_ms": round(pick(0.50), 3), "p99_ms": round(pick(0.99), 3),
                "mean_ms": round(float(lat.mean()), 3) if len(lat) else None,
                "GB_s": round(self.bytes / self.wall_s / 1e9, 2), "batches": self.batches,
                "max_device_bytes_in_use": int(self.max_in_use)}


def run_trace(scheduler: Scheduler, executor, reqs, on_complete=None, time_fn=time.perf_counter,
              keep_outputs: bool = False) -> ServeStats:
    """Open-loop replay: request i is submitted at start + reqs[i].arrival.
    ``on_complete(req)`` runs on the host once the request's batch has
    finished; unless ``keep_outputs``, the request's output space is released
    as soon as it returns, so any device read of the output it enqueues must
    have completed by then (e.g. a synchronous copy)."""
    reqs = sorted(reqs, key=lambda r: r.arrival)
    t0 = time_fn()
    for r in reqs:
        r.arrival += t0
    i, batches, max_in_use, total = 0, 0, 0, 0
    finished = []

    def complete(group, ok):
        nonlocal total
        scheduler.finish(group, time_fn(), ok)
        for r in group:
            if ok and on_complete:
                on_complete(r)
            if not keep_outputs or not ok:
                scheduler.release_output(r)
            if ok:
                total += r.nbytes
        finished.extend(group)

    while len(finished) < len(reqs):
        now = time_fn()
        while i < len(reqs) and reqs[i].arrival <= now:
            try:
                scheduler.submit(reqs[i])
            except AdmissionError:
                reqs[i].status = "rejected"
                reqs[i].done = now
                finished.append(reqs[i])
            i += 1
        for group, ok in executor.poll():
            complete(group, ok)
        slot = executor.free_slot()
        if slot is not None and scheduler.pending:
            batch = scheduler.admit(time_fn())
            if batch:
                max_in_use = max(max_in_use, scheduler.in_use)
                try:
                    executor.launch(slot, batch)
                    batches += 1
                except Exception:  # the batch fails; its budget and output space come back
                    complete(batch, False)
        if i < len(reqs) and not scheduler.pending and not executor.busy():
            # idle: sleep until shortly before the next arrival
            wait = reqs[i].arrival - time_fn()
            if wait > 2e-4:
                time.sleep(wait - 1e-4)
    ok = [r for r in finished if r.status == "done"]
    wall = (max(r.done for r in ok) - min(r.arrival for r in ok)) if ok else 0.0
    lat = np.array([r.latency for r in ok])
    return ServeStats(lat, total, max(wall, 1e-9), batches, max_in_use, finished)


def requests_from_trace(trace, pool_blocks: int, seed: int = 0):
    """Requests for an ``inputs.RequestTrace``; each reads a seeded random
    window of a device input pool of ``pool_blocks`` blocks."""
    from . import inputs
    g = inputs.rng(9, seed)
    out = []
    for k in range(len(trace.nblocks)):
        nb = int(min(trace.nblocks[k], pool_blocks))
        start = int(g.integers(0, pool_blocks - nb + 1))
        out.append(Request(k, int(trace.key_slot[k]), bool(trace.decrypt[k]), start, nb, float(trace.arrival_s[k])))
    return out
