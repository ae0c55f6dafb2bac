"""Autotuner for the plain and batched ECB kernels.

Search space (plain path): blocks per thread {1, 2, 4} (16/32/64 bytes per
thread) x workgroup size {64, 128, 256, 512, 1024} x table placement (the
placements built into the library).  Every variant must reproduce the
reference variant's output bit for bit (and decrypt back to the input)
before it is timed.  Each (key size, direction, size bucket) is timed at two or
three sizes spread over the bucket: the best variant for a bucket changes
inside it (a buffer of a few wave units leaves waves idle with 64 bytes per
thread but not with 16), so the winner is the variant whose worst ratio to
the fastest variant over those sizes is highest.  The record is JSON keyed
by device and library source hash and can be installed into the library's
tuning table with ``apply``.

Batched path: chunk size (blocks per work item) x blocks per thread.

    python -m paper_1902_05234_amd.autotune --out tune.json
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

from . import aes, inputs

BPTS = (1, 2, 4)
WGS = (64, 128, 256, 512, 1024)
PLACEMENTS = (aes.AES_PLACEMENT_TTABLE4, aes.AES_PLACEMENT_TTABLE2, aes.AES_PLACEMENT_TTABLE1,
              aes.AES_PLACEMENT_BITSLICED)
BITSLICE_MAX_WG = 256
# sizes timed for each tuning bucket (bytes; bucket limits in aesgpu.h: 4 KiB,
# 64 KiB, 2 MiB, 8 MiB, 32 MiB, larger)
BUCKET_SIZES = ((2 << 10, 4 << 10), (16 << 10, 64 << 10), (256 << 10, 1 << 20, 2 << 20), (3 << 20, 8 << 20),
                (12 << 20, 32 << 20), (256 << 20,))


def source_hash() -> str:
    """Hash of the device code the timings depend on (the .hip and .hpp
    sources; host-only files and caches are left out)."""
    h = hashlib.sha256()
    csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    for f in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.hpp"))):
        h.update(os.path.basename(f).encode())
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


GRAPH_TIMED_MAX = 64 << 20  # below this the host's per-call cost would dominate an eager timing
GRAPH_LAUNCHES = 20


def _graph_times(torch, fn, reps):
    """Per-launch device time (ms) of fn from HIP-graph replays of 20 captured
    launches: the host's per-call cost stays out of the figure."""
    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(GRAPH_LAUNCHES):
            fn()
    g.replay()
    out = [t / GRAPH_LAUNCHES for t in _times(torch, g.replay, reps)]
    del g
    return out


def _times(torch, fn, reps):
    """Durations (ms) of reps launches of fn, HIP events on the launch stream."""
    fn()
    s = torch.cuda.current_stream()
    evs = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        fn()
        b.record(s)
        evs.append((a, b))
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in evs]


def _time(torch, fn, reps):
    ms = sorted(_times(torch, fn, reps))
    return ms[len(ms) // 2]


def variants(log=None):
    """The search space.  The bitsliced placement always takes 32 blocks per
    lane (bpt does not apply) and at most 256-thread workgroups; the
    combinations it cannot run are skipped and logged once."""
    skipped = []
    for p in PLACEMENTS:
        for b in BPTS:
            for w in WGS:
                if p == aes.AES_PLACEMENT_BITSLICED and (b != 1 or w > BITSLICE_MAX_WG):
                    skipped.append((p, b, w))
                    continue
                yield aes.Variant(bpt=b, wg=w, placement=p)
    if log is not None and skipped:
        log("  skipped %d bitsliced combinations (bpt does not apply; wg <= %d)" % (len(skipped), BITSLICE_MAX_WG))


def tune_plain(torch, keybits: int, decrypt: bool, nbytes: int, reps: int = 10, rounds: int = 3, log=print):
    """Time every variant on one (key size, direction, size); returns rows
    sorted by time.  The variants are timed in ``rounds`` interleaved passes
    (reps launches each) and ranked by the median over all launches, so a
    drift of the engine clock during the sweep does not favour whichever
    variant ran first.  Up to 64 MiB a launch is timed inside a replayed HIP
    graph, which leaves the host's per-call cost out."""
    key = inputs.random_key(7, keybits)
    ks = aes.aes_expand_key(key)
    x = inputs.device_random_bytes(7, nbytes)
    ref = torch.empty_like(x)
    rk = ks.rk_dec if decrypt else ks.rk_enc
    aes.aes_ecb_crypt_variant(rk, ks.nr, decrypt, x, ref, aes.Variant())
    back = torch.empty_like(x)
    inv = ks.rk_enc if decrypt else ks.rk_dec
    aes.aes_ecb_crypt_variant(inv, ks.nr, not decrypt, ref, back, aes.Variant())
    torch.cuda.synchronize()
    if not torch.equal(back, x):
        raise RuntimeError("reference variant does not round-trip")
    out = torch.empty_like(x)
    vs = list(variants(log))
    for v in vs:
        out.zero_()
        aes.aes_ecb_crypt_variant(rk, ks.nr, decrypt, x, out, v)
        torch.cuda.synchronize()
        if not torch.equal(out, ref):
            raise RuntimeError("variant %s differs from the reference output" % (v,))
    times = {i: [] for i in range(len(vs))}
    timer = _graph_times if nbytes <= GRAPH_TIMED_MAX else _times
    for _ in range(max(1, rounds)):
        for i, v in enumerate(vs):
            times[i] += timer(torch, lambda: aes.aes_ecb_crypt_variant(rk, ks.nr, decrypt, x, out, v), reps)
    rows = []
    for i, v in enumerate(vs):
        t = sorted(times[i])
        ms = t[len(t) // 2]
        rows.append({"bpt": v.bpt, "wg": v.wg, "placement": v.placement, "ms": ms, "GB_s": nbytes / (ms * 1e-3) / 1e9})
    rows.sort(key=lambda r: r["ms"])
    log("  %d-bit %s %d B: best bpt=%d wg=%d placement=%d %.1f GB/s (worst %.1f)" % (
        keybits, "dec" if decrypt else "enc", nbytes, rows[0]["bpt"], rows[0]["wg"], rows[0]["placement"],
        rows[0]["GB_s"], rows[-1]["GB_s"]))
    return rows


def tune_batch(torch, n_messages: int = 20000, chunks=(256, 1024, 4096), reps: int = 5, log=print):
    from . import batch
    mix = inputs.message_mix(2, n_messages)
    keys = [inputs.random_key(int(s), int(b)) for s, b in zip(mix.key_seed, mix.keybits)]
    kt = batch.key_table(keys)
    in_arena = inputs.device_random_bytes(2, 16 * mix.total_blocks)
    out_arena = torch.empty_like(in_arena)
    ref = None
    rows = []
    for chunk in chunks:
        for bpt in BPTS:
            b = batch.prepare(batch.messages_from_mix(mix), kt, in_arena, out_arena, chunk_blocks=chunk,
                              cfg=aes.BatchConfig(bpt=bpt))
            out_arena.zero_()
            b.launch()
            torch.cuda.synchronize()
            if ref is None:
                ref = out_arena.clone()
            elif not torch.equal(out_arena, ref):
                raise RuntimeError("batch chunk=%d bpt=%d differs from the first configuration" % (chunk, bpt))
            ms = _time(torch, b.launch, reps)
            rows.append({"chunk_blocks": chunk, "bpt": bpt, "ms": ms, "GB_s": b.total_bytes / (ms * 1e-3) / 1e9})
            log("  batch chunk=%d bpt=%d: %.1f GB/s" % (chunk, bpt, rows[-1]["GB_s"]))
    rows.sort(key=lambda r: r["ms"])
    return rows


def bucket_winner(per_size: dict) -> dict:
    """The variant whose worst ratio to the fastest variant, over the sizes
    timed for one bucket, is highest.  per_size: {nbytes: rows}."""
    def vid(r):
        return (r["bpt"], r["wg"], r["placement"])
    best = {n: max(r["GB_s"] for r in rows) for n, rows in per_size.items()}
    score = {}
    for n, rows in per_size.items():
        for r in rows:
            score[vid(r)] = min(score.get(vid(r), 1.0), r["GB_s"] / best[n])
    common = [v for v in score if all(any(vid(r) == v for r in rows) for rows in per_size.values())]
    v = max(common, key=lambda k: score[k])
    return {"bpt": v[0], "wg": v[1], "placement": v[2], "worst_ratio": round(score[v], 4)}


def run(buckets=BUCKET_SIZES, key_sizes=(128, 192, 256), batch_too=True, reps=10, rounds=3, log=print):
    """buckets: one tuple of sizes per tuning bucket (the library's bucket of
    each tuple's sizes must agree)."""
    import torch
    rec = {"device": torch.cuda.get_device_properties(0).name, "source_hash": source_hash(),
           "created": time.strftime("%Y-%m-%dT%H:%M:%S"), "plain": {}, "batch": None}
    for kb in key_sizes:
        for dec in (False, True):
            for sizes in buckets:
                bucket = {aes.aes_size_bucket(n // 16) for n in sizes}
                if len(bucket) != 1:
                    raise ValueError("sizes %s span several tuning buckets" % (sizes,))
                per_size = {n: tune_plain(torch, kb, dec, n, reps=reps, rounds=rounds, log=log) for n in sizes}
                w = bucket_winner(per_size)
                log("  %d-bit %s bucket %d: bpt=%d wg=%d placement=%d (worst ratio %.3f)" % (
                    kb, "dec" if dec else "enc", bucket.pop(), w["bpt"], w["wg"], w["placement"], w["worst_ratio"]))
                rec["plain"]["%d/%s/%d" % (kb, "dec" if dec else "enc", max(sizes))] = {
                    "winner": w, "sizes": list(sizes), "all": {str(n): rows for n, rows in per_size.items()}}
    if batch_too:
        rec["batch"] = tune_batch(torch, log=log)
    return rec


def apply(record: dict):
    """Install the plain-path winners of a record into the library's tuning table."""
    n = 0
    for k, v in record.get("plain", {}).items():
        kb, d, nbytes = k.split("/")
        w = v["winner"]
        nr = {128: 10, 192: 12, 256: 14}[int(kb)]
        aes.aes_tune_set(nr, d == "dec", int(nbytes) // 16, aes.Variant(w["bpt"], w["wg"], w["placement"]))
        n += 1
    return n


def load(path: str) -> dict:
    with open(path) as f:
        return json.load(f)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", default="aesgpu_tune.json")
    ap.add_argument("--quick", action="store_true", help="AES-256 decrypt of 256 MiB plus the batch mix only")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--reps", type=int, default=10, help="launches per variant per round")
    ap.add_argument("--rounds", type=int, default=3, help="interleaved passes over the variants")
    ap.add_argument("--sizes", default=None,
                    help="comma-separated byte sizes, each tuned on its own (default: two or three per size bucket)")
    a = ap.parse_args(argv)
    log = lambda *x: print(*x, file=sys.stderr, flush=True)
    if a.quick:
        rec = run(buckets=((256 << 20,),), key_sizes=(256,), batch_too=not a.no_batch, reps=a.reps, rounds=a.rounds,
                  log=log)
    else:
        buckets = tuple((int(x),) for x in a.sizes.split(",")) if a.sizes else BUCKET_SIZES
        rec = run(buckets=buckets, batch_too=not a.no_batch, reps=a.reps, rounds=a.rounds, log=log)
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
    log("wrote", a.out)


if __name__ == "__main__":
    main()
