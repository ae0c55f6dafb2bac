"""Autotuner for the plain and batched ECB kernels.

Search space (plain path): bytes per thread {4, 16, 32, 64} (4: one column
word per lane, four lanes per block; 16-64: one to four whole blocks per
thread) x workgroup size {64, 128, 256, 512, 1024} x table placement (the
placements built into the library).  Every variant must reproduce the
reference variant's output bit for bit (and decrypt back to the input)
before it is timed.  Each (key size, direction, size bucket) is timed at two or
three sizes spread over the bucket: the best variant for a bucket changes
inside it (a buffer of a few wave units leaves waves idle with 64 bytes per
thread but not with 16), so the winner is the variant whose worst ratio to
the fastest variant over those sizes is highest.  Launches up to 64 MiB are
timed inside replayed HIP graphs (the host's per-call cost stays out); the
largest bucket is timed the way the library runs it there, with sustained
back-to-back launches: every variant is screened with short interleaved
timings, and the best few are then timed again over seconds of back-to-back
load in interleaved passes, where the engine clock has settled.

Batched path: chunk size (blocks per work item) x blocks per thread x
workgroup size x table placement, on the 20,000-message mix.

The record is JSON keyed by device (name and architecture) and by the hash
of the library's device sources.  ``apply`` installs its plain-path winners
into the library's tuning table and refuses a record made on another device
or for other kernel sources unless forced.  ``emit_defaults`` turns a record
into the compiled-in default table (``csrc/aes_tune_defaults.inc``), so the
library's defaults are the record's winners.

    python -m paper_1902_05234_amd.autotune --out tune.json
    python -m paper_1902_05234_amd.autotune --emit-defaults tuning/mi355x_sweep.json
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

from . import aes, inputs

BPTS = (1, 2, 4)
PLAIN_BPTS = (aes.AES_BPT_COLUMN,) + BPTS  # the plain path also has one column per lane (4 bytes per thread)
WGS = (64, 128, 256, 512, 1024)
PLACEMENTS = (aes.AES_PLACEMENT_TTABLE4, aes.AES_PLACEMENT_TTABLE2, aes.AES_PLACEMENT_TTABLE1,
              aes.AES_PLACEMENT_BITSLICED)
BITSLICE_MAX_WG = 256
# sizes timed for each tuning bucket (bytes; bucket limits in aesgpu.h: 4 KiB,
# 64 KiB, 512 KiB, 2 MiB, 8 MiB, 32 MiB, larger)
BUCKET_SIZES = ((2 << 10, 4 << 10), (16 << 10, 64 << 10), (256 << 10, 512 << 10), (1 << 20, 2 << 20),
                (3 << 20, 8 << 20), (12 << 20, 32 << 20), (256 << 20,))


HERE = os.path.dirname(os.path.abspath(__file__))
RECORD = os.path.join(HERE, "tuning", "mi355x_sweep.json")
DEFAULTS_INC = os.path.join(HERE, "csrc", "aes_tune_defaults.inc")


# Kernels whose timings a record holds: the plain ECB kernels (every table
# placement, one column per lane, bitsliced) with their dispatcher, and,
# tuned apart, the batched kernel.  The record's source hash covers the plain
# kernels' files and the csrc headers they include, followed transitively;
# its batch entry carries the same hash of the batched kernel's files.  Other
# device code (CTR, CBC, probes), host code and the public header do not
# change those timings.
PLAIN_KERNELS = ("aes_ecb.hip", "aes_ecb_p4.hip", "aes_ecb_p2.hip", "aes_ecb_p1.hip", "aes_ecb_col.hip",
                 "aes_bitslice.hip")
BATCH_KERNELS = ("aes_batch.hip",)


def tuned_sources(kernels=PLAIN_KERNELS) -> list:
    """``kernels`` and every csrc header they include (transitively)."""
    csrc = os.path.join(HERE, "csrc")
    seen, todo = set(), list(kernels)
    while todo:
        f = todo.pop()
        if f in seen:
            continue
        seen.add(f)
        with open(os.path.join(csrc, f)) as fh:
            text = fh.read()
        for m in re.finditer(r'^\s*#\s*include\s+"([^"/]+)"', text, re.M):
            if os.path.exists(os.path.join(csrc, m.group(1))):
                todo.append(m.group(1))
    return sorted(seen)


def source_hash(kernels=PLAIN_KERNELS) -> str:
    """Hash of the device code that timings of ``kernels`` depend on
    (tuned_sources); the default is the plain kernels'."""
    h = hashlib.sha256()
    for f in tuned_sources(kernels):
        h.update(f.encode())
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


GRAPH_TIMED_MAX = 64 << 20  # below this the host's per-call cost would dominate an eager timing
GRAPH_LAUNCHES = 20
SUSTAINED_TOP = 8           # variants re-timed under sustained load in the largest bucket
SUSTAINED_SECONDS = 0.5     # back-to-back load per variant per pass (after 0.3 s of warm-up)
SUSTAINED_PASSES = 2


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


def _sustained_gbps(torch, fn, nbytes, seconds=SUSTAINED_SECONDS, warm_s=0.3):
    """GB/s of fn launched back to back for ``seconds`` after ``warm_s`` of
    the same load (events on the launch stream around the timed launches)."""
    fn()
    torch.cuda.synchronize()
    t_end = time.perf_counter() + warm_s
    while time.perf_counter() < t_end:
        fn()
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    k = 0
    a.record(s)
    t_end = time.perf_counter() + seconds
    while time.perf_counter() < t_end:
        for _ in range(4):
            fn()
        k += 4
    b.record(s)
    torch.cuda.synchronize()
    return nbytes * k / (a.elapsed_time(b) * 1e-3) / 1e9


def _time(torch, fn, reps):
    ms = sorted(_times(torch, fn, reps))
    return ms[len(ms) // 2]


def variants(log=None):
    """The search space.  The bitsliced placement always takes 32 blocks per
    lane (bpt does not apply) and at most 256-thread workgroups; the
    combinations it cannot run are skipped and logged once."""
    skipped = []
    for p in PLACEMENTS:
        for b in PLAIN_BPTS:
            for w in WGS:
                if p == aes.AES_PLACEMENT_BITSLICED and (b != 1 or w > BITSLICE_MAX_WG):
                    skipped.append((p, b, w))
                    continue
                yield aes.Variant(bpt=b, wg=w, placement=p)
    if log is not None and skipped:
        log("  skipped %d bitsliced combinations (bpt does not apply; wg <= %d)" % (len(skipped), BITSLICE_MAX_WG))


def tune_plain(torch, keybits: int, decrypt: bool, nbytes: int, reps: int = 10, rounds: int = 3, log=print,
               sustained_top: int = SUSTAINED_TOP):
    """Time every variant on one (key size, direction, size); returns rows
    sorted by time.  The variants are timed in ``rounds`` interleaved passes
    (reps launches each) and ranked by the median over all launches, so a
    drift of the engine clock during the sweep does not favour whichever
    variant ran first.  Up to 64 MiB a launch is timed inside a replayed HIP
    graph, which leaves the host's per-call cost out.  Above that the
    ``sustained_top`` fastest variants of this screen are timed again over
    seconds of back-to-back launches (SUSTAINED_PASSES interleaved passes)
    and only they are ranked, by their sustained rate; the other rows keep
    their screen timings ("timing": "screen") and cannot win."""
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
        rows.append({"bpt": v.bpt, "wg": v.wg, "placement": v.placement, "ms": ms, "GB_s": nbytes / (ms * 1e-3) / 1e9,
                     "timing": "graph" if nbytes <= GRAPH_TIMED_MAX else "screen"})
    rows.sort(key=lambda r: r["ms"])
    if nbytes > GRAPH_TIMED_MAX:
        # the library runs this bucket back to back: re-time the best few
        # under sustained load, interleaved, and rank them by that alone
        top = rows[:sustained_top]
        rates = {i: [] for i in range(len(top))}
        for _ in range(SUSTAINED_PASSES):
            for i, r in enumerate(top):
                v = aes.Variant(r["bpt"], r["wg"], r["placement"])
                rates[i].append(_sustained_gbps(
                    torch, lambda v=v: aes.aes_ecb_crypt_variant(rk, ks.nr, decrypt, x, out, v), nbytes))
        sustained = []
        for i, r in enumerate(top):
            g = sorted(rates[i])[len(rates[i]) // 2] if len(rates[i]) % 2 else sum(rates[i]) / len(rates[i])
            sustained.append(dict(r, GB_s=g, ms=nbytes / (g * 1e9) * 1e3, timing="sustained",
                                  screen_GB_s=r["GB_s"], passes_GB_s=[round(v, 1) for v in rates[i]]))
        sustained.sort(key=lambda r: r["ms"])
        rows = sustained + rows[sustained_top:]
    log("  %d-bit %s %d B: best bpt=%d wg=%d placement=%d %.1f GB/s (%s; worst %.1f)" % (
        keybits, "dec" if decrypt else "enc", nbytes, rows[0]["bpt"], rows[0]["wg"], rows[0]["placement"],
        rows[0]["GB_s"], rows[0]["timing"], rows[-1]["GB_s"]))
    return rows


BATCH_CHUNKS = (256, 1024, 2048, 4096)
BATCH_WGS = (256, 512, 1024)
BATCH_PLACEMENTS = (aes.AES_PLACEMENT_TTABLE4, aes.AES_PLACEMENT_TTABLE2, aes.AES_PLACEMENT_TTABLE1)


def batch_variants():
    """The batched search space: chunk x bytes per thread x workgroup x placement."""
    for chunk in BATCH_CHUNKS:
        for p in BATCH_PLACEMENTS:
            for wg in BATCH_WGS:
                for bpt in BPTS:
                    yield chunk, aes.BatchConfig(bpt=bpt, wg=wg, placement=p)


def tune_batch(torch, n_messages: int = 20000, reps: int = 3, rounds: int = 2, log=print):
    """Time every batch variant on the mixed workload (20,000 messages, own
    key and key size each, half encrypt, half decrypt), in ``rounds``
    interleaved passes.  The first variant's output is checked against one
    plain-kernel launch per message, and every other variant against that
    output, bit for bit, before anything is timed."""
    from . import batch
    mix = inputs.message_mix(2, n_messages)
    keys = [inputs.random_key(int(s), int(b)) for s, b in zip(mix.key_seed, mix.keybits)]
    kt = batch.key_table(keys)
    in_arena = inputs.device_random_bytes(2, 16 * mix.total_blocks)
    out_arena = torch.empty_like(in_arena)
    msgs = batch.messages_from_mix(mix)
    ref = torch.zeros_like(in_arena)
    batch.run_per_message(msgs, [aes.aes_expand_key(k) for k in keys], in_arena, ref)
    torch.cuda.synchronize()
    vs = list(batch_variants())
    prepared = []
    for chunk, cfg in vs:
        b = batch.prepare(msgs, kt, in_arena, out_arena, chunk_blocks=chunk, cfg=cfg)
        out_arena.zero_()
        b.launch()
        torch.cuda.synchronize()
        if b.rejected_items() or not torch.equal(out_arena, ref):
            raise RuntimeError("batch chunk=%d %s differs from the per-message plain launches" % (chunk, cfg))
        prepared.append(b)
        if len(prepared) % 12 == 0:
            log("  batch variants checked: %d of %d" % (len(prepared), len(vs)))
    del ref
    times = {i: [] for i in range(len(vs))}
    for r in range(max(1, rounds)):
        for i, b in enumerate(prepared):
            times[i] += _times(torch, b.launch, reps)
        log("  batch timing pass %d of %d done" % (r + 1, max(1, rounds)))
    rows = []
    for i, (chunk, cfg) in enumerate(vs):
        t = sorted(times[i])
        ms = t[len(t) // 2]
        rows.append({"chunk_blocks": chunk, "bpt": cfg.bpt, "wg": cfg.wg, "placement": cfg.placement, "ms": ms,
                     "GB_s": prepared[i].total_bytes / (ms * 1e-3) / 1e9})
    rows.sort(key=lambda r: r["ms"])
    for r in rows[:5]:
        log("  batch chunk=%d bpt=%d wg=%d placement=%d: %.1f GB/s" % (
            r["chunk_blocks"], r["bpt"], r["wg"], r["placement"], r["GB_s"]))
    w = rows[0]
    return {"source_hash": source_hash(BATCH_KERNELS), "created": time.strftime("%Y-%m-%dT%H:%M:%S"),
            "winner": {k: w[k] for k in ("chunk_blocks", "bpt", "wg", "placement")}, "GB_s": round(w["GB_s"], 1),
            "messages": n_messages, "bytes": prepared[0].total_bytes, "all": rows}


def batch_winner(record: dict):
    """(chunk_blocks, BatchConfig) of a record's batched winner, or None when
    the record has none or timed other batch-kernel sources."""
    b = record.get("batch")
    if not isinstance(b, dict) or "winner" not in b or b.get("source_hash") != source_hash(BATCH_KERNELS):
        return None
    w = b["winner"]
    return w["chunk_blocks"], aes.BatchConfig(bpt=w["bpt"], wg=w["wg"], placement=w["placement"])


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


def device_identity(torch=None):
    """(name, architecture) of the current device."""
    if torch is None:
        import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return p.name, getattr(p, "gcnArchName", "")


def run(buckets=BUCKET_SIZES, key_sizes=(128, 192, 256), batch_too=True, reps=10, rounds=3, log=print):
    """buckets: one tuple of sizes per tuning bucket (the library's bucket of
    each tuple's sizes must agree)."""
    import torch
    name, arch = device_identity(torch)
    rec = {"device": name, "arch": arch, "source_hash": source_hash(), "hip": torch.version.hip,
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


class RecordMismatch(RuntimeError):
    """A tuning record made on another device or for other kernel sources."""


def record_mismatch(record: dict, device=None, arch=None, src_hash=None, hip=None):
    """Reasons the record does not describe this device, runtime and these
    kernels (empty when it does).  device/arch: the current device's name and
    architecture; hip: the HIP runtime version the timings ran under (None:
    not checked); src_hash: defaults to source_hash()."""
    why = []
    want = source_hash() if src_hash is None else src_hash
    if record.get("source_hash") != want:
        why.append("made for kernel sources %s, these are %s" % (record.get("source_hash"), want))
    if device is not None and record.get("device") != device:
        why.append("made on device %r, this is %r" % (record.get("device"), device))
    if arch is not None and record.get("arch") is not None and record.get("arch") != arch:
        why.append("made for architecture %r, this is %r" % (record.get("arch"), arch))
    if hip is not None and record.get("hip") is not None and record.get("hip") != hip:
        why.append("timed under HIP runtime %s, this is %s" % (record.get("hip"), hip))
    return why


def winners(record: dict):
    """{(nr, decrypt, bucket): (bpt, wg, placement)} of a record's plain path."""
    out = {}
    for k, v in record.get("plain", {}).items():
        kb, d, nbytes = k.split("/")
        sizes = v.get("sizes") or [int(nbytes)]
        bucket = aes.aes_size_bucket(max(sizes) // 16)
        w = v["winner"]
        out[({128: 10, 192: 12, 256: 14}[int(kb)], d == "dec", bucket)] = (w["bpt"], w["wg"], w["placement"])
    return out


def apply(record: dict, force: bool = False):
    """Install the plain-path winners of a record into the library's tuning
    table.  A record made on another device or architecture, under another
    HIP runtime, or for other kernel sources, is refused (RecordMismatch)
    unless ``force``."""
    if not force:
        try:
            import torch
            name, arch = device_identity(torch)
            hip = torch.version.hip
        except Exception:  # no device to compare with: only the sources are checked
            name = arch = hip = None
        why = record_mismatch(record, name, arch, hip=hip)
        if why:
            raise RecordMismatch("tuning record refused (%s); pass force=True to install it anyway" % "; ".join(why))
    n = 0
    for (nr, dec, bucket), (bpt, wg, pl) in winners(record).items():
        aes.aes_tune_set(nr, dec, _bucket_size(bucket), aes.Variant(bpt, wg, pl))
        n += 1
    return n


def _bucket_size(bucket: int) -> int:
    """A block count that lies in tuning bucket ``bucket``."""
    return BUCKET_SIZES[bucket][-1] // 16


def emit_defaults(record: dict) -> str:
    """The compiled-in default table (csrc/aes_tune_defaults.inc) that
    reproduces a record's plain-path winners, one entry per key size,
    direction and size bucket."""
    w = winners(record)
    lines = ["// aes_tune_defaults.inc -- generated by `python -m paper_1902_05234_amd.autotune",
             "// --emit-defaults` from tuning/%s (device %s, kernel sources %s, %s);" % (
                 os.path.basename(RECORD), record.get("device"), record.get("source_hash"), record.get("created")),
             "// do not edit: regenerate it from a new record instead.",
             "// kTuneDefaults[nr index][decrypt][size bucket] = {bytes per thread / 16, workgroup, placement}",
             "static constexpr TuneDefault kTuneDefaults[3][2][AES_SIZE_BUCKETS] = {"]
    for ni, nr in enumerate((10, 12, 14)):
        lines.append("    {  // Nr = %d" % nr)
        for dec in (False, True):
            cells = []
            for b in range(aes.AES_SIZE_BUCKETS):
                if (nr, dec, b) not in w:
                    raise ValueError("record has no winner for Nr=%d %s bucket %d" % (nr, "dec" if dec else "enc", b))
                cells.append("{%d, %d, %d}" % w[(nr, dec, b)])
            lines.append("        {%s},  // %s" % (", ".join(cells), "decrypt" if dec else "encrypt"))
        lines.append("    },")
    lines.append("};")
    return "\n".join(lines) + "\n"


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
    ap.add_argument("--buckets", default=None,
                    help="comma-separated bucket indices to tune (all key sizes and directions); the results "
                         "replace those buckets' entries of the record given by --merge")
    ap.add_argument("--merge", default=None, help="record to update with --buckets (same kernel sources)")
    ap.add_argument("--batch-only", action="store_true",
                    help="tune the batched mix only and store it into the record given by --out (which must exist)")
    ap.add_argument("--emit-defaults", metavar="RECORD", default=None,
                    help="write csrc/aes_tune_defaults.inc from RECORD (no GPU needed) and exit")
    a = ap.parse_args(argv)
    log = lambda *x: print(*x, file=sys.stderr, flush=True)
    if a.emit_defaults:
        with open(DEFAULTS_INC, "w") as f:
            f.write(emit_defaults(load(a.emit_defaults)))
        log("wrote", DEFAULTS_INC)
        return
    if a.buckets is not None:
        rec = load(a.merge)
        if rec.get("source_hash") != source_hash():
            raise SystemExit("%s was made for kernel sources %s, these are %s: tune everything again" % (
                a.merge, rec.get("source_hash"), source_hash()))
        idx = [int(b) for b in a.buckets.split(",") if b]
        part = run(buckets=tuple(BUCKET_SIZES[b] for b in idx), batch_too=False, reps=a.reps, rounds=a.rounds, log=log)
        for k in list(rec["plain"]):
            if aes.aes_size_bucket(max(rec["plain"][k].get("sizes") or [int(k.split("/")[2])]) // 16) in idx:
                del rec["plain"][k]
        rec["plain"].update(part["plain"])
        rec["merged"] = rec.get("merged", []) + [{"buckets": idx, "created": part["created"]}]
        with open(a.out, "w") as f:
            json.dump(rec, f, indent=1)
        log("wrote", a.out)
        return
    if a.batch_only:
        import torch
        rec = load(a.out)
        name, arch = device_identity(torch)
        if (rec.get("device"), rec.get("arch")) != (name, arch):
            raise SystemExit("%s was made on %s (%s), this is %s (%s): tune everything again" % (
                a.out, rec.get("device"), rec.get("arch"), name, arch))
        rec["batch"] = tune_batch(torch, log=log)
        with open(a.out, "w") as f:
            json.dump(rec, f, indent=1)
        log("wrote", a.out)
        return
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
