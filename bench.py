#!/usr/bin/env python3
"""Benchmark of the AES-ECB hot path on one MI355X.

One step = expand the key (host), encrypt a 1 GiB device buffer with
AES-128 ECB, decrypt the ciphertext again (two launches of the plain
persistent kernels).  Inputs are seeded synthetic bytes resident in HBM
before timing starts.  Prints ONE JSON line:

  value        whole-step throughput, 10^9 payload bytes per second
               (encrypt + decrypt bytes / wall time of the timed steps)
  roofline     the encrypt kernel against the LDS lookup roof (the binding
               unit: 16 table lookups per block per round), with the HBM and
               VALU roofs beside it, the HBM bytes rocprofv3 counted, and the
               engine clock, socket power and encryption rate held over 2 s
               of back-to-back load
  cpu_baseline the CPU oracle (byte-wise FIPS-197, all host cores) on a
               bounded slice of the same workload
  batched      20,000 mixed messages in one persistent launch (graph replay)
               vs per-message plain launches and vs the bulk-equivalent rate
  sweep        GB/s for every key size and direction, 1 MiB ... 4 GiB (device
               time: graph replays up to 64 MiB, event-timed launches above), plus
               an all-zero control, CTR and CBC decryption at 1 GiB, and CBC
               encryption and decryption of 1 GiB as 2^18 independent 4 KiB
               messages
  host_path    the paper's file sizes (1,202 ... 1,190,402 bytes) host buffer
               in, host buffer out (host-link transfers included), pinned and
               pageable, beside the paper's own GPU times; and the 1 GiB
               pinned rate
  serving      open-loop Poisson requests (80 % 64 B-16 KiB, 20 % 1-64 MiB,
               4,096 resident keys, 32 GiB device budget, 20,000 requests per
               level) at offered loads rho x the batched rate: p50/p99 latency
               and sustained GB/s; the engine's capacity under overload; 2000
               served requests checked against each request run alone

Flags: --gpus N (only 1 is supported), --steps K (default 100), --warmup W
(default 30) plus --warmup-seconds S (default 1: warm-up continues until S
seconds of back-to-back steps have passed), --no-batch / --no-sweep / --no-cpu / --no-host / --no-serve to
skip sections, --profile to run only a few bulk and copy launches (for
rocprofv3).
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import platform
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

GiB = 1 << 30
MiB = 1 << 20

# MI355X published figures (gfx950): 256 CUs at 2.4 GHz peak engine clock.
MI355X_CUS = 256
MI355X_CLOCK_HZ = 2.4e9
HBM_PEAK_BPS = 8.0e12
LDS_LOOKUPS_PER_CLK_PER_CU = 32          # 32 banks x 4 B per clock, one ds_read_b32 lane each
VALU_LANE_OPS_PER_CLK_PER_CU = 128       # fp32 vector peak 157.3 TFLOP/s = 2 x 78.6 T lane-ops/s
LDS_PEAK = MI355X_CUS * MI355X_CLOCK_HZ * LDS_LOOKUPS_PER_CLK_PER_CU     # 19.66 T lookups/s
VALU_PEAK = MI355X_CUS * MI355X_CLOCK_HZ * VALU_LANE_OPS_PER_CLK_PER_CU  # 78.6 T lane-ops/s


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def lookups_per_block(nr: int) -> int:
    return 16 * nr                      # 16 per inner round + 16 in the final round


def valu_floor_per_block(nr: int) -> int:
    return 24 * nr + 12                 # address/byte-select + XOR3 + final merge


# Sources that hold the device code of the plain ECB kernels; a traffic
# figure taken on other versions of these is not reused.
KERNEL_SOURCES = ["aes_device.hpp", "aes_tables.hpp", "aes_ecb_kernel.hpp", "aes_ecb_p4.hip", "aes_ecb_p2.hip",
                  "aes_ecb_p1.hip"]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1902_05234_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def kernel_instance(v) -> str:
    """Template instance of the AES-128 encrypt kernel for variant v, as the
    profiler names it."""
    return "ecb_kernel<10, false, %d, %d>" % (v.bpt, v.placement)


def read_traffic(nbytes_payload: int, instance: str):
    """HBM bytes per encrypt launch from the committed rocprofv3 PMC summary,
    or None if it is missing, was taken on other kernel sources or on another
    kernel instance than the one the tuning table picks."""
    path = os.path.join(ROOT, "profiles", "aes128_ecb_encrypt_1GiB_pmc.txt")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    m = re.search(r"kernel_source_hash:\s*(\w+)", text)
    t = re.search(r"hbm_bytes_per_launch:\s*([0-9.eE+]+)", text)
    k = re.search(r"kernel_instance:\s*(.+)", text)
    if not m or not t or not k or m.group(1) != kernel_source_hash() or k.group(1).strip() != instance:
        return None
    return float(t.group(1))


class Timer:
    """HIP events on the stream the kernels are launched on.  `prepare` pairs
    are created up front, so a timed loop of that many launches only records
    them; further pairs are created as needed."""

    def __init__(self, torch, prepare=0):
        self.torch = torch
        self.free = [self._pair() for _ in range(prepare)]
        self.pairs = []

    def _pair(self):
        return self.torch.cuda.Event(enable_timing=True), self.torch.cuda.Event(enable_timing=True)

    def run(self, fn):
        s = self.torch.cuda.current_stream()
        a, b = self.free.pop() if self.free else self._pair()
        a.record(s)
        fn()
        b.record(s)
        self.pairs.append((a, b))

    def ms(self):
        self.torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in self.pairs]


def bulk(torch, aes, inputs, args):
    nbytes = GiB
    key = inputs.random_key(1, 128)
    x = inputs.device_random_bytes(1, nbytes)
    c = torch.empty_like(x)
    p = torch.empty_like(x)
    t_enc, t_dec = Timer(torch, args.steps), Timer(torch, args.steps)

    def step(timed: bool):
        ks = aes.aes_expand_key(key)
        if timed:
            t_enc.run(lambda: aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, x, c))
            t_dec.run(lambda: aes.aes_ecb_decrypt(ks.rk_dec, ks.nr, c, p))
        else:
            aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, x, c)
            aes.aes_ecb_decrypt(ks.rk_dec, ks.nr, c, p)

    # Warm-up: at least --warmup steps, then more back-to-back steps until
    # --warmup-seconds of load have passed.  The engine clock ramps up from
    # idle and then settles under sustained load over a few hundred ms, so a
    # count of steps alone (a few ms at 1 GiB) would time the ramp.  The host
    # syncs every 10 steps only to read the clock.
    tw = time.perf_counter()
    warm_steps = 0
    while warm_steps < args.warmup or time.perf_counter() - tw < args.warmup_seconds:
        for _ in range(10 if warm_steps >= args.warmup else 1):
            step(False)
            warm_steps += 1
        if warm_steps >= args.warmup:
            torch.cuda.synchronize()
    # The timed steps follow the warm-up directly: an idle gap would let the
    # engine clock settle again and the first timed launches would pay its
    # ramp.  The round trip is checked on the output of the timed steps.
    torch.cuda.synchronize()
    warm_s = time.perf_counter() - tw
    gc.disable()  # no collector pause between launches inside the timed region
    try:
        t0 = time.perf_counter()
        for _ in range(args.steps):
            step(True)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
    finally:
        gc.enable()
    if not torch.equal(p, x):
        raise RuntimeError("round trip failed on the 1 GiB buffer")
    enc_ms, dec_ms = t_enc.ms(), t_dec.ms()
    return dict(key=key, x=x, c=c, nbytes=nbytes, elapsed=elapsed, enc_ms=enc_ms, dec_ms=dec_ms,
                warmup_steps=warm_steps, warmup_ms=warm_s * 1e3)


def launch_stats(ms):
    """Mean and median of per-launch durations (ms)."""
    s = sorted(ms)
    return {"mean_ms": round(sum(s) / len(s), 4), "median_ms": round(s[len(s) // 2], 4), "launches": len(s)}


def roofline(b, traffic, aes):
    nblocks = b["nbytes"] // 16
    v = aes.aes_tune_get(10, False, nblocks)
    places = {0: "4 tables", 1: "2 tables", 2: "1 table"}
    t = sum(b["enc_ms"]) / len(b["enc_ms"]) * 1e-3
    td = sum(b["dec_ms"]) / len(b["dec_ms"]) * 1e-3
    nr = 10
    lookups = lookups_per_block(nr) * nblocks
    ach = lookups / t / 1e9
    ach_d = lookups / td / 1e9
    peak = LDS_PEAK / 1e9
    hbm_alg = 32 * nblocks
    vd = aes.aes_tune_get(10, True, nblocks)
    return {
        "kernel": "ecb_kernel<Nr=10, encrypt, %d B/thread, %s in LDS, %d-thread workgroups>" % (
            16 * v.bpt, places.get(v.placement, "?"), v.wg),
        "bound": "lds",
        "achieved": round(ach, 1),
        "peak": round(peak, 1),
        "unit": "Glookup/s",
        "frac": round(ach / peak, 4),
        "traffic": traffic,
        "per_launch": {"blocks": nblocks, "lookups": lookups, "hbm_bytes_algorithmic": hbm_alg,
                       "avg_ms": round(t * 1e3, 4), **launch_stats(b["enc_ms"])},
        "decrypt": {"kernel": "ecb_kernel<Nr=10, decrypt, %d B/thread, %s in LDS, %d-thread workgroups>" % (
                        16 * vd.bpt, places.get(vd.placement, "?"), vd.wg),
                    "achieved": round(ach_d, 1), "peak": round(peak, 1), "unit": "Glookup/s",
                    "frac": round(ach_d / peak, 4), "avg_ms": round(td * 1e3, 4), **launch_stats(b["dec_ms"])},
        "roofs": {
            "lds": {"achieved_Glookup_s": round(ach, 1), "peak": round(peak, 1), "frac": round(ach / peak, 4)},
            "hbm": {"achieved_GB_s": round(hbm_alg / t / 1e9, 1), "peak": HBM_PEAK_BPS / 1e9,
                    "frac": round(hbm_alg / t / HBM_PEAK_BPS, 4)},
            "valu_floor": {"achieved_Tlane_op_s": round(valu_floor_per_block(nr) * nblocks / t / 1e12, 2),
                           "peak": round(VALU_PEAK / 1e12, 1),
                           "frac": round(valu_floor_per_block(nr) * nblocks / t / VALU_PEAK, 4)},
            "payload_roof_GB_s": round(min(LDS_PEAK * 16 / lookups_per_block(nr), HBM_PEAK_BPS / 2,
                                           VALU_PEAK * 16 / valu_floor_per_block(nr)) / 1e9, 1),
        },
    }


def openssl_context(cores):
    """`openssl speed` for AES-128-ECB on 16 KiB buffers (AES-NI), one thread and
    all host threads: a labelled fast-CPU context line, not the baseline."""
    import subprocess
    out = {}
    for label, extra in (("one_thread", []), ("all_threads", ["-multi", str(cores)])):
        try:
            r = subprocess.run(["openssl", "speed"] + extra + ["-evp", "aes-128-ecb", "-bytes", "16384", "-seconds", "1"],
                               capture_output=True, text=True, timeout=60)
        except (OSError, subprocess.TimeoutExpired):
            return None
        rate = None
        for line in r.stdout.splitlines():
            parts = line.split()
            if len(parts) == 2 and parts[0] in ("AES-128-ECB", "evp") and parts[1].endswith("k"):
                rate = float(parts[1][:-1]) * 1e3
        if rate is None:
            return None
        out[label + "_GB_s"] = round(rate / 1e9, 3)
    out["threads"] = cores
    out["what"] = "openssl speed -evp aes-128-ecb -bytes 16384 (AES-NI; context, not the oracle baseline)"
    return out


def clock_under_load(torch, aes, b, seconds=2.0):
    """Engine clock and socket power while the bulk encryption runs back to
    back for `seconds` (after the timed steps): `rocm-smi --showclocks` and
    `amd-smi metric -p`, sampled every 0.25 s from a thread.  None if the
    tools are missing.  Context for the roofline: the published LDS peak
    assumes 2.4 GHz."""
    import shutil
    import subprocess
    import threading
    if not shutil.which("rocm-smi"):
        return None
    samples, stop = [], threading.Event()

    def sample():
        while not stop.is_set():
            clk = pw = None
            try:
                r = subprocess.run(["rocm-smi", "--showclocks", "--json"], capture_output=True, text=True, timeout=5)
                card = json.loads(r.stdout)
                card = card[sorted(card)[0]]
                clk = int(card["sclk clock speed:"].strip("()Mhz"))
            except Exception:
                pass
            try:
                r = subprocess.run(["amd-smi", "metric", "-p"], capture_output=True, text=True, timeout=5)
                pw = float(r.stdout.split("SOCKET_POWER:")[1].split()[0])
            except Exception:
                pass
            samples.append((clk, pw))
            stop.wait(0.25)

    ks = aes.aes_expand_key(b["key"])
    th = threading.Thread(target=sample)
    th.start()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    launches = 0
    t0 = time.perf_counter()
    ev0.record()
    while time.perf_counter() - t0 < seconds:
        for _ in range(10):
            aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, b["x"], b["c"])
        launches += 10
        torch.cuda.synchronize()
    ev1.record()
    torch.cuda.synchronize()
    stop.set()
    th.join()
    # throughput over the whole window (the host syncs every 10 launches, a
    # gap of microseconds per ~7 ms): the rate the clock settles at
    sustained = launches * b["x"].numel() / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    clks = [c for c, _ in samples[1:] if c]
    pws = [p for _, p in samples[1:] if p]
    if not clks:
        return None
    mhz = sum(clks) / len(clks)
    return {"sclk_MHz": round(mhz), "socket_power_W": round(sum(pws) / len(pws)) if pws else None,
            "samples": len(clks), "lds_roof_at_clock_Glookup_s": round(LDS_PEAK / 1e9 * mhz * 1e6 / MI355X_CLOCK_HZ, 1),
            "encrypt_GB_s": round(sustained, 1), "launches": launches,
            "what": "bulk AES-128 encryption of 1 GiB back to back for %.0f s after the timed steps" % seconds}


def measured_roofs(torch, aes, inputs):
    """The probes of the roofs: a 1 GiB device copy (HBM), conflict-free LDS
    lookups at 32 waves per CU, full-rate VALU chains; median of 5 timed
    launches each."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    scratch = torch.empty(cus * 2048, dtype=torch.int32, device="cuda")
    res = {}
    for name, which, iters in (("lds", aes.AES_PROBE_LDS, 20000), ("valu", aes.AES_PROBE_VALU, 20000)):
        work = aes.aes_roof_probe(which, 10, scratch)
        tm = Timer(torch)
        for _ in range(5):
            tm.run(lambda: aes.aes_roof_probe(which, iters, scratch))
        ms = sorted(tm.ms())[2]
        work = aes.aes_roof_probe(which, iters, scratch)
        res[name] = work / (ms * 1e-3)
    x = inputs.device_random_bytes(8, GiB)
    y = torch.empty_like(x)
    aes.aes_device_copy(x, y)
    tm = Timer(torch)
    for _ in range(5):
        tm.run(lambda: aes.aes_device_copy(x, y))
    ms = sorted(tm.ms())[2]
    del x, y
    torch.cuda.empty_cache()
    return {"hbm_copy_GB_s": round(2 * GiB / (ms * 1e-3) / 1e9, 1),
            "lds_Glookup_s": round(res["lds"] / 1e9, 1),
            "valu_Tlane_op_s": round(res["valu"] / 1e12, 2),
            "what": "1 GiB device copy (read + write bytes); conflict-free ds_read_b32 with random per-lane "
                    "entries, 32 waves/CU; independent v_bitop3_b32 chains, 32 waves/CU"}


def cpu_baseline(b, args):
    import numpy as np

    import oracle
    o = oracle.load()
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    probe = b["x"][:MiB].cpu().numpy()
    t0 = time.perf_counter()
    o.ecb_encrypt(b["key"], probe, nthreads=cores)
    dt = max(time.perf_counter() - t0, 1e-6)
    nbytes = int(min(GiB, max(MiB, args.cpu_seconds / 2 / dt * MiB)))
    nbytes -= nbytes % MiB
    xs = b["x"][:nbytes].cpu().numpy()
    t0 = time.perf_counter()
    enc = o.ecb_encrypt(b["key"], xs, nthreads=cores)
    dec = o.ecb_decrypt(b["key"], enc, nthreads=cores)
    dt = time.perf_counter() - t0
    gpu_match = bool(np.array_equal(enc, b["c"][:nbytes].cpu().numpy())) and bool(np.array_equal(dec, xs))
    # one thread on 4 MiB: the figure comparable to a single-core C program
    t1 = time.perf_counter()
    o.ecb_encrypt(b["key"], xs[:4 * MiB], nthreads=1)
    one_thread = 4 * MiB / (time.perf_counter() - t1) / 1e6
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": round(2 * nbytes / dt / 1e9, 6), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": "AES-128 ECB encrypt then decrypt of the first %d MiB of the 1 GiB workload" % (nbytes // MiB),
            "seconds": round(dt, 2), "cpu_model": model or platform.processor(),
            "one_thread_encrypt_MB_s": round(one_thread, 2),
            "openssl_context": openssl_context(cores),
            "matches_gpu_on_sample": gpu_match}


GRAPH_TIMED_MAX = 64 * MiB   # up to this size the host's per-call cost would dominate an eager timing
GRAPH_LAUNCHES = 20


WARM_SECONDS = 0.05  # the engine clock takes a few tens of ms of load to ramp up from idle
WARM_SECONDS_LARGE = 0.25  # long launches: load long enough for the clock to settle, as in the bulk warm-up


def warm(torch, fn, seconds=WARM_SECONDS):
    """Run fn back to back, with no synchronisation in between, for about
    `seconds` before a timing (the timed launches are back to back too)."""
    t0 = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    one = max(time.perf_counter() - t0, 1e-6)
    for _ in range(max(1, min(4000, int(seconds / one)))):
        fn()
    torch.cuda.synchronize()


def launch_ms(torch, fn, n):
    """Device time of one launch of fn on an n-byte buffer, after a warm-up.
    Small buffers: 20 launches captured in a HIP graph, replayed 5 times
    (median replay / 20), so the host's per-call cost stays out of the figure;
    large buffers: HIP events around single eager launches (median)."""
    fn()
    torch.cuda.synchronize()
    if n <= GRAPH_TIMED_MAX:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(GRAPH_LAUNCHES):
                fn()
        warm(torch, g.replay)
        tm = Timer(torch)
        for _ in range(5):
            tm.run(g.replay)
        ms = sorted(tm.ms())[2] / GRAPH_LAUNCHES
        del g
        return ms
    warm(torch, fn, WARM_SECONDS_LARGE)
    reps = max(5, min(50, int(8 * GiB / n)))
    tm = Timer(torch)
    for _ in range(reps):
        tm.run(fn)
    return sorted(tm.ms())[reps // 2]


def cbc_records(ms):
    """aes_cbc_msg records (aes.CBC_MSG_DTYPE) of a CBC message set."""
    from paper_1902_05234_amd import aes
    recs = np.zeros(len(ms), dtype=aes.CBC_MSG_DTYPE)
    recs["in_block"], recs["out_block"], recs["nblocks"], recs["iv"] = ms.in_block, ms.out_block, ms.nblocks, ms.iv
    return recs


def sweep(torch, aes, inputs, sizes):
    out = {}
    buf_in = inputs.device_random_bytes(3, max(sizes))
    buf_out = torch.empty_like(buf_in)
    for keybits in (128, 192, 256):
        ks = aes.aes_expand_key(inputs.random_key(3, keybits))
        for dec in (False, True):
            for n in sizes:
                xi, xo = buf_in[:n], buf_out[:n]
                fn = (lambda: aes.aes_ecb_decrypt(ks.rk_dec, ks.nr, xi, xo)) if dec else \
                     (lambda: aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, xi, xo))
                ms = launch_ms(torch, fn, n)
                out["aes%d_%s_%s" % (keybits, "dec" if dec else "enc", size_name(n))] = round(n / (ms * 1e-3) / 1e9, 1)
    ks = aes.aes_expand_key(inputs.random_key(3, 128))
    n = min(GiB, max(sizes))
    xi, xo = buf_in[:n], buf_out[:n]

    def timed10(fn):
        warm(torch, fn, WARM_SECONDS_LARGE)
        tm = Timer(torch)
        for _ in range(10):
            tm.run(fn)
        return sorted(tm.ms())[5]

    # counter mode: same round core; the lookups depend on the counters only
    ms = timed10(lambda: aes.aes_ctr_crypt(ks.rk_enc, ks.nr, bytes(range(16)), 0, xi, xo))
    out["aes128_ctr_%s" % size_name(n)] = round(n / (ms * 1e-3) / 1e9, 1)
    # CBC decryption (random ciphertext): ECB decryption plus the XOR of the
    # preceding ciphertext block
    ms = timed10(lambda: aes.aes_cbc_decrypt(ks.rk_dec, ks.nr, bytes(16), xi, xo))
    out["aes128_cbc_dec_%s" % size_name(n)] = round(n / (ms * 1e-3) / 1e9, 1)
    # CBC encryption across independent messages: the buffer as 4 KiB
    # messages (one chain per lane, 2^18 of them at 1 GiB), each with its own
    # initialisation vector
    nm = n // 4096
    msgs = torch.from_numpy(cbc_records(inputs.cbc_equal_messages(3, nm, 256)).view(np.uint8)).to("cuda")
    ms = timed10(lambda: aes.aes_cbc_encrypt_msgs(ks.rk_enc, ks.nr, msgs, nm, xi, xo))
    out["aes128_cbc_enc_4KiB_msgs_%s" % size_name(n)] = round(n / (ms * 1e-3) / 1e9, 1)
    ms = timed10(lambda: aes.aes_cbc_decrypt_msgs(ks.rk_dec, ks.nr, msgs, nm, xi, xo))
    out["aes128_cbc_dec_4KiB_msgs_%s" % size_name(n)] = round(n / (ms * 1e-3) / 1e9, 1)
    del msgs
    # structured control, last because it overwrites the input: in an
    # all-zero buffer every block is the same, so every lane reads the same
    # table entry in every round (LDS broadcast); random data spreads the
    # lanes over the 32 replicas
    xi.zero_()
    ms = timed10(lambda: aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, xi, xo))
    out["aes128_enc_%s_all_zero" % size_name(n)] = round(n / (ms * 1e-3) / 1e9, 1)
    del buf_in, buf_out
    torch.cuda.empty_cache()
    return out


def size_name(n):
    return "%dGiB" % (n // GiB) if n >= GiB else "%dMiB" % (n // MiB)


# The paper's GPU times (seconds) per file size, GeForce 940MX, files in host
# memory (section 5, Table 4 encryption, Table 5 decryption): context only.
PAPER_GPU_SECONDS = {
    1202: (0.000732, 0.000771), 4652: (0.000770, 0.000821), 9302: (0.000784, 0.000790),
    18602: (0.000807, 0.000821), 37202: (0.000886, 0.000918), 74402: (0.001048, 0.001040),
    148802: (0.001302, 0.001331), 297602: (0.001896, 0.002018), 595202: (0.003145, 0.003577),
    1190402: (0.005316, 0.005847),
}


def host_sweep(torch, aes, inputs, reps=20):
    """The paper's file sizes through the host-inclusive path (host buffer in,
    host buffer out; AES-128, sizes padded to whole blocks), pinned and
    pageable host buffers, plus one 1 GiB pinned buffer for the rate over the
    host link.  Wall time of the synchronous call, median of reps."""
    ks = aes.aes_expand_key(inputs.random_key(5, 128))
    pipe = aes.HostPipe(chunk_bytes=32 * MiB, nslots=2, staging=True)
    out = {"keybits": 128, "chunk_bytes": 32 * MiB, "nslots": 2, "sizes": []}
    big = max(PAPER_GPU_SECONDS)
    src_pin = torch.from_numpy(inputs.random_bytes(6, (big + 15) // 16 * 16)).pin_memory()
    dst_pin = torch.empty_like(src_pin).pin_memory()
    src_pg = src_pin.numpy().copy()
    dst_pg = np.empty_like(src_pg)

    def timed(op, a, b):
        pipe.run(op, ks, a, out=b)
        t = []
        for _ in range(reps):
            t0 = time.perf_counter()
            pipe.run(op, ks, a, out=b)
            t.append(time.perf_counter() - t0)
        return sorted(t)[reps // 2]

    for size, (p_enc, p_dec) in sorted(PAPER_GPU_SECONDS.items()):
        n = (size + 15) // 16 * 16
        row = {"bytes": size, "padded": n, "paper_940MX_s": {"enc": p_enc, "dec": p_dec}}
        for mode, a, b in (("pinned", src_pin[:n], dst_pin[:n]), ("pageable", src_pg[:n], dst_pg[:n])):
            te = timed(aes.AES_PIPE_ECB_ENCRYPT, a, b)
            td = timed(aes.AES_PIPE_ECB_DECRYPT, a, b)
            row[mode] = {"enc_s": round(te, 7), "dec_s": round(td, 7), "enc_GB_s": round(n / te / 1e9, 3),
                         "dec_GB_s": round(n / td / 1e9, 3)}
        out["sizes"].append(row)
    del src_pin, dst_pin
    # 1 GiB host-resident, pinned: the rate over the host link (not the headline value)
    x = torch.from_numpy(inputs.random_bytes(7, 64 * MiB)).repeat(16).pin_memory()
    y = torch.empty_like(x).pin_memory()
    pipe.run(aes.AES_PIPE_ECB_ENCRYPT, ks, x, out=y)
    ts = []
    for _ in range(5):
        t0 = time.perf_counter()
        pipe.run(aes.AES_PIPE_ECB_ENCRYPT, ks, x, out=y)
        ts.append(time.perf_counter() - t0)
    out["pinned_1GiB_encrypt_GB_s"] = round(GiB / sorted(ts)[2] / 1e9, 2)
    pipe.close()
    return out


def batched(torch, aes, inputs, bulk_rates):
    from paper_1902_05234_amd import batch
    mix = inputs.message_mix(2, 20000)
    keys = [inputs.random_key(int(s), int(b)) for s, b in zip(mix.key_seed, mix.keybits)]
    kt = batch.key_table(keys)
    total = mix.total_blocks
    in_arena = inputs.device_random_bytes(2, 16 * total)
    out_arena = torch.empty_like(in_arena)
    # work-item size and batch kernel variant: the autotune record's winner
    # (the library's default shape if the record timed other batch-kernel sources)
    from paper_1902_05234_amd import autotune
    won = autotune.batch_winner(autotune.load(autotune.RECORD))
    chunk, cfg = won if won else (2048, aes.BatchConfig())
    b = batch.prepare(batch.messages_from_mix(mix), kt, in_arena, out_arena, chunk_blocks=chunk, cfg=cfg)
    b.capture()
    warm(torch, b.replay)
    tm = Timer(torch)
    for _ in range(5):
        tm.run(b.replay)
    ms = sorted(tm.ms())[2]
    nbytes = 16 * total
    batched_gbps = nbytes / (ms * 1e-3) / 1e9
    # per-message plain launches, same arenas, same bytes
    scheds = [aes.aes_expand_key(k) for k in keys]
    batch.run_per_message(b.msgs, scheds, in_arena, out_arena)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.run_per_message(b.msgs, scheds, in_arena, out_arena)
    torch.cuda.synchronize()
    per_msg_s = time.perf_counter() - t0
    # bulk-equivalent: each (key size, direction) share at its 1 GiB bulk rate
    t_eq = 0.0
    for kb in (128, 192, 256):
        for dec in (False, True):
            sel = (mix.keybits == kb) & (mix.decrypt == dec)
            t_eq += 16 * int(mix.nblocks[sel].sum()) / (bulk_rates["aes%d_%s_1GiB" % (kb, "dec" if dec else "enc")] * 1e9)
    bulk_eq = nbytes / t_eq / 1e9
    return {"messages": len(mix), "bytes": nbytes, "GB_s": round(batched_gbps, 1), "ms": round(ms, 3),
            "bulk_equivalent_GB_s": round(bulk_eq, 1), "vs_bulk": round(batched_gbps / bulk_eq, 4),
            "per_message_launch_GB_s": round(nbytes / per_msg_s / 1e9, 2),
            "rejected_items": b.rejected_items(), "chunk_blocks": chunk, "bpt": cfg.bpt, "wg": cfg.wg,
            "placement": cfg.placement,
            "variant_from": "tuning record batch winner" if won else "default (record timed other sources)",
            "graph": True}


SATURATION_RHO = 1.5
VERIFY_REQUESTS = 2000


def verify_served(torch, aes, inputs, pool, kt, in_pool, out_arena):
    """Served results against each request run alone: VERIFY_REQUESTS
    requests of the serving mix, submitted in ten bursts 1 ms apart so that
    batches form while others run, outputs kept (no auto release) until every
    one has been compared, byte for byte, with the plain kernel's output for
    that request alone.  Raises on any difference."""
    import numpy as np
    n = VERIFY_REQUESTS
    pool_blocks = in_pool.numel() // 16
    tr = inputs.request_trace(200, n, 1.0, len(pool))
    g = inputs.rng(9, 200)
    reqs = np.zeros(n, dtype=aes.REQUEST_DTYPE)
    reqs["nblocks"] = np.minimum(tr.nblocks, pool_blocks)
    reqs["in_block"] = (g.random(n) * (pool_blocks - reqs["nblocks"] + 1)).astype(np.uint64)
    reqs["key_slot"] = tr.key_slot
    reqs["decrypt"] = tr.decrypt
    if int(reqs["nblocks"].sum()) * 16 > out_arena.numel():
        raise RuntimeError("verification requests do not fit the output arena")
    srv = aes.Server(kt, in_pool, out_arena, budget_bytes=2 * out_arena.numel(), chunk_blocks=2048,
                     max_batch_items=1 << 18, nslots=4, bpt=4, auto_release=False)
    for part in np.array_split(np.arange(n), 10):
        srv.submit(reqs[part])
        time.sleep(0.001)
    got, t0 = [], time.time()
    while sum(len(x) for x in got) < n:
        got.append(srv.poll())
        if time.time() - t0 > 60:
            raise RuntimeError("served requests did not finish")
        time.sleep(0.0002)
    out = np.concatenate(got)
    out = out[np.argsort(out["id"])]
    if (out["status"] != aes.AES_SERVED_DONE).any():
        raise RuntimeError("a verification request was not served")
    scratch = torch.empty(int(reqs["nblocks"].max()) * 16, dtype=torch.uint8, device="cuda")
    scheds = {}
    bad = 0
    for i in range(n):
        q = reqs[i]
        slot = int(q["key_slot"])
        if slot not in scheds:
            scheds[slot] = aes.aes_expand_key(pool[slot][1])
        ks = scheds[slot]
        lo, nb = int(q["in_block"]) * 16, int(q["nblocks"]) * 16
        ob = int(out[i]["out_block"]) * 16
        alone = scratch[:nb]
        if q["decrypt"]:
            aes.aes_ecb_decrypt(ks.rk_dec, ks.nr, in_pool[lo:lo + nb], alone)
        else:
            aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, in_pool[lo:lo + nb], alone)
        if not torch.equal(alone, out_arena[ob:ob + nb]):
            bad += 1
    srv.release(out)
    srv.close()
    if bad:
        raise RuntimeError("%d served requests differ from the request run alone" % bad)
    return {"requests": n, "bytes": int(reqs["nblocks"].sum()) * 16,
            "batches": int(len(np.unique(out["batch"]))), "mismatches": 0}


def serving(torch, aes, inputs, peak_gbps, levels, n_req, bulk_equivalent_gbps=None):
    """Open-loop Poisson arrivals at offered loads rho x peak through the
    native engine (aes_server_*, 4 streams, 2048-block work items and
    256-block items for requests of at most 2048 blocks, 64 bytes per
    thread, 32 GiB budget, 4,096 resident keys): p50/p99 latency
    (scheduled arrival -> completion seen by the engine) and sustained GB/s
    per load.  One more
    trace at SATURATION_RHO x peak keeps the queue from ever emptying, so its
    GB/s is the engine's capacity; its latencies only measure the backlog
    and are not reported."""
    import numpy as np
    from paper_1902_05234_amd import batch
    pool = inputs.key_pool(4, 4096)
    kt = batch.key_table([k for _, k in pool])
    pool_bytes = 4 * GiB
    in_pool = inputs.device_random_bytes(4, pool_bytes)
    budget = 32 * GiB
    out_arena = torch.empty(budget // 2, dtype=torch.uint8, device="cuda")
    srv = aes.Server(kt, in_pool, out_arena, budget_bytes=budget, chunk_blocks=2048, max_batch_items=1 << 18,
                     nslots=4, bpt=4, auto_release=True, size_classes=True)
    mean_b = inputs.mean_trace_bytes()
    rows = []
    pool_blocks = pool_bytes // 16
    capacity = None
    for k, rho in enumerate(list(levels) + [SATURATION_RHO]):
        rate = rho * peak_gbps * 1e9 / mean_b
        tr = inputs.request_trace(100 + k, n_req, rate, len(pool))
        g = inputs.rng(9, k)
        reqs = np.zeros(n_req, dtype=aes.REQUEST_DTYPE)
        reqs["nblocks"] = np.minimum(tr.nblocks, pool_blocks)
        reqs["in_block"] = (g.random(n_req) * (pool_blocks - reqs["nblocks"] + 1)).astype(np.uint64)
        reqs["key_slot"] = tr.key_slot
        reqs["decrypt"] = tr.decrypt
        out = srv.replay(reqs, tr.arrival_s - tr.arrival_s[0])
        ok = out["status"] == aes.AES_SERVED_DONE
        if k == len(levels):
            wall = float(out["done_s"][ok].max() - out["arrival_s"][ok].min())
            capacity = {"rho": rho, "requests": int(ok.sum()), "GB_s": round(int(reqs["nblocks"][ok].sum()) * 16 / wall / 1e9, 1),
                        "seconds": round(wall, 4), "batches": int(len(np.unique(out["batch"][ok])))}
            log("serving capacity (rho=%.2f): %.1f GB/s" % (rho, capacity["GB_s"]))
            break
        lat = np.sort(out["done_s"][ok] - out["arrival_s"][ok]) * 1e3
        nbytes = int(reqs["nblocks"][ok].sum()) * 16
        wall = float(out["done_s"][ok].max() - out["arrival_s"][ok].min())
        small = ok & (reqs["nblocks"] * 16 <= 16 << 10)
        lat_small = np.sort(out["done_s"][small] - out["arrival_s"][small]) * 1e3
        pick = lambda a, q: round(float(a[min(len(a) - 1, int(q * len(a)))]), 4) if len(a) else None
        row = {"rho": rho, "offered_GB_s": round(rho * peak_gbps, 1), "requests": int(ok.sum()),
               "p50_ms": pick(lat, 0.5), "p99_ms": pick(lat, 0.99), "p99_small_ms": pick(lat_small, 0.99),
               "GB_s": round(nbytes / wall / 1e9, 1), "seconds": round(wall, 4),
               "rejected": int((~ok).sum()), "batches": int(len(np.unique(out["batch"][ok])))}
        rows.append(row)
        log("serving rho=%.2f: p50 %.3f ms p99 %.3f ms %.1f GB/s (%d batches)" % (
            rho, row["p50_ms"], row["p99_ms"], row["GB_s"], row["batches"]))
    st = srv.stats()
    srv.close()
    verified = verify_served(torch, aes, inputs, pool, kt, in_pool, out_arena)
    log("serving verified: %d requests, %d batches, all equal to the request run alone" % (
        verified["requests"], verified["batches"]))
    del in_pool, out_arena
    torch.cuda.empty_cache()
    best = max(r["GB_s"] for r in rows)
    res = {"engine": "native (aes_server_*)", "peak_GB_s": round(peak_gbps, 1), "budget_bytes": budget,
           "key_pool": len(pool), "mean_request_bytes": round(mean_b), "streams": 4, "chunk_blocks": 2048, "bpt": 4,
           "small_item_blocks": 256, "completion": "words written by the batch kernel's last workgroup",
           "size_classes": True,
           "requests_per_level": n_req, "max_device_bytes_in_use": st["max_device_bytes_in_use"],
           "batches": st["batches"], "direct_batches": st["direct_batches"],
           "launch_us_per_batch": round(st["launch_ns"] / 1e3 / max(1, st["batches"]), 2), "levels": rows,
           "max_sustained_GB_s": best, "capacity": capacity, "verified": verified}
    if bulk_equivalent_gbps:
        res["max_sustained_vs_bulk"] = round(best / bulk_equivalent_gbps, 4)
        res["capacity_vs_bulk"] = round(capacity["GB_s"] / bulk_equivalent_gbps, 4)
    return res


PROFILE_MID_SIZES = (64 << 10, MiB, 4 * MiB, 16 * MiB, 32 * MiB)


def profile_mid(torch, aes, inputs, replays=10):
    """Launches for a kernel trace of the mid-size regime: for each size, a
    HIP graph of GRAPH_LAUNCHES back-to-back AES-128 encryptions with the
    tuned default variant, warmed up and then replayed `replays` times; first
    the same for a 16-byte device copy (the dispatch floor).  In the trace,
    each kernel's duration and the gap to the next kernel of its graph split
    the per-launch time into work inside the kernel and dispatch between
    kernels."""
    ks = aes.aes_expand_key(inputs.random_key(1, 128))
    x = inputs.device_random_bytes(1, max(PROFILE_MID_SIZES))
    y = torch.empty_like(x)
    cases = [("copy 16 B", lambda: aes.aes_device_copy(x[:16], y[:16]))]
    for n in PROFILE_MID_SIZES:
        xi, yi = x[:n], y[:n]
        cases.append(("AES-128 encrypt %s %s" % (size_name(n) if n >= MiB else "%dKiB" % (n >> 10),
                                                 aes.aes_tune_get(10, False, n // 16)),
                      lambda xi=xi, yi=yi: aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, xi, yi)))
    for name, fn in cases:
        fn()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(GRAPH_LAUNCHES):
                fn()
        warm(torch, g.replay)
        tm = Timer(torch)
        for _ in range(replays):
            tm.run(g.replay)
        ms = sorted(tm.ms())[replays // 2] / GRAPH_LAUNCHES
        del g
        log("%s: %.2f us per launch (graph replay, events)" % (name, ms * 1e3))


def corun(torch, aes, inputs, sweep: bool):
    """The bitsliced kernel (VALU only, no LDS) on one stream beside the
    4-table kernel (LDS-bound) on another, each on its share of one 1 GiB
    buffer: can the VALU that the table kernel leaves idle carry blocks?
    sweep: sustained GB/s for bitsliced shares 0 ... 0.24, two interleaved
    passes, and the bitsliced kernel alone; else 30 steps at share 0.10 (for
    a kernel trace that shows whether the two kernels overlap)."""
    x = inputs.device_random_bytes(1, GiB)
    y = torch.empty_like(x)
    ref = torch.empty_like(x)
    ks = aes.aes_expand_key(inputs.random_key(1, 128))
    nblocks = GiB // 16
    v4 = aes.Variant(bpt=4, wg=1024, placement=aes.AES_PLACEMENT_TTABLE4)
    vb = aes.Variant(bpt=1, wg=256, placement=aes.AES_PLACEMENT_BITSLICED,
                     grid=torch.cuda.get_device_properties(0).multi_processor_count)
    aes.aes_ecb_crypt_variant(ks.rk_enc, ks.nr, False, x, ref, v4)
    cur = torch.cuda.current_stream()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()

    def step(nb):
        sa.wait_stream(cur)
        sb.wait_stream(cur)
        if nb:
            with torch.cuda.stream(sa):  # first, so it is resident when the table kernel arrives
                aes.aes_ecb_crypt_variant(ks.rk_enc, ks.nr, False, x[:nb * 16], y[:nb * 16], vb)
        with torch.cuda.stream(sb):
            aes.aes_ecb_crypt_variant(ks.rk_enc, ks.nr, False, x[nb * 16:], y[nb * 16:], v4)
        cur.wait_stream(sa)
        cur.wait_stream(sb)

    def share(f):
        return (int(f * nblocks) // 8192) * 8192

    def rate(nb, seconds=1.0):
        step(nb)
        torch.cuda.synchronize()
        if not torch.equal(y, ref):
            raise RuntimeError("co-run output differs from the 4-table kernel alone (share %d blocks)" % nb)
        warm(torch, lambda: step(nb), 0.5)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(cur)
        k, t_end = 0, time.perf_counter() + seconds
        while time.perf_counter() < t_end:
            step(nb)
            k += 1
        b.record(cur)
        torch.cuda.synchronize()
        return GiB * k / (a.elapsed_time(b) * 1e-3) / 1e9

    if not sweep:
        nb = share(0.10)
        step(nb)
        torch.cuda.synchronize()
        if not torch.equal(y, ref):
            raise RuntimeError("co-run output differs from the 4-table kernel alone")
        for _ in range(30):
            step(nb)
        torch.cuda.synchronize()
        log("co-run trace steps done: bitsliced share %d blocks" % nb)
        return
    for p in range(2):
        log("co-run pass %d: %s" % (p, "  ".join("f=%.2f %.1f GB/s" % (f, rate(share(f)))
                                                 for f in (0.0, 0.04, 0.08, 0.12, 0.16, 0.24))))
    t = Timer(torch)
    aes.aes_ecb_crypt_variant(ks.rk_enc, ks.nr, False, x, y, vb)
    for _ in range(20):
        t.run(lambda: aes.aes_ecb_crypt_variant(ks.rk_enc, ks.nr, False, x, y, vb))
    log("bitsliced kernel alone: %.1f GB/s" % (GiB / (sorted(t.ms())[10] * 1e-3) / 1e9))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--warmup-seconds", type=float, default=1.0,
                    help="after --warmup steps, keep warming up until this much load has passed")
    ap.add_argument("--no-batch", action="store_true")
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-host", action="store_true", help="skip the host-inclusive file-size sweep")
    ap.add_argument("--serve-levels", default="0.1,0.2,0.3,0.4,0.5,0.6,0.7,0.8,0.9,1.0")
    ap.add_argument("--serve-requests", type=int, default=20000)
    ap.add_argument("--profile", nargs="?", const="bulk",
                    choices=("bulk", "mid", "corun", "corun-sweep", "ctr", "cbc-msgs", "variants", "host"),
                    default=None,
                    help="bulk: only a few copy and 1 GiB launches; mid: graph-replayed AES-128 encryptions of "
                         "64 KiB ... 32 MiB and of a 16-byte copy (for rocprofv3 kernel traces); corun: the "
                         "bitsliced kernel beside the 4-table kernel on two streams, 30 steps (for a kernel "
                         "trace); corun-sweep: their sustained rates over bitsliced shares 0 ... 0.24; ctr: 1 GiB CTR and ECB "
                         "encryptions in turn (for counters); cbc-msgs: 3 copies of 1 GiB, then CBC encryption of 1 GiB as "
                         "2^18 messages of 4 KiB and ECB encryption of the same buffer, in turn, then CBC encryption "
                         "of 1 GiB as 2^16 messages of 16 KiB, then CBC decryption of the 4 KiB set (for counters and "
                         "traces); variants: the tuned defaults at 256 KiB, 4 and 16 MiB "
                         "and the bitsliced kernel at 1 GiB (for counters); host: the host-inclusive file-size sweep "
                         "only (for a kernel and copy trace)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: ECB blocks are independent, so N GPUs would each run this same "
              "single-GPU kernel on 1/N of the buffer with no communication; only --gpus 1 is supported.",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1902_05234_amd import aes, inputs
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    aes._lib()
    props = torch.cuda.get_device_properties(0)
    log("device:", props.name, "CUs:", props.multi_processor_count)

    if args.profile == "mid":
        profile_mid(torch, aes, inputs)
        return
    if args.profile in ("corun", "corun-sweep"):
        corun(torch, aes, inputs, args.profile == "corun-sweep")
        return
    if args.profile == "variants":
        # the tuned defaults below 32 MiB and the bitsliced kernel, three launches
        # each (for counters of the kernels that serve small and mid sizes)
        x = inputs.device_random_bytes(1, GiB)
        y = torch.empty_like(x)
        ks = aes.aes_expand_key(inputs.random_key(1, 128))
        for n in (256 << 10, 4 * MiB, 16 * MiB):
            log("variant at %d bytes:" % n, aes.aes_tune_get(10, False, n // 16))
            for _ in range(3):
                aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, x[:n], y[:n])
        vb = aes.Variant(bpt=1, wg=256, placement=aes.AES_PLACEMENT_BITSLICED)
        for _ in range(3):
            aes.aes_ecb_crypt_variant(ks.rk_enc, ks.nr, False, x, y, vb)
        torch.cuda.synchronize()
        log("variant profile launches done")
        return
    if args.profile == "host":
        log(json.dumps(host_sweep(torch, aes, inputs, reps=5)))
        return
    if args.profile == "ctr":
        # counter mode beside ECB encryption, 1 GiB each, tuned defaults (for
        # counters: LDS instructions per block with and without the caching)
        x = inputs.device_random_bytes(1, GiB)
        y = torch.empty_like(x)
        ks = aes.aes_expand_key(inputs.random_key(1, 128))
        iv = bytes(range(16))
        for _ in range(max(1, args.steps)):
            aes.aes_ctr_crypt(ks.rk_enc, ks.nr, iv, 0, x, y)
            aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, x, y)
        torch.cuda.synchronize()
        log("ctr profile launches done")
        return
    if args.profile == "cbc-msgs":
        # CBC encryption across 2^18 independent 4 KiB messages (one chain per
        # lane, default shape) beside ECB encryption of the same 1 GiB
        x = inputs.device_random_bytes(1, GiB)
        y = torch.empty_like(x)
        ks = aes.aes_expand_key(inputs.random_key(1, 128))
        nm = GiB // 4096
        msgs = torch.from_numpy(cbc_records(inputs.cbc_equal_messages(3, nm, 256)).view(np.uint8)).to("cuda")
        # and 1 GiB as 2^16 messages of 16 KiB, which the default runs four
        # lanes per message
        nq = GiB // 16384
        msgs_q = torch.from_numpy(cbc_records(inputs.cbc_equal_messages(4, nq, 1024)).view(np.uint8)).to("cuda")
        for _ in range(3):
            aes.aes_device_copy(x, y)  # known bytes: the counters' calibration
        for _ in range(max(1, args.steps)):
            aes.aes_cbc_encrypt_msgs(ks.rk_enc, ks.nr, msgs, nm, x, y)
            aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, x, y)
        for _ in range(max(1, args.steps)):
            aes.aes_cbc_encrypt_msgs(ks.rk_enc, ks.nr, msgs_q, nq, x, y)
        for _ in range(max(1, args.steps)):  # decryption of the 4 KiB set: one wave per message
            aes.aes_cbc_decrypt_msgs(ks.rk_dec, ks.nr, msgs, nm, x, y)
        torch.cuda.synchronize()
        log("cbc-msgs profile launches done")
        return
    if args.profile:
        x = inputs.device_random_bytes(1, GiB)
        y = torch.empty_like(x)
        for _ in range(3):
            aes.aes_device_copy(x, y)
        ks = aes.aes_expand_key(inputs.random_key(1, 128))
        for dec in (False, True):
            log("variant", "decrypt" if dec else "encrypt", aes.aes_tune_get(10, dec, GiB // 16))
        for _ in range(max(1, args.steps)):
            aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, x, y)
            aes.aes_ecb_decrypt(ks.rk_dec, ks.nr, y, x)
        torch.cuda.synchronize()
        log("profile launches done")
        return

    b = bulk(torch, aes, inputs, args)
    log("bulk: %.3f s for %d steps" % (b["elapsed"], args.steps))
    traffic = read_traffic(b["nbytes"], kernel_instance(aes.aes_tune_get(10, False, b["nbytes"] // 16)))
    result = {
        "metric": "AES-ECB enc/dec GB/s at 1 GiB + % roofline; batched vs plain GB/s; p99 latency",
        "value": round(2 * b["nbytes"] * args.steps / b["elapsed"] / 1e9, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "warmup_steps_run": b["warmup_steps"],
        "warmup_ms": round(b["warmup_ms"], 1),
        "ms_per_step": round(b["elapsed"] / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "AES-128 ECB encrypt then decrypt of one 1 GiB device buffer (67,108,864 blocks), "
                               "seeded uniform random bytes and key", "keybits": 128, "bytes": b["nbytes"],
                   "parallelism": "single GPU",
                   "seeds": {"base": inputs.BASE_SEED, "data": "device_random_bytes(1)", "key": "random_key(1, 128)"}},
        "enc_GB_s": round(b["nbytes"] / (sum(b["enc_ms"]) / len(b["enc_ms"]) * 1e-3) / 1e9, 1),
        "dec_GB_s": round(b["nbytes"] / (sum(b["dec_ms"]) / len(b["dec_ms"]) * 1e-3) / 1e9, 1),
        "roofline": roofline(b, traffic, aes),
        "measured_roofs": None,
        "kernel_source_hash": kernel_source_hash(),
        "device": props.name,
        "platform": {"arch": getattr(props, "gcnArchName", None), "cus": props.multi_processor_count,
                     "hbm_bytes": props.total_memory, "hip": torch.version.hip, "torch": torch.__version__,
                     "tune_file": os.environ.get(aes.TUNE_FILE_ENV)},
    }
    clock = clock_under_load(torch, aes, b)
    if clock:
        rl0 = result["roofline"]
        clock["frac_at_clock"] = round(rl0["achieved"] / clock["lds_roof_at_clock_Glookup_s"], 4)
        result["roofline"]["clock_under_load"] = clock
        log("clock under load:", clock)
    roofs = measured_roofs(torch, aes, inputs)
    result["measured_roofs"] = roofs
    rl = result["roofline"]
    rl["measured_peak"] = roofs["lds_Glookup_s"]
    rl["frac_of_measured"] = round(rl["achieved"] / roofs["lds_Glookup_s"], 4)
    log("measured roofs:", roofs)
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(b, args)
        log("cpu baseline done")
    del b
    torch.cuda.empty_cache()
    rates = None
    if not args.no_sweep or not args.no_batch:
        sizes = [MiB, 16 * MiB, 256 * MiB, GiB] + ([] if args.no_sweep else [4 * GiB])
        rates = sweep(torch, aes, inputs, sizes)
        log("sweep done")
        if not args.no_sweep:
            result["sweep_GB_s"] = rates
    if not args.no_host:
        result["host_path"] = host_sweep(torch, aes, inputs)
        log("host path done")
    if not args.no_batch:
        result["batched"] = batched(torch, aes, inputs, rates)
        log("batched done")
    if not args.no_serve:
        peak = result["batched"]["GB_s"] if "batched" in result else result["value"]
        levels = [float(v) for v in args.serve_levels.split(",") if v]
        beq = result["batched"]["bulk_equivalent_GB_s"] if "batched" in result else None
        result["serving"] = serving(torch, aes, inputs, peak, levels, args.serve_requests, beq)
        log("serving done")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
