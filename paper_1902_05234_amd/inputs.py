"""Seeded synthetic inputs for the AES-ECB workloads.

This module only draws random numbers (numpy PCG64 via SeedSequence); it
holds none of the cipher's arithmetic.  Both the GPU path's tests/benchmark
and the CPU oracle take their inputs from here.

Recipes (the paper measures unspecified "files" of 1,202 ... 1,190,402 bytes,
section 5, Tables 4-5; uniform random bytes stand in for them):

* buffers: uniform random bytes; keys: uniform random 16/24/32 bytes;
* batch mix: message lengths log-uniform between 16 B and 8 MiB, rounded to
  whole 16-byte blocks, key size uniform over {128, 192, 256}, direction
  encrypt/decrypt with probability 1/2 each;
* serving mix: Poisson arrivals; sizes 80 % log-uniform 64 B - 16 KiB and
  20 % log-uniform 1 - 64 MiB (rounded to 16 B); keys drawn from a pool;
* CBC message sets: many independent messages under one key, each with a
  uniform random 16-byte initialisation vector; either a ragged set (lengths
  uniform in 0 .. max blocks, inputs packed in order with gaps, outputs in a
  shuffled order with gaps) or equal lengths back to back.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

BASE_SEED = 190205234
KEY_BITS = (128, 192, 256)


def rng(*path: int) -> np.random.Generator:
    """Independent generator for a tuple of integers under BASE_SEED."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([BASE_SEED, *path])))


def random_bytes(seed: int, nbytes: int) -> np.ndarray:
    """``nbytes`` uniform random bytes (uint8 array)."""
    return rng(1, seed).integers(0, 256, size=nbytes, dtype=np.uint8)


def random_key(seed: int, keybits: int) -> bytes:
    if keybits not in KEY_BITS:
        raise ValueError("keybits must be 128, 192 or 256")
    return rng(2, seed, keybits).integers(0, 256, size=keybits // 8, dtype=np.uint8).tobytes()


def _log_uniform_blocks(g: np.random.Generator, lo_bytes: float, hi_bytes: float, n: int) -> np.ndarray:
    size = np.exp(g.uniform(np.log(lo_bytes), np.log(hi_bytes), size=n))
    blocks = np.rint(size / 16.0).astype(np.int64)
    return np.clip(blocks, max(1, int(lo_bytes) // 16), int(hi_bytes) // 16)


@dataclass
class MessageMix:
    """A set of independent messages packed back to back in one arena."""

    nblocks: np.ndarray   # int64 [n]
    keybits: np.ndarray   # int32 [n]
    decrypt: np.ndarray   # bool  [n]
    key_seed: np.ndarray  # int64 [n]  seed for random_key(seed, keybits)
    offset: np.ndarray    # int64 [n]  first block of each message in the arena

    @property
    def total_blocks(self) -> int:
        return int(self.nblocks.sum())

    def __len__(self) -> int:
        return int(self.nblocks.size)


def message_mix(seed: int, n: int, lo_bytes: int = 16, hi_bytes: int = 8 << 20) -> MessageMix:
    """``n`` messages, lengths log-uniform in [lo_bytes, hi_bytes], whole blocks."""
    g = rng(3, seed)
    nblocks = _log_uniform_blocks(g, lo_bytes, hi_bytes, n)
    keybits = g.choice(np.array(KEY_BITS, dtype=np.int32), size=n)
    decrypt = g.random(n) < 0.5
    key_seed = g.integers(0, 2**62, size=n, dtype=np.int64)
    offset = np.zeros(n, dtype=np.int64)
    if n:
        offset[1:] = np.cumsum(nblocks)[:-1]
    return MessageMix(nblocks, keybits, decrypt, key_seed, offset)


@dataclass
class RequestTrace:
    """An open-loop request trace for the serving loop."""

    arrival_s: np.ndarray  # float64 [n] absolute arrival times
    nblocks: np.ndarray    # int64 [n]
    key_slot: np.ndarray   # int64 [n] index into the key pool
    decrypt: np.ndarray    # bool  [n]


def request_trace(seed: int, n: int, rate_per_s: float, pool_size: int = 4096) -> RequestTrace:
    """Poisson arrivals at ``rate_per_s``; 80 % small (64 B-16 KiB), 20 % large (1-64 MiB)."""
    g = rng(4, seed)
    gaps = g.exponential(1.0 / rate_per_s, size=n)
    arrival = np.cumsum(gaps)
    small = g.random(n) < 0.8
    nb_small = _log_uniform_blocks(g, 64, 16 << 10, n)
    nb_large = _log_uniform_blocks(g, 1 << 20, 64 << 20, n)
    nblocks = np.where(small, nb_small, nb_large)
    key_slot = g.integers(0, pool_size, size=n, dtype=np.int64)
    decrypt = g.random(n) < 0.5
    return RequestTrace(arrival, nblocks, key_slot, decrypt)


def key_pool(seed: int, n: int):
    """``n`` (keybits, key) pairs, key size uniform over {128, 192, 256}."""
    g = rng(5, seed)
    bits = g.choice(np.array(KEY_BITS), size=n)
    return [(int(b), random_key(int(seed) * 1_000_003 + i, int(b))) for i, b in enumerate(bits)]


def mean_trace_bytes() -> float:
    """Expected request size of ``request_trace`` in bytes (log-uniform means)."""
    def lu_mean(a, b):
        return (b - a) / np.log(b / a)
    return 0.8 * lu_mean(64, 16 << 10) + 0.2 * lu_mean(1 << 20, 64 << 20)


def device_random_bytes(seed: int, nbytes: int, device="cuda"):
    """``nbytes`` uniform random bytes generated on the GPU by torch's seeded
    Philox generator (for buffers too large to draw on the host)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(np.random.SeedSequence([BASE_SEED, 6, seed]).generate_state(1)[0]))
    return torch.randint(0, 256, (nbytes,), dtype=torch.uint8, device=device, generator=g)


@dataclass
class CbcMessageSet:
    """Positions (in 16-byte blocks) and initialisation vectors of independent
    messages in an input and an output arena."""

    nblocks: np.ndarray    # uint64 [n]
    in_block: np.ndarray   # uint64 [n]
    out_block: np.ndarray  # uint64 [n]
    iv: np.ndarray         # uint8 [n, 16]
    in_blocks: int         # arena sizes
    out_blocks: int

    def __len__(self) -> int:
        return int(self.nblocks.size)


def cbc_message_set(seed: int, n: int, max_blocks: int) -> CbcMessageSet:
    """A ragged set: the first min(n, 10) messages have 0 .. 9 blocks, the
    rest uniform in [0, max_blocks]; inputs in order with gaps of 0 .. 3
    blocks, outputs in a random order with gaps of 0 .. 3 blocks."""
    g = rng(7, seed)
    nb = g.integers(0, max_blocks + 1, size=n).astype(np.uint64)
    k = min(n, 10)
    nb[:k] = np.arange(k, dtype=np.uint64)
    gap_in = g.integers(0, 4, size=n).astype(np.uint64)
    in_block = np.cumsum(gap_in + nb) - nb
    order = g.permutation(n)
    gap_out = g.integers(0, 4, size=n).astype(np.uint64)
    ends = np.cumsum(gap_out + nb[order])
    out_block = np.empty(n, dtype=np.uint64)
    out_block[order] = ends - nb[order]
    iv = g.integers(0, 256, size=(n, 16), dtype=np.uint8)
    return CbcMessageSet(nb, in_block.astype(np.uint64), out_block, iv,
                         int(in_block[-1] + nb[-1]) + 3 if n else 0, int(ends[-1]) + 3 if n else 0)


def cbc_equal_messages(seed: int, n: int, blocks: int) -> CbcMessageSet:
    """n messages of ``blocks`` blocks each, back to back in both arenas at
    the same positions (message m at block m * blocks)."""
    g = rng(8, seed)
    pos = (np.arange(n, dtype=np.uint64) * np.uint64(blocks))
    iv = g.integers(0, 256, size=(n, 16), dtype=np.uint8)
    return CbcMessageSet(np.full(n, blocks, dtype=np.uint64), pos, pos.copy(), iv, n * blocks, n * blocks)
