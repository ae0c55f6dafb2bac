"""Batched ECB over many independent messages: host orchestration.

Builds the device key table and the device work list for a set of messages
packed into one input arena, then runs them in one persistent launch of
``aes_ecb_batch`` (optionally replayed from a captured HIP graph).  Cipher
work happens only in the library's kernels.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import aes


@dataclass
class Batch:
    """Device-resident state of one batch (reusable across launches)."""

    items_dev: object       # uint8 tensor holding ITEM_DTYPE entries
    n_enc: int
    n_dec: int
    key_table_dev: object   # uint32 tensor [n_slots * 128]
    counters_dev: object    # uint32 tensor [4]
    in_arena: object        # uint8 tensor
    out_arena: object       # uint8 tensor
    msgs: np.ndarray        # MSG_DTYPE, host copy
    cfg: aes.BatchConfig
    graph: object = None

    def launch(self, stream=None):
        aes.aes_ecb_batch(self.items_dev, self.n_enc, self.n_dec, self.key_table_dev, self.in_arena,
                          self.out_arena, self.counters_dev, self.cfg, stream)

    def capture(self):
        """Capture one launch in a HIP graph (the kernel resets its own claim
        counters, so the graph holds a single kernel node)."""
        import torch
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.launch()  # warm-up launch outside the capture
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.launch()
        self.graph = g
        return g

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()

    def rejected_items(self) -> int:
        return int(self.counters_dev[3].item())

    @property
    def total_bytes(self) -> int:
        return int(self.msgs["nblocks"].sum()) * 16


def key_table(keys, device="cuda"):
    """Device key table from a list of raw keys (16/24/32 bytes each)."""
    import torch
    table = np.zeros((len(keys), aes.AES_KEY_SLOT_WORDS), dtype=np.uint32)
    for i, k in enumerate(keys):
        table[i] = aes.aes_key_slot(k)
    return torch.from_numpy(table.reshape(-1)).to(device)


def prepare(msgs: np.ndarray, key_table_dev, in_arena, out_arena, chunk_blocks: int = 1024,
            cfg: aes.BatchConfig | None = None, device="cuda") -> Batch:
    """Plan ``msgs`` (MSG_DTYPE) into a device work list over the given arenas."""
    import torch
    items, ne, nd = aes.aes_batch_plan(msgs, chunk_blocks)
    items_dev = torch.from_numpy(items.view(np.uint8).copy()).to(device) if len(items) else torch.zeros(
        24, dtype=torch.uint8, device=device)
    counters = torch.zeros(4, dtype=torch.int32, device=device)
    c = cfg or aes.BatchConfig()
    if c.enc_groups < 0 and ne + nd:
        # split the persistent groups by bytes, not by item count
        enc_b = int(items["nblocks"][:ne].sum())
        tot = int(items["nblocks"].sum())
        import dataclasses
        c = dataclasses.replace(c, enc_groups=max(1 if ne else 0, round(_grid(c) * enc_b / max(1, tot))))
    return Batch(items_dev, ne, nd, key_table_dev, counters, in_arena, out_arena, np.ascontiguousarray(msgs), c)


def _grid(c: aes.BatchConfig) -> int:
    return aes.aes_batch_max_grid(c)


def messages_from_mix(mix, key_slots=None) -> np.ndarray:
    """MSG_DTYPE array for an ``inputs.MessageMix`` packed back to back in
    both arenas (message i reads and writes blocks offset[i] ...)."""
    m = np.zeros(len(mix), dtype=aes.MSG_DTYPE)
    m["in_block"] = mix.offset
    m["out_block"] = mix.offset
    m["nblocks"] = mix.nblocks
    m["key_slot"] = np.arange(len(mix)) if key_slots is None else key_slots
    m["decrypt"] = mix.decrypt.astype(np.uint32)
    return m


def run_per_message(msgs: np.ndarray, schedules, in_arena, out_arena, stream=None):
    """Reference form: one plain-kernel launch per message (same arenas)."""
    a = in_arena.view(-1)
    b = out_arena.view(-1)
    for m in msgs:
        ks = schedules[int(m["key_slot"])]
        lo = int(m["in_block"]) * 16
        ol = int(m["out_block"]) * 16
        n = int(m["nblocks"]) * 16
        if n == 0:
            continue
        if m["decrypt"]:
            aes.aes_ecb_decrypt(ks.rk_dec, ks.nr, a[lo:lo + n], b[ol:ol + n], stream=stream)
        else:
            aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, a[lo:lo + n], b[ol:ol + n], stream=stream)
