"""The host-inclusive path (aes_pipe_*): host buffer in, host buffer out,
chunks pipelined over several streams.  Bit-exact against the CPU oracle:
the paper's file sizes (section 5, Tables 4-5, padded to whole blocks for
ECB), pageable buffers through the pinned staging and pinned buffers copied
directly, chunk boundaries that cut through the data, CTR with a partial
last block and a counter continued across chunks, and in-place host
buffers."""
import numpy as np
import pytest

from paper_1902_05234_amd import aes, inputs
from tests.gpu_util import cuda, first_mismatch

pytestmark = pytest.mark.gpu

PAPER_SIZES = [1202, 4652, 9302, 18602, 37202, 74402, 148802, 297602, 595202, 1190402]


def assert_same(got, want, what):
    i = first_mismatch(np.asarray(got), np.asarray(want))
    assert i is None, "%s: first differing byte %d" % (what, i)


def padded(n):
    return (n + 15) // 16 * 16


@pytest.fixture(scope="module")
def pipe():
    cuda()
    p = aes.HostPipe(chunk_bytes=64 << 10, nslots=3)
    yield p
    p.close()


@pytest.mark.parametrize("keybits", [128, 256])
def test_pipe_paper_sizes_pageable(oracle_lib, pipe, keybits):
    key = inputs.random_key(800, keybits)
    ks = aes.aes_expand_key(key)
    for size in PAPER_SIZES:
        x = inputs.random_bytes(801 + size, padded(size))
        c = pipe.run(aes.AES_PIPE_ECB_ENCRYPT, ks, x)
        assert_same(c, oracle_lib.ecb_encrypt(key, x), "enc %d" % size)
        assert_same(pipe.run(aes.AES_PIPE_ECB_DECRYPT, ks, c), x, "dec %d" % size)


def test_pipe_pinned_direct_and_in_place(oracle_lib):
    torch = cuda()
    key = inputs.random_key(810, 192)
    ks = aes.aes_expand_key(key)
    n = 16 * 300001
    x = inputs.random_bytes(811, n)
    p = aes.HostPipe(chunk_bytes=1 << 20, nslots=4, staging=False)
    try:
        src = torch.from_numpy(x.copy()).pin_memory()
        dst = torch.empty(n, dtype=torch.uint8).pin_memory()
        p.run(aes.AES_PIPE_ECB_ENCRYPT, ks, src, out=dst)
        assert_same(dst.numpy(), oracle_lib.ecb_encrypt(key, x), "pinned enc")
        p.run(aes.AES_PIPE_ECB_DECRYPT, ks, dst, out=dst)          # in place
        assert_same(dst.numpy(), x, "pinned dec in place")
        with pytest.raises(aes.AesError):                          # pageable without staging
            p.run(aes.AES_PIPE_ECB_ENCRYPT, ks, x)
    finally:
        p.close()


def test_pipe_pinned_small_buffers_run_on_host_memory(oracle_lib):
    """Buffers of at most one chunk in pinned memory take the single-launch
    path on host memory: ECB both ways, CTR with a partial block, slices that
    start inside a pinned allocation, and in place."""
    torch = cuda()
    key = inputs.random_key(815, 256)
    ks = aes.aes_expand_key(key)
    iv = bytes(range(16))
    p = aes.HostPipe(chunk_bytes=256 << 10, nslots=2, staging=False)
    try:
        big = torch.zeros(1 << 20, dtype=torch.uint8).pin_memory()
        for n, at in ((16, 0), (1216, 4096), (18608, 12345 * 16), (256 << 10, 512 << 10)):
            x = inputs.random_bytes(816 + n, n)
            src = big[at:at + n]
            src.copy_(torch.from_numpy(x))
            dst = torch.zeros(n, dtype=torch.uint8).pin_memory()
            p.run(aes.AES_PIPE_ECB_ENCRYPT, ks, src, out=dst)
            assert_same(dst.numpy(), oracle_lib.ecb_encrypt(key, x), "pinned enc n=%d" % n)
            p.run(aes.AES_PIPE_ECB_DECRYPT, ks, dst, out=dst)
            assert_same(dst.numpy(), x, "pinned dec in place n=%d" % n)
            m = n - 5 if n > 16 else 11
            p.run(aes.AES_PIPE_CTR, ks, src[:m], out=dst[:m], iv=iv)
            assert_same(dst[:m].numpy(), oracle_lib.ctr_crypt(key, iv, x[:m]), "pinned ctr n=%d" % m)
        x = inputs.random_bytes(819, 1024)
        src = big[8:8 + 1024]                                      # not 16-byte aligned: copy path
        src.copy_(torch.from_numpy(x))
        dst = torch.zeros(1024, dtype=torch.uint8).pin_memory()
        p.run(aes.AES_PIPE_ECB_ENCRYPT, ks, src, out=dst)
        assert_same(dst.numpy(), oracle_lib.ecb_encrypt(key, x), "unaligned pinned enc")
    finally:
        p.close()


def test_pipe_many_small_calls_in_a_row(oracle_lib):
    """Back-to-back calls that take the single-launch path, pinned and staged,
    ECB both ways and CTR, each result read as soon as its call returns: the
    call must not return before the kernel's output is in host memory."""
    torch = cuda()
    key = inputs.random_key(818, 128)
    ks = aes.aes_expand_key(key)
    iv = bytes(range(16, 32))
    p = aes.HostPipe(chunk_bytes=256 << 10, nslots=2)
    try:
        src = torch.zeros(256 << 10, dtype=torch.uint8).pin_memory()
        dst = torch.zeros(256 << 10, dtype=torch.uint8).pin_memory()
        g = inputs.rng(818)
        for i in range(240):
            n = int(g.integers(1, 4097)) * 16
            x = inputs.random_bytes(900 + i, n)
            kind = i % 4
            if kind == 0:                                          # pinned, direct on the caller's buffers
                src[:n].copy_(torch.from_numpy(x))
                p.run(aes.AES_PIPE_ECB_ENCRYPT, ks, src[:n], out=dst[:n])
                got, want = dst[:n].numpy(), oracle_lib.ecb_encrypt(key, x)
            elif kind == 1:                                        # pageable, through the staging
                got, want = p.run(aes.AES_PIPE_ECB_ENCRYPT, ks, x), oracle_lib.ecb_encrypt(key, x)
            elif kind == 2:
                c = oracle_lib.ecb_encrypt(key, x)
                got, want = p.run(aes.AES_PIPE_ECB_DECRYPT, ks, c), x
            else:
                m = n - int(g.integers(0, 16))
                src[:m].copy_(torch.from_numpy(x[:m]))
                p.run(aes.AES_PIPE_CTR, ks, src[:m], out=dst[:m], iv=iv)
                got, want = dst[:m].numpy(), oracle_lib.ctr_crypt(key, iv, x[:m])
            assert_same(got, want, "call %d (kind %d, %d bytes)" % (i, kind, n))
    finally:
        p.close()


def test_pipe_staged_buffers_in_pieces(oracle_lib):
    """Pageable buffers up to 4 MiB go through the pinned staging in up to four
    pieces, each copied in, run and copied out while the next one runs: sizes
    around the piece boundaries, the largest single-launch buffer, CTR with a
    partial last block across pieces, and in place."""
    cuda()
    key = inputs.random_key(825, 192)
    ks = aes.aes_expand_key(key)
    iv = bytes([0xff] * 8 + [0xfe] + [0xff] * 7)  # the counter's low half wraps inside the buffer
    p = aes.HostPipe()  # 2 slots x 32 MiB: every size here takes the single-launch path
    try:
        for n in (256 << 10, (512 << 10) - 16, (512 << 10) + 16, 1190416, (3 << 20) + 48, 4 << 20):
            x = inputs.random_bytes(826 + n, n)
            c = p.run(aes.AES_PIPE_ECB_ENCRYPT, ks, x)
            assert_same(c, oracle_lib.ecb_encrypt(key, x), "staged enc n=%d" % n)
            assert_same(p.run(aes.AES_PIPE_ECB_DECRYPT, ks, c), x, "staged dec n=%d" % n)
        for m in (1000003, (4 << 20) - 5):
            x = inputs.random_bytes(827 + m, m)
            assert_same(p.run(aes.AES_PIPE_CTR, ks, x, iv=iv), oracle_lib.ctr_crypt(key, iv, x), "staged ctr n=%d" % m)
        x = inputs.random_bytes(828, 2 << 20)
        buf = x.copy()
        p.run(aes.AES_PIPE_ECB_ENCRYPT, ks, buf, out=buf)                                   # in place
        assert_same(buf, oracle_lib.ecb_encrypt(key, x), "staged enc in place")
    finally:
        p.close()


def test_pipe_pieces_smaller_than_the_chunk(oracle_lib):
    """With the default 2 x 32 MiB pipe a buffer of a few MiB is cut into
    1-2 MiB pieces (two per slot) so its copies still overlap: ECB and CTR
    over pinned and pageable buffers with a ragged last piece equal the
    oracle, the CTR counter continuing at every piece offset."""
    torch = cuda()
    key = inputs.random_key(831, 128)
    ks = aes.aes_expand_key(key)
    iv = bytes([0xff] * 8 + [0xfe] + [0xff] * 7)
    p = aes.HostPipe()
    try:
        for n in ((8 << 20) + 48, (5 << 20) + 16 * 7, (20 << 20) + 16):
            x = inputs.random_bytes(832 + n % 97, n)
            want = oracle_lib.ecb_encrypt(key, x)
            got = p.run(aes.AES_PIPE_ECB_ENCRYPT, ks, x)                      # pageable, staged
            assert_same(got, want, "staged enc n=%d" % n)
            src = torch.from_numpy(x).pin_memory()
            dst = torch.zeros(n, dtype=torch.uint8).pin_memory()
            p.run(aes.AES_PIPE_ECB_ENCRYPT, ks, src, out=dst)                 # pinned, copied directly
            assert_same(dst.numpy(), want, "pinned enc n=%d" % n)
            p.run(aes.AES_PIPE_ECB_DECRYPT, ks, dst, out=dst)
            assert_same(dst.numpy(), x, "pinned dec in place n=%d" % n)
            m = n - 3
            got = p.run(aes.AES_PIPE_CTR, ks, x[:m], iv=iv)
            assert_same(got, oracle_lib.ctr_crypt(key, iv, x[:m]), "ctr n=%d" % m)
    finally:
        p.close()


def test_pipe_ctr_across_chunks(oracle_lib, pipe):
    key = inputs.random_key(820, 128)
    ks = aes.aes_expand_key(key)
    iv = bytes(8) + b"\xff" * 7 + b"\xf0"        # the low half carries inside the buffer
    for n in (1, 17, (64 << 10) * 3 + 5, (64 << 10) * 7 - 3):
        x = inputs.random_bytes(821 + n, n)
        y = pipe.run(aes.AES_PIPE_CTR, ks, x, iv=iv)
        assert_same(y, oracle_lib.ctr_crypt(key, iv, x), "ctr n=%d" % n)
        buf = x.copy()
        pipe.run(aes.AES_PIPE_CTR, ks, buf, out=buf, iv=iv)        # in place, staged
        assert_same(buf, y, "ctr in place n=%d" % n)


def test_pipe_large_buffer_many_chunks(oracle_lib):
    """64 MiB + 48 B through 4 MiB chunks on 4 streams against the device path."""
    torch = cuda()
    key = inputs.random_key(830, 256)
    ks = aes.aes_expand_key(key)
    n = (64 << 20) + 48
    x = inputs.random_bytes(831, n)
    p = aes.HostPipe(chunk_bytes=4 << 20, nslots=4)
    try:
        c = p.run(aes.AES_PIPE_ECB_ENCRYPT, ks, x)
    finally:
        p.close()
    xd = torch.from_numpy(x).to("cuda")
    want = torch.empty_like(xd)
    aes.aes_ecb_encrypt(ks.rk_enc, ks.nr, xd, want)
    assert_same(c, want.cpu().numpy(), "64 MiB")
    assert_same(c[-(1 << 20):], oracle_lib.ecb_encrypt(key, x[-(1 << 20):]), "last MiB vs oracle")
