"""The oracle is clean under AddressSanitizer and UndefinedBehaviorSanitizer:
a sanitized copy is built on the CPU (host code only) and every entry point
runs in a child process with the sanitizer runtimes preloaded, on key sizes,
odd lengths, partial CTR blocks and several threads; any report aborts the
child.  Its results must also equal the regular build's."""
import os
import subprocess
import sys

import pytest

from oracle import build as obuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
import numpy as np
import oracle

san = oracle.Oracle(sys.argv[1])
ref = oracle.load()
g = np.random.default_rng(7)
for kb in (128, 192, 256):
    key = g.integers(0, 256, kb // 8, dtype=np.uint8).tobytes()
    iv = g.integers(0, 256, 16, dtype=np.uint8).tobytes()
    ws = san.expand_key(key)
    assert np.array_equal(np.asarray(ws[0]), np.asarray(ref.expand_key(key)[0]))
    for nblocks in (0, 1, 2, 63, 65, 1000):
        x = g.integers(0, 256, 16 * nblocks, dtype=np.uint8)
        for nt in (1, 3):
            c = san.ecb_encrypt(key, x, nthreads=nt)
            assert np.array_equal(c, ref.ecb_encrypt(key, x, nthreads=1))
            assert np.array_equal(san.ecb_decrypt(key, c, nthreads=nt), x)
            if nblocks:
                e = san.cbc_encrypt(key, iv, x)
                assert np.array_equal(e, ref.cbc_encrypt(key, iv, x))
                assert np.array_equal(san.cbc_decrypt(key, iv, e, nthreads=nt), x)
    for nbytes in (0, 1, 15, 17, 4099):
        x = g.integers(0, 256, nbytes, dtype=np.uint8)
        for off in (0, 5, (1 << 64) - 2):
            y = san.ctr_crypt(key, iv, x, offset=off, nthreads=3)
            assert np.array_equal(y, ref.ctr_crypt(key, iv, x, offset=off, nthreads=1))
for a in range(256):
    san.gf_inv(a)
    san.xtime(a)
san.gf_mul_table()
san.sbox()
san.inv_sbox()
san.inv_mix_matrix()
print("sanitized oracle ok")
"""


def _runtime(cc, name):
    out = subprocess.run([cc, "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    cc = os.environ.get("CC", "gcc")
    asan, ubsan = _runtime(cc, "libasan.so"), _runtime(cc, "libubsan.so")
    if not asan or not ubsan:
        pytest.skip("the C compiler ships no sanitizer runtimes")
    lib = obuild.build(output=str(tmp_path / "liboracle_san.so"),
                       extra_flags=("-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                                    "-fno-omit-frame-pointer", "-g"), cc=cc)
    env = dict(os.environ, LD_PRELOAD=asan + " " + ubsan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    out = subprocess.run([sys.executable, "-c", CHILD, lib], cwd=ROOT, env=env, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr[-4000:]
    assert "sanitized oracle ok" in out.stdout
