"""Build libaesgpu.so for gfx950 in-tree with hipcc.

    python -m paper_1902_05234_amd.build

The library is written to ``paper_1902_05234_amd/libaesgpu.so``; objects go to
``paper_1902_05234_amd/_build/``.  hipcc cross-compiles for gfx950, so no GPU
is needed to build.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIBRARY = os.path.join(HERE, "libaesgpu.so")
INCLUDE = os.path.join(ROOT, "include")

ARCH = os.environ.get("AESGPU_ARCH", "gfx950")
SOURCES = ["aes_ecb_p4.hip", "aes_ecb_p2.hip", "aes_ecb_p1.hip", "aes_ecb_col.hip", "aes_ecb.hip", "aes_ctr.hip", "aes_cbc.hip", "aes_cbc_msgs.hip", "aes_host_word.hip", "aes_bitslice.hip", "aes_microbench.hip", "aes_batch.hip", "aes_abi.cpp", "aes_serve.cpp", "aes_pipe.cpp"]
HEADERS = ["aes_sbox_circuit.hpp", "aes_device.hpp", "aes_ecb_kernel.hpp", "aes_internal.hpp", "aes_tables.hpp",
           "aes_batch_signal.hpp", "aes_cbc_msgs.hpp", "aes_col_round.hpp", "aes_host_word.hpp", "aes_tune_defaults.inc"]

# Packed-FP32 instruction forms stay off for every GPU compile.
COMMON = [
    "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-command-line-argument",
    "--offload-arch=" + ARCH, "-I" + INCLUDE, "-I" + CSRC,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; the ROCm toolchain is required to build libaesgpu")
    return exe


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *COMMON, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return obj


def build(verbose: bool = False) -> str:
    """Compile every source and link the shared library; returns its path."""
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIBRARY + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIBRARY)
    if verbose:
        print("built", LIBRARY)
    return LIBRARY


def is_stale() -> bool:
    if not os.path.exists(LIBRARY):
        return True
    t = os.path.getmtime(LIBRARY)
    deps = [os.path.join(CSRC, f) for f in SOURCES + HEADERS] + [os.path.join(INCLUDE, "aesgpu.h")]
    return any(os.path.getmtime(d) > t for d in deps)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
