"""Build step for the CPU oracle (test infrastructure only).

Compiles ``aes_oracle.c`` with the system C compiler into ``liboracle.so``
next to it.  Nothing here is used by the GPU library.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(HERE, "aes_oracle.c")
LIBRARY = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-Wall", "-Wextra", "-Werror"]


def build(source: str = SOURCE, output: str = LIBRARY, extra_flags=(), cc: str | None = None) -> str:
    """Compile ``source`` into the shared library ``output``; returns ``output``."""
    cc = cc or os.environ.get("CC", "gcc")
    tmp = output + ".tmp%d" % os.getpid()
    cmd = [cc, *CFLAGS, *extra_flags, source, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, output)
    return output


def is_stale(source: str = SOURCE, output: str = LIBRARY) -> bool:
    return not os.path.exists(output) or os.path.getmtime(output) < os.path.getmtime(source)


if __name__ == "__main__":
    print(build(*sys.argv[1:2]))
