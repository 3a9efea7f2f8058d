"""Compile the C oracle (``ac_oracle.c``) into ``libacoracle.so`` with gcc.

Test infrastructure: building the checker is not using it.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ac_oracle.c")
# ORACLE_LIBRARY points the tests at another build (the sanitized one)
LIB = os.environ.get("ORACLE_LIBRARY") or os.path.join(HERE, "libacoracle.so")


def build(src: str = SRC, out: str = LIB, extra=(), cc: str = "gcc") -> str:
    tmp = out + ".tmp"
    cmd = [cc, "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-Wextra",
           *extra, src, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(), file=sys.stderr)
