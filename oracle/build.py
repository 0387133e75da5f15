"""Build the oracle's C helpers (test infrastructure only).

``oracle/eft_c.c`` holds the compensated products of ``oracle.eft`` in plain
C with OpenMP threads; ``oracle.eft`` loads ``oracle/_eft_c.so`` when it is
built and otherwise runs the numpy forms, which give the same bits.
"""

from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "eft_c.c")
LIB = os.path.join(HERE, "_eft_c.so")


def build() -> str:
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           SRC, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("gcc failed for the oracle helpers:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
