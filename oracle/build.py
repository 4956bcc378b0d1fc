"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, IEEE double arithmetic (no fast-math, no FMA contraction), so the
oracle's rounding is that of the written expressions.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")
SRC = [os.path.join(HERE, "dmpc_oracle.c")]
DEPS = SRC + [os.path.join(HERE, "dmpc_oracle.h"), os.path.join(HERE, "dyn_impl.inc")]


def build(force: bool = True) -> str:
    if not force and os.path.exists(LIB):
        newest = max(os.path.getmtime(p) for p in DEPS)
        if os.path.getmtime(LIB) >= newest:
            return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-Wno-unused-function", "-o", tmp] + SRC + ["-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
