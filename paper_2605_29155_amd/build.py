"""Build the HIP library libdmpc.so for gfx950 (in-tree, next to this file)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libdmpc.so")
SRC = os.path.join(HERE, "csrc", "dmpc.hip")
DEPS = [SRC, os.path.join(HERE, "csrc", "dmpc_device.hpp"), os.path.join(HERE, "csrc", "dmpc_theta.hpp"),
        os.path.join(ROOT, "include", "dmpc.h")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # packed FP32 VALU ops stay disabled: they are not used by this library
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # a multiply and an add are fused only where one expression holds both
         # (or fmaf says so), never across statements: the arithmetic then does
         # not depend on how the code is split into blocks
         "-ffp-contract=on",
         "-I" + os.path.join(ROOT, "include")]


# measured FMA and copy rates (the roofline's ceilings), a separate small library
PEAKS_LIB = os.path.join(HERE, "libdmpc_peaks.so")
PEAKS_SRC = os.path.join(HERE, "csrc", "peaks.hip")


def build(force: bool = True) -> str:
    for lib, src, deps in ((LIB, SRC, DEPS), (PEAKS_LIB, PEAKS_SRC, [PEAKS_SRC])):
        if not force and os.path.exists(lib) and os.path.getmtime(lib) >= max(os.path.getmtime(p) for p in deps):
            continue
        tmp = lib + ".tmp"
        subprocess.run([HIPCC] + FLAGS + [src, "-o", tmp], check=True)
        os.replace(tmp, lib)
    return LIB


if __name__ == "__main__":
    print(build(force="--if-stale" not in sys.argv))
