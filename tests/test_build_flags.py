"""The library's compiler flags (CPU only): gfx950, packed FP32 off, multiply-adds
fused within an expression only (so that the kernels' rounding does not depend
on how the compiler splits the code into blocks), and a kernel hash that
changes with the flags (the committed traffic profile is keyed on it)."""
import bench
from paper_2605_29155_amd import build


def test_flags():
    f = build.FLAGS
    assert "--offload-arch=gfx950" in f
    assert "-ffp-contract=on" in f
    i = f.index("-packed-fp32-ops")
    assert f[i - 1] == "-Xclang" and f[i - 2] == "-target-feature"


def test_kernel_hash_covers_the_flags(monkeypatch):
    h0 = bench.kernel_source_hash()
    monkeypatch.setattr(build, "FLAGS", [x for x in build.FLAGS if x != "-ffp-contract=on"])
    assert bench.kernel_source_hash() != h0
