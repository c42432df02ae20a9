"""Build libaalcsim.so (gfx950) in-tree with hipcc.

Flags that the arithmetic depends on:
  -ffp-contract=off   every multiply and add rounds on its own (no FMA), so
                      codes and streams are reproducible bit for bit;
  no fast-math        IEEE division and square root, NaN/inf semantics;
  -Xclang -target-feature -Xclang -packed-fp32-ops
                      no packed FP32 instructions are generated.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libaalcsim.so")
ROOT = os.path.dirname(HERE)
SOURCES = ["kernels.hip", "sv.hip", "entropy.hip", "sim.cpp"]
HEADERS = ["device.h", "gates.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


def build(verbose=False):
    """Compile every HIP source into the in-tree shared library."""
    srcs = [os.path.join(CSRC, f) for f in SOURCES]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC] + FLAGS + srcs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)
