"""Build libblgpu.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "blgpu.hip")
LIB = os.path.join(HERE, "libblgpu.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# FP32 division and square root need not be correctly rounded (a few ulp):
# only the mixed form's FP32 arithmetic and the step network use them, both
# far coarser than that.  FP32 values below 2^-126 are flushed to zero, which
# lets a division or square root be one hardware instruction instead of a
# scaled sequence: the mixed form keeps its quantities many decades above
# that range (intensities in camera units), so nothing it computes is lost.
# FP64 code is unaffected by both.
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-fno-hip-fp32-correctly-rounded-divide-sqrt", "-fgpu-flush-denormals-to-zero",
         "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]


def build(verbose=False, extra=()):
    cmd = [HIPCC] + FLAGS + list(extra) + ["-o", LIB + ".tmp", SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
