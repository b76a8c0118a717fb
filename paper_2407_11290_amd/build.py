"""Build the gfx950 HIP library paper_2407_11290_amd/libttcross.so with hipcc.

Flags: gfx950 code object only, no floating-point contraction beyond the
explicit fma calls in the kernels (the FP64 path is meant to be bitwise
reproducible), and no packed FP32 instructions.
"""
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libttcross.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


LIB_STAMPS = os.path.join(HERE, "libttcross_stamps.so")


def build(verbose=False, stamps=False):
    """Compile every HIP source into the shared library (always recompiles).
    stamps=True builds the instrumented variant libttcross_stamps.so, whose
    search and commit kernels record phase times (tt_cross_get_stamps)."""
    out = LIB_STAMPS if stamps else LIB
    tmp = out + ".tmp"
    cmd = [HIPCC, *FLAGS, *(["-DTT_STAMPS"] if stamps else []), "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
