"""Build librsft.so in-tree with hipcc for gfx950."""

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["fold.hip", "dft.hip", "vote.hip", "estimate.hip", "refine.hip", "plan.cpp", "design.cpp"]
OUTPUT = os.path.join(HERE, "librsft.so")

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build_library(verbose=False):
    """Compile every HIP/C++ source into paper_1610_01050_amd/librsft.so.
    Always recompiles. Raises CalledProcessError on failure."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = OUTPUT + ".tmp"
    cmd = [hipcc] + FLAGS + ["-I", os.path.join(ROOT, "include"), "-I", CSRC,
                             "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if verbose or res.returncode != 0:
        # hipcc's host pass does not know the packed-fp32 feature: harmless
        lines = [ln for ln in (res.stdout + res.stderr).splitlines()
                 if "packed-fp32-ops" not in ln]
        if lines:
            print("\n".join(lines))
    if res.returncode != 0:
        raise subprocess.CalledProcessError(res.returncode, cmd, res.stdout, res.stderr)
    os.replace(tmp, OUTPUT)
    return OUTPUT


if __name__ == "__main__":
    print(build_library(verbose=True))
