"""Build librsft.so in-tree with hipcc for gfx950: every source compiled to
an object in parallel, then one shared-library link."""

import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["fold.hip", "dft.hip", "vote.hip", "estimate.hip", "refine.hip", "plan.cpp", "design.cpp"]
OUTPUT = os.path.join(HERE, "librsft.so")

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _report(res, verbose):
    if verbose or res.returncode != 0:
        # hipcc's host pass does not know the packed-fp32 feature: harmless
        lines = [ln for ln in (res.stdout + res.stderr).splitlines()
                 if "packed-fp32-ops" not in ln]
        if lines:
            print("\n".join(lines))


def build_library(verbose=False):
    """Compile every HIP/C++ source into paper_1610_01050_amd/librsft.so.
    Always recompiles. Raises CalledProcessError on failure."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    with tempfile.TemporaryDirectory(prefix="rsft_build_") as tmpdir:
        procs = []
        objs = []
        for src in SOURCES:
            obj = os.path.join(tmpdir, src + ".o")
            cmd = [hipcc] + FLAGS + inc + ["-c", os.path.join(CSRC, src), "-o", obj]
            procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                                text=True)))
            objs.append(obj)
        failed = None
        for cmd, pr in procs:
            out, err = pr.communicate()
            res = subprocess.CompletedProcess(cmd, pr.returncode, out, err)
            _report(res, verbose)
            if res.returncode != 0 and failed is None:
                failed = res
        if failed is not None:
            raise subprocess.CalledProcessError(failed.returncode, failed.args, failed.stdout, failed.stderr)
        tmp = OUTPUT + ".tmp"
        cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
        res = subprocess.run(cmd, capture_output=True, text=True)
        _report(res, verbose)
        if res.returncode != 0:
            raise subprocess.CalledProcessError(res.returncode, cmd, res.stdout, res.stderr)
    os.replace(tmp, OUTPUT)
    return OUTPUT


if __name__ == "__main__":
    print(build_library(verbose=True))
