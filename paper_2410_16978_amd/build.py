"""Build the HIP rasterizer library (paper_2410_16978_amd/libgsr.so) for gfx950.

Every source is compiled by hipcc for gfx950 only.  Packed FP32 instructions
are disabled (-packed-fp32-ops).  The projection and the blend are compiled
without implicit FMA contraction: the projection must reproduce the oracle's
records and keys bit for bit, and the blend's forward and backward must take
identical skip decisions (it writes its FMAs explicitly).
"""
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgsr.so")
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-Wall", "-Wno-unused-function"]
SOURCES = {
    "project.hip": ["-ffp-contract=off"],
    "pairs.hip": [],
    "sort.hip": [],
    "blend.hip": ["-ffp-contract=off"],
    "project_bwd.hip": [],
    "loss.hip": [],
    "train.hip": [],
    "api.cpp": ["-x", "hip"],
}


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose=False, jobs=6):
    hipcc = os.environ.get("HIPCC", "hipcc")
    with tempfile.TemporaryDirectory(prefix="gsr_build_") as tmp:
        objs, procs = [], []
        for src, extra in SOURCES.items():
            obj = os.path.join(tmp, src + ".o")
            cmd = [hipcc, *COMMON, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd)))
            objs.append(obj)
            while len([p for _, p in procs if p.poll() is None]) >= jobs:
                procs[0][1].wait()
        failed = [src for src, p in procs if p.wait() != 0]
        if failed:
            raise RuntimeError(f"hipcc failed for {failed}")
        tmp_lib = LIB + ".tmp"
        _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp_lib, *objs], verbose)
        os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
