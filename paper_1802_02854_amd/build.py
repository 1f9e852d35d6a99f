"""Build libftkw.so and its debug twin libftkw_check.so (HIP, gfx950) in-tree with hipcc.

python -m paper_1802_02854_amd.build   (also called by __graft_entry__.build())
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libftkw.so")
SOURCES = ["kernels.hip", "cocg.hip", "capi.cpp", "host_math.cpp", "server.cpp"]

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # the arithmetic contract: no implicit fused multiply-add anywhere
    "-ffp-contract=off",
    # no packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
    "-Wno-unused-result",
    "-pthread",
]


# the debug build: device bounds checks on every gather/scatter index (ftk_device_checks)
LIB_CHECK = os.path.join(HERE, "libftkw_check.so")
VARIANTS = [(LIB, [], ""), (LIB_CHECK, ["-DFTK_DEVICE_CHECKS"], "_check")]


def build(verbose=False):
    """Builds both libraries; the translation units of both compile in parallel."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    procs, links = [], []
    for lib, extra, tag in VARIANTS:
        objs = []
        for src in SOURCES:
            obj = os.path.join(CSRC, os.path.splitext(src)[0] + tag + ".o")
            cmd = [hipcc, *FLAGS, *extra, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((cmd, subprocess.Popen(cmd)))
            objs.append(obj)
        links.append((lib, objs))
    for cmd, p in procs:
        if p.wait() != 0:
            raise subprocess.CalledProcessError(p.returncode, cmd)
    for lib, objs in links:
        cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", lib + ".tmp", *objs]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(lib + ".tmp", lib)
        for o in objs:
            os.remove(o)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
