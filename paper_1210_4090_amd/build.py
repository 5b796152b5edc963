"""Build step of the HIP library (liblo.so, gfx950) -- run in-tree on the CPU.

hipcc cross-compiles for gfx950 without a GPU.  Floating point is built with
-ffp-contract=off (no fused multiply-add anywhere: the sweeps must round
every sum exactly as the definition does) and packed FP32 disabled.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblo.so")
ARCH = os.environ.get("LO_OFFLOAD_ARCH", "gfx950")


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False, out: str = LIB, csrc: str = CSRC) -> str:
    """Compile every source of `csrc` to an object (in parallel), then link
    them into the shared library `out`."""
    import concurrent.futures
    import tempfile
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    flags = ["--offload-arch=%s" % ARCH, "-O3", "-std=c++17", "-fPIC",
             "-ffp-contract=off", "-fno-fast-math", "-fno-honor-nans", "-mno-amdgpu-ieee",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument",
             "-I", os.path.join(ROOT, "include"), "-I", csrc]
    srcs = sorted(glob.glob(os.path.join(csrc, "*.hip")))
    with tempfile.TemporaryDirectory(prefix="lo_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(f) + ".o") for f in srcs]

        def compile_one(i):
            cmd = [hipcc] + flags + ["-c", srcs[i], "-o", objs[i]]
            if verbose:
                print(" ".join(cmd), flush=True)
            subprocess.check_call(cmd)

        with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
            list(ex.map(compile_one, range(len(srcs))))
        tmp = out + ".tmp%d" % os.getpid()
        cmd = [hipcc, "--offload-arch=%s" % ARCH, "-shared", "-fPIC", "-o", tmp] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
