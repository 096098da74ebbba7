"""Build ``libmclbm.so`` (HIP kernels + C ABI) for gfx950, in-tree.

Run ``python -m paper_2207_01534_amd.build`` (or call :func:`build`).  The
library is written next to this file; tests, the smoke check and the
benchmark load it from there and never build it themselves.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmclbm.so")
SOURCES = [os.path.join(CSRC, "lbm_kernels.hip"), os.path.join(CSRC, "lbm_adjoint.hip"),
           os.path.join(CSRC, "lbm_open.hip"), os.path.join(CSRC, "mclbm_api.cpp")]
HEADERS = [os.path.join(CSRC, "lbm_device.hpp"), os.path.join(CSRC, "lbm_tiles.hpp"),
           os.path.join(CSRC, "lbm_kernels.hpp"),
           os.path.join(CSRC, "lbm_adjoint.hpp"), os.path.join(CSRC, "lbm_open.hpp"),
           os.path.join(ROOT, "include", "mclbm.h")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def build(verbose: bool = False, extra=()) -> str:
    cmd = [HIPCC, "-x", "hip", "-std=c++17", "-O3", f"--offload-arch={ARCH}", "-fPIC", "-shared",
           "-Wall", "-Wno-unused-function",
           # packed FP32 instructions stay off (they have given wrong results)
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), *extra, *SOURCES, "-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops' is not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + errs)
    if verbose and errs.strip():
        print(errs)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
