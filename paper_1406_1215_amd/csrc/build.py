"""Build libclgen.so (HIP, gfx950) in-tree, and libclceil.so (the memory
ceilings the benchmark measures beside the generation kernel).

One translation unit per library (cl_api.hip includes the kernel headers).
Floating-point contraction is off so that every binary64 operation of the
sampler is one IEEE-754 operation; packed fp32 instructions are disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libclgen.so")
SOURCES = ["cl_api.hip"]
CEIL_LIB = os.path.join(PKG, "libclceil.so")
CEIL_SOURCES = ["cl_ceilings.hip"]
HEADERS = ["cl_device.hpp", "cl_plan.hpp", "cl_scan.hpp", "cl_kernels.hpp", "cl_stats.hpp", "cl_expdeg.hpp"]


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def command(out: str, sources=SOURCES):
    return [
        hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
        "-ffp-contract=off", "-fno-fast-math",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"), "-I", HERE,
        *[os.path.join(HERE, s) for s in sources],
        "-o", out,
    ]


def _build_one(lib: str, sources, verbose: bool) -> str:
    tmp = lib + ".tmp"
    cmd = command(tmp, sources)
    if verbose:
        print(" ".join(cmd))
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        sys.stderr.write(err + "\n")
        raise RuntimeError("hipcc failed")
    if verbose and err.strip():
        sys.stderr.write(err + "\n")
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    _build_one(CEIL_LIB, CEIL_SOURCES, verbose)
    return _build_one(LIB, SOURCES, verbose)


if __name__ == "__main__":
    print(build(verbose=True))
