"""Build liblik.so (HIP kernels + C ABI) for gfx950, in-tree.

Floating-point flags matter for reproducibility: no FMA contraction (every
fused multiply-add is written explicitly), IEEE-correct binary32 division and
square root, no flush of denormals, and packed-FP32 instructions disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblik.so")
SOURCES = ["kernels.hip", "api.cpp"]

HIP_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


def hip_runtime_dir():
    """Directory of the HIP runtime the process will use.  PyTorch-ROCm ships
    its own libamdhip64/libhsa-runtime64; linking against that copy keeps a
    single HIP runtime in processes that also use torch for device memory and
    streams (two runtimes in one process do not share initialisation)."""
    try:
        import torch
        d = os.path.join(os.path.dirname(torch.__file__), "lib")
        if os.path.exists(os.path.join(d, "libamdhip64.so")):
            return d
    except ImportError:
        pass
    return "/opt/rocm/lib"


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc, *HIP_FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    rt = hip_runtime_dir()
    # plain host link (no -fgpu-rdc: device code is already embedded per object)
    cmd = ["g++", "-shared", "-fPIC", "-o", tmp, *objs, f"-L{rt}", f"-Wl,-rpath,{rt}",
           "-l:libamdhip64.so", "-Wl,--no-undefined"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
