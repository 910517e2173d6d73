"""Builds libpp.so for gfx950 with hipcc (cross-compiles; no GPU needed).

Run ``python -m paper_2411_01919_amd.build`` from the repository root, or call
``build()``.  Every HIP source is compiled with packed FP32 instructions
disabled and FP contraction off (FMAs are written explicitly where wanted).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpp.so")
SOURCES = ["csrc/pp_kernels.hip", "csrc/pp_regions.hip", "csrc/pp_segment.hip", "csrc/pp_polygons.cpp", "csrc/pp_map.cpp", "csrc/pp_api.hip", "csrc/pp_server.hip"]
ARCH = os.environ.get("PP_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    f"--offload-arch={ARCH}",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    # matrix-core results straight into VGPRs (no accumulation-register round trip)
    "-mllvm", "-amdgpu-mfma-vgpr-form",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(HERE, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"), *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=HERE)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
