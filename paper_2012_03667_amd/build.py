"""Builds the gfx950 shared library libqdse.so in-tree with hipcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqdse.so")
SOURCES = ["qdse_grid.cpp", "qdse_kernels.hip", "qdse_persistent.hip", "qdse_mfma.hip",
           "qdse_mu.hip", "qdse_api.cpp", "qdse_mu_api.cpp", "qdse_fred.hip", "qdse_fred_api.cpp", "qdse_peaks.hip",
           "qdse_band.hip", "qdse_noalloc.hip"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950",
    # no packed FP32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # matrix-core accumulators in VGPRs: with the default form the allocator
    # splits them between VGPRs and AGPRs and copies half of them every
    # k-step of the contraction loop
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    srcs = [os.path.join(CSRC, f) for f in SOURCES if os.path.exists(os.path.join(CSRC, f))]
    tmp = LIB + ".tmp"
    cmd = [hipcc] + HIPCC_FLAGS + srcs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd, cwd=CSRC)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
