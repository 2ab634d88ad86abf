"""Build libhyb.so (HIP kernels + C ABI) in-tree for gfx950 with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["lbm_kernels.hip", "adjoint_kernels.hip", "coarse_kernels.hip", "coarse_adjoint.hip", "coarse_setup.hip",
           "dissolve_kernels.hip", "diag_kernels.hip", "hyb1d.hip",
           "hyb_api.hip"]
LIB = os.path.join(HERE, "libhyb.so")
ARCH = "gfx950"


def hipcc_command(out=LIB):
    return (["/opt/rocm/bin/hipcc", "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-result", "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", out]
            + [os.path.join(CSRC, s) for s in SOURCES])


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = hipcc_command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
