"""Build the gfx950 HIP library libgic.so (the C ABI of include/gic.h) and the
input generator's helper, in-tree, with hipcc.

    python -m paper_2504_00745_amd.build [-v]
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgic.so")
RSA_LIB = os.path.join(HERE, "libgicrsa.so")
HIP_SOURCES = ["gic_api.hip", "sort.hip", "contact.hip", "transfer.hip", "integrate.hip", "adjoint.hip", "step.hip", "idp.hip"]
ARCH = "gfx950"

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-result",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc():
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    return os.path.join(rocm, "bin", "hipcc")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in HIP_SOURCES if os.path.exists(os.path.join(CSRC, s))]
    cmd = [hipcc()] + HIPCC_FLAGS + ["-I", os.path.join(os.path.dirname(HERE), "include"), "-o", LIB + ".tmp"] + srcs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-o", RSA_LIB + ".tmp", os.path.join(CSRC, "rsa.c"), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(RSA_LIB + ".tmp", RSA_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
