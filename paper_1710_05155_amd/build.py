"""Build libka.so (host C++ + gfx950 HIP kernels) in-tree with hipcc."""
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libka.so")
ARCH = os.environ.get("KA_OFFLOAD_ARCH", "gfx950")

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-I", INCLUDE, "-I", CSRC]
# No packed-FP32 instructions in any device code.
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False) -> str:
    hipcc = _hipcc()
    bdir = os.path.join(PKG, "_build")
    os.makedirs(bdir, exist_ok=True)
    k_obj = os.path.join(bdir, "ka_kernels.o")
    h_obj = os.path.join(bdir, "ka_host.o")
    _run([hipcc, *COMMON, *DEVICE, "-c", os.path.join(CSRC, "ka_kernels.hip"), "-o", k_obj], verbose)
    _run([hipcc, *COMMON, *DEVICE, "-c", os.path.join(CSRC, "ka_host.cpp"), "-o", h_obj], verbose)
    tmp = LIB + ".tmp"
    _run([hipcc, *DEVICE, "-shared", "-fPIC", k_obj, h_obj, "-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
