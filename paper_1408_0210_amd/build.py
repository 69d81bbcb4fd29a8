"""Build libeifmm.so in-tree with hipcc for gfx950."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libeifmm.so")
SOURCES = ["capi.hip", "tree.hip", "pass.hip", "scan.hip", "eim_gpu.hip", "setup.cpp"]
ARCH = "gfx950"

# Packed FP32 instructions stay disabled for every device code object.
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Xclang", "-target-feature",
             "-Xclang", "-packed-fp32-ops", "-Wall", "-Wno-unused-function",
             "-Wno-unused-variable", "-Wno-unused-value", "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]


def build(verbose=False):
    """Compile every source to an object, then link the shared library."""
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    objs = []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(bdir, src + ".o")
        if src.endswith(".cpp"):
            # host-only setup: no FMA contraction so the EIM arithmetic is the
            # plain sequence of products and differences
            cmd = ["hipcc", "-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-x", "c++",
                   "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include",
                   "-I", os.path.join(ROOT, "include"), "-c", path, "-o", obj]
        else:
            cmd = ["hipcc", *HIP_FLAGS, "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lpthread"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
