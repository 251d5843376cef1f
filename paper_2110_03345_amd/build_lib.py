"""Build libstride_hip.so (HIP kernels for gfx950 + host library + C ABI) in-tree."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libstride_hip.so")
SOURCES = ["csrc/stride_kernels.hip", "csrc/stride_api.cpp", "csrc/stride_engine.cpp",
           "csrc/revolve.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("STRIDE_ARCH", "gfx950")

# Packed-FP32 instructions stay disabled: the kernels are plain scalar FP32.
GPU_FLAGS = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    objs = []
    for src in SOURCES:
        path = os.path.join(HERE, src)
        obj = os.path.join(build_dir, os.path.basename(src) + ".o")
        cmd = [HIPCC, "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
               "-I" + os.path.join(ROOT, "include"), "-c", path, "-o", obj]
        cmd[1:1] = ["-x", "hip"] + GPU_FLAGS
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
