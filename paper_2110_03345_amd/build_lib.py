"""Build libstride_hip.so (HIP kernels for gfx950 + host library + C ABI) in-tree.

The kernel source is compiled with the compiler's per-kernel resource remarks;
they are kept in _build/kernel_resources.json (registers, scratch, occupancy
per kernel) so that register spills of the step kernels are caught on the
build host.  The sources compile in parallel.

Build option: STRIDE_TILE_SWEEP=1 in the environment of the build compiles
every tile shape the launch-shape sweeps try and lets the library read its
shape from the environment at plan creation (sweeps only; the default build
has fixed shapes and reads no environment variable).
"""
import json
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libstride_hip.so")
SOURCES = ["csrc/step3d_adj.hip", "csrc/step3d_fwd.hip", "csrc/step2d.hip", "csrc/stride_kernels.hip",
           "csrc/stride_api.cpp", "csrc/stride_engine.cpp", "csrc/revolve.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# roctx trace ranges around the entry points (recorded only under a tool)
LINK_LIBS = ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx"]
ARCH = os.environ.get("STRIDE_ARCH", "gfx950")

# Packed-FP32 instructions stay disabled: the kernels are plain scalar FP32.
GPU_FLAGS = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
RESOURCES = os.path.join(HERE, "_build", "kernel_resources.json")
_KEYS = {"VGPRs": "vgpr", "AGPRs": "agpr", "SGPRs": "sgpr", "ScratchSize [bytes/lane]": "scratch",
         "Occupancy [waves/SIMD]": "occupancy", "LDS Size [bytes/block]": "lds"}


def parse_resources(remarks: str) -> dict:
    """{mangled kernel name: {vgpr, sgpr, scratch, occupancy, lds, ...}} from
    the compiler's kernel-resource-usage remarks."""
    out, cur = {}, None
    for line in remarks.splitlines():
        m = re.search(r"Function Name: (\S+)", line)
        if m:
            cur = out.setdefault(m.group(1), {})
            continue
        for key, short in _KEYS.items():
            m = re.search(re.escape(key) + r": (\d+)", line)
            if m and cur is not None:
                cur[short] = int(m.group(1))
    return out


def build(verbose: bool = False) -> str:
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    defines = ["-DSTRIDE_TILE_SWEEP"] if os.environ.get("STRIDE_TILE_SWEEP") == "1" else []
    jobs = []
    for src in SOURCES:
        path = os.path.join(HERE, src)
        obj = os.path.join(build_dir, os.path.basename(src) + ".o")
        cmd = [HIPCC, "-x", "hip"] + GPU_FLAGS + defines + [
            "-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
            "-I" + os.path.join(ROOT, "include"), "-c", path, "-o", obj]
        kernels = src.endswith(".hip")
        if kernels:
            cmd.append("-Rpass-analysis=kernel-resource-usage")
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((src, obj, cmd, kernels,
                     subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True)))
    failed = None
    objs = []
    resources = {}
    for src, obj, cmd, kernels, proc in jobs:
        _, err = proc.communicate()
        if kernels:
            resources.update(parse_resources(err))
            err = "\n".join(l for l in err.splitlines() if "remark" not in l and l.strip()
                            and "packed-fp32-ops" not in l and "Function Name" not in l)
        if proc.returncode:
            sys.stderr.write(err)
            failed = failed or subprocess.CalledProcessError(proc.returncode, cmd)
        objs.append(obj)
    if failed:
        raise failed
    with open(RESOURCES, "w") as f:
        json.dump(resources, f, indent=0, sort_keys=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH] + objs + LINK_LIBS + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
