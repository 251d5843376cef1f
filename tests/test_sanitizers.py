"""Address and undefined-behaviour sanitizer builds, run on the host:

- the oracle (plain C) with a driver that calls every entry point on small 2D
  and 3D grids (tests/sanitize/oracle_driver.c);
- the library with its host code instrumented (the C ABI, plans, workspace
  layout, checkpointing schedule, engine bookkeeping; the device code is the
  ordinary build), loaded into a Python subprocess with the sanitizer runtime
  preloaded, whose host-only paths tests/sanitize/host_driver.py drives.

Any sanitizer report aborts the run and fails the test."""
import glob
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2110_03345_amd", "csrc")
BUILD = os.path.join(ROOT, "paper_2110_03345_amd", "_build")
HIPCC = "/opt/rocm/bin/hipcc"
SAN = "address,undefined"


def test_oracle_under_sanitizers():
    if not shutil.which("gcc"):
        pytest.skip("no gcc")
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "oracle_driver")
        subprocess.run(["gcc", "-g", "-O1", "-fsanitize=" + SAN, "-fno-sanitize-recover=all",
                        "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "stride_oracle.c"),
                        os.path.join(HERE, "oracle_driver.c"), "-o", exe, "-lm"], check=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "ok" in r.stdout, r.stdout + r.stderr


def _asan_runtime():
    hits = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    return hits[0] if hits else None


def test_host_library_under_sanitizers():
    kernels = [os.path.join(BUILD, f + ".o") for f in
               ("step3d_adj.hip", "step3d_fwd.hip", "step2d.hip", "stride_kernels.hip")]
    runtime = _asan_runtime()
    if not os.path.exists(HIPCC) or not runtime or not all(os.path.exists(k) for k in kernels):
        pytest.skip("needs hipcc, its sanitizer runtime and the built kernel objects")
    with tempfile.TemporaryDirectory() as tmp:
        procs, objs = [], []
        for src in ("stride_api.cpp", "stride_engine.cpp", "revolve.cpp"):
            obj = os.path.join(tmp, src + ".o")
            cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-Xclang", "-target-feature",
                   "-Xclang", "-packed-fp32-ops", "-O1", "-g", "-std=c++17", "-fPIC",
                   "-Xarch_host", "-fsanitize=" + SAN,
                   "-Xarch_host", "-fno-omit-frame-pointer",
                   "-I" + os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, src), "-o", obj]
            procs.append(subprocess.Popen(cmd, stderr=subprocess.DEVNULL))
            objs.append(obj)
        assert all(p.wait() == 0 for p in procs)
        lib = os.path.join(tmp, "libstride_san.so")
        subprocess.run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950",
                        "-Xarch_host", "-fsanitize=" + SAN] + objs + kernels +
                       ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocprofiler-sdk-roctx",
                        "-o", lib],
                       check=True, stderr=subprocess.DEVNULL)
        env = dict(os.environ, LD_PRELOAD=runtime,
                   ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = subprocess.run([sys.executable, os.path.join(HERE, "host_driver.py"), lib], env=env,
                           capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout[-2000:] + r.stderr[-4000:]
