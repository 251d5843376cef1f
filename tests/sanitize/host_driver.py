"""Drives the host-only paths of a sanitizer build of the library (run by
tests/test_sanitizers.py in a subprocess with the ASan runtime preloaded):
grid and geometry validation, workspace sizes for every mode, the binomial
schedule for many step and field counts, the gradient path (full, segmented
or binomial) for many workspace sizes, error strings and switches, and
plan creation up to the first device call (which fails on a host without a
GPU).  Prints "ok" when every call returned as expected."""
import ctypes
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from paper_2110_03345_amd._abi import make_grid  # noqa: E402  (struct only; loads nothing)

L = ctypes.CDLL(sys.argv[1])
sz = ctypes.c_size_t
i32, i64 = ctypes.c_int32, ctypes.c_int64
dp = ctypes.POINTER(ctypes.c_double)
L.stride_workspace_query.argtypes = [ctypes.c_void_p, i32, i32, i32, sz, ctypes.POINTER(sz)]
L.stride_schedule_info.argtypes = [i32, i64, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i32)]
L.stride_plan_create.argtypes = [ctypes.c_void_p, i32, dp, i32, dp, ctypes.POINTER(ctypes.c_void_p)]
L.stride_error_string.restype = ctypes.c_char_p
L.stride_last_error.restype = ctypes.c_char_p
L.stride_engine_create.argtypes = [ctypes.c_void_p, i32, i32, i32, i32, ctypes.POINTER(ctypes.c_void_p)]
L.stride_gradient_path.argtypes = [ctypes.c_void_p, i32, sz, ctypes.POINTER(i32), ctypes.POINTER(i64),
                                   ctypes.POINTER(i32)]

calls = 0
for nd, shape in ((2, (40, 51)), (3, (17, 19, 23))):
    for order in (6, 8, 10):
        for torder in (2, 4, 3):
            for boundary in (0, 1, 2):
                for interp in (0, 1, 5):
                    g = make_grid(shape, 0.3e-3, order, 6, 1500.0, 5e-8, 37, torder, interp, boundary)
                    for mode in (0, 1, 2, 3, 7):
                        for budget in (0, 1 << 20, 1 << 40):
                            out = sz(0)
                            L.stride_workspace_query(ctypes.byref(g), 2, 5, mode, budget, ctypes.byref(out))
                            calls += 1
                            L.stride_last_error()
snaps, steps, peak = i32(), i64(), i32()
for nt in list(range(2, 90)) + [500, 3000]:
    for fields in (3, 4, 5, 9, nt // 3 + 3, nt + 4):
        L.stride_schedule_info(nt, fields, ctypes.byref(snaps), ctypes.byref(steps), ctypes.byref(peak))
        calls += 1
path, fsteps, nseg = i32(), i64(), i32()
for nd, shape in ((2, (40, 51)), (3, (17, 19, 23))):
    for nt in (2, 3, 17, 64, 301):
        for torder in (2, 4):
            for ck in (0, 1):
                g = make_grid(shape, 0.3e-3, 8, 6, 1500.0, 5e-8, nt, torder, 0, 0, ck)
                full = sz(0)
                L.stride_workspace_query(ctypes.byref(g), 1, 5, 1, 0, ctypes.byref(full))
                for frac in (0.01, 0.05, 0.1, 0.2, 0.35, 0.5, 0.7, 0.9, 1.0, 1.5):
                    L.stride_gradient_path(ctypes.byref(g), 5, int(full.value * frac),
                                           ctypes.byref(path), ctypes.byref(fsteps),
                                           ctypes.byref(nseg))
                    calls += 1
for code in range(-8, 2):
    L.stride_error_string(code)
L.stride_check_finite(0)
L.stride_check_finite(1)
L.stride_timing_enable(1)
L.stride_timing_enable(0)
# plan creation: invalid geometry fails in validation; a valid one reaches the
# first device allocation
g = make_grid((40, 51), 0.3e-3, 8, 6, 1500.0, 5e-8, 37)
plan = ctypes.c_void_p()
bad = (ctypes.c_double * 2)(1.0, 1.0)
good = (ctypes.c_double * 4)(1e-3, 2e-3, 4e-3, 5e-3)
rc_bad = L.stride_plan_create(ctypes.byref(g), 1, bad, 2, good, ctypes.byref(plan))
rc_any = L.stride_plan_create(ctypes.byref(g), 1, good, 2, good, ctypes.byref(plan))
eng = ctypes.c_void_p()
rc_eng = L.stride_engine_create(ctypes.byref(g), 0, 0, 0, 0, ctypes.byref(eng))
assert rc_bad == -3 and rc_eng == -1, (rc_bad, rc_eng)
print(f"ok ({calls} calls; plan creation on this host returned {rc_any})")
