"""ctypes binding of libstride_hip.so (include/stride_hip.h).

Argument marshalling only: every step of the solves runs in the HIP library.
torch supplies device memory and the current stream.  When the library is
missing this module raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstride_hip.so")

STRIDE_OK = 0
STRIDE_E_INVALID_ARG = -1
STRIDE_E_CFL = -2
STRIDE_E_GEOMETRY = -3
STRIDE_E_WORKSPACE = -4
STRIDE_E_HIP = -5
STRIDE_E_NONFINITE = -6
STRIDE_MODE_FORWARD = 0
STRIDE_MODE_GRADIENT = 1
STRIDE_MODE_FORWARD_MEDIUM = 2
STRIDE_MODE_GRADIENT_MEDIUM = 3

EXPORTS = (
    "stride_plan_create", "stride_plan_destroy", "stride_plan_padded_shape",
    "stride_workspace_bytes", "stride_plan_forward", "stride_plan_forward_static",
    "stride_plan_forward_medium", "stride_plan_gradient_medium", "stride_lowpass",
    "stride_descent_step",
    "stride_forward_save", "stride_backward",
    "stride_plan_gradient", "stride_forward", "stride_gradient", "stride_workspace_query",
    "stride_schedule_info", "stride_gradient_path", "stride_last_error", "stride_error_string",
    "stride_timing_enable", "stride_timing_read", "stride_check_finite",
    "stride_engine_create", "stride_engine_destroy", "stride_engine_attach", "stride_engine_run",
    "stride_engine_detach", "stride_engine_slot_ticks", "stride_accumulate",
)


class StrideError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class stride_grid_t(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int32),
        ("space_order", ctypes.c_int32),
        ("sponge_cells", ctypes.c_int32),
        ("nt", ctypes.c_int32),
        ("shape", ctypes.c_int64 * 3),
        ("spacing", ctypes.c_double * 3),
        ("sponge_vref", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("time_order", ctypes.c_int32),
        ("interp", ctypes.c_int32),
        ("boundary", ctypes.c_int32),
        ("checkpointing", ctypes.c_int32),
    ]


_LIB = None


def lib():
    """Load the library (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp_ = ctypes.c_void_p
        i32 = ctypes.c_int32
        dp = ctypes.POINTER(ctypes.c_double)
        gp = ctypes.POINTER(stride_grid_t)
        sz = ctypes.c_size_t
        L.stride_plan_create.argtypes = [gp, i32, dp, i32, dp, ctypes.POINTER(vp_)]
        L.stride_plan_destroy.argtypes = [vp_]
        L.stride_plan_padded_shape.argtypes = [vp_, ctypes.POINTER(ctypes.c_int64)]
        L.stride_workspace_bytes.argtypes = [vp_, i32, sz, ctypes.POINTER(sz)]
        L.stride_plan_forward.argtypes = [vp_, vp_, vp_, vp_, vp_, sz, vp_]
        L.stride_plan_forward_static.argtypes = [vp_, vp_, vp_, vp_, vp_]
        L.stride_plan_forward_medium.argtypes = [vp_, vp_, vp_, vp_, i32, vp_, vp_, vp_, sz, vp_]
        L.stride_plan_gradient_medium.argtypes = [vp_, vp_, vp_, vp_, i32, vp_, vp_, vp_, vp_, vp_,
                                                  vp_, sz, vp_]
        L.stride_lowpass.argtypes = [vp_, vp_, i32, i32, ctypes.c_double, ctypes.c_double, vp_]
        L.stride_descent_step.argtypes = [vp_, vp_, vp_, ctypes.c_int64, ctypes.c_float,
                                          ctypes.c_float, ctypes.c_float, vp_, vp_]
        L.stride_forward_save.argtypes = [vp_, vp_, vp_, vp_, vp_, sz, vp_]
        L.stride_backward.argtypes = [vp_, vp_, vp_, vp_, vp_, vp_, vp_, sz, vp_]
        L.stride_plan_gradient.argtypes = [vp_, vp_, vp_, vp_, vp_, vp_, vp_, vp_, sz, vp_]
        L.stride_forward.argtypes = [gp, vp_, vp_, i32, dp, i32, dp, vp_, vp_, sz, vp_]
        L.stride_gradient.argtypes = [gp, vp_, vp_, i32, dp, i32, dp, vp_, vp_, vp_, vp_, sz, vp_]
        L.stride_workspace_query.argtypes = [gp, i32, i32, i32, sz, ctypes.POINTER(sz)]
        L.stride_schedule_info.argtypes = [i32, ctypes.c_int64, ctypes.POINTER(i32),
                                           ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(i32)]
        L.stride_gradient_path.argtypes = [gp, i32, sz, ctypes.POINTER(i32),
                                           ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(i32)]
        L.stride_timing_enable.argtypes = [i32]
        L.stride_check_finite.argtypes = [i32]
        L.stride_timing_read.argtypes = [dp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                         dp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.stride_engine_create.argtypes = [gp, i32, i32, i32, i32, ctypes.POINTER(vp_)]
        L.stride_engine_destroy.argtypes = [vp_]
        L.stride_engine_attach.argtypes = [vp_, vp_, i32, vp_, ctypes.c_float, vp_, vp_, vp_, vp_, vp_,
                                           vp_, sz, vp_, ctypes.POINTER(i32)]
        L.stride_engine_run.argtypes = [vp_, i32, vp_, ctypes.POINTER(i32), ctypes.POINTER(i32)]
        L.stride_engine_detach.argtypes = [vp_, i32]
        L.stride_engine_slot_ticks.argtypes = [vp_, i32, ctypes.POINTER(ctypes.c_int64)]
        L.stride_accumulate.argtypes = [vp_, vp_, ctypes.c_int64, vp_]
        L.stride_last_error.restype = ctypes.c_char_p
        L.stride_error_string.restype = ctypes.c_char_p
        L.stride_error_string.argtypes = [ctypes.c_int]
        _LIB = L
    return _LIB


def _check(rc: int):
    if rc != STRIDE_OK:
        msg = lib().stride_last_error().decode() or lib().stride_error_string(rc).decode()
        raise StrideError(rc, msg)


def make_grid(shape: Sequence[int], spacing, space_order: int, nb: int, vref: float, dt: float,
              nt: int, time_order: int = 2, interp: int = 0, boundary: int = 0,
              checkpointing: int = 0) -> stride_grid_t:
    g = stride_grid_t()
    nd = len(shape)
    sp = (float(spacing),) * nd if np.isscalar(spacing) else tuple(float(s) for s in spacing)
    g.ndim = nd
    g.space_order = int(space_order)
    g.sponge_cells = int(nb)
    g.nt = int(nt)
    for a in range(3):
        g.shape[a] = int(shape[a]) if a < nd else 1
        g.spacing[a] = sp[a] if a < nd else 1.0
    g.sponge_vref = float(vref)
    g.dt = float(dt)
    g.time_order = int(time_order)
    g.interp = int(interp)
    g.boundary = int(boundary)
    g.checkpointing = int(checkpointing)
    return g


def _coords(xyz, ndim) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1, ndim))
    return a


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stream(stream) -> ctypes.c_void_p:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t, shape=None, dtype=None, name="tensor"):
    """Device pointer of a contiguous CUDA tensor after checking it."""
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise StrideError(STRIDE_E_INVALID_ARG, f"{name} must be a CUDA tensor")
    if dtype is not None and t.dtype != dtype:
        raise StrideError(STRIDE_E_INVALID_ARG, f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise StrideError(STRIDE_E_INVALID_ARG, f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise StrideError(STRIDE_E_INVALID_ARG, f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    return ctypes.c_void_p(t.data_ptr())


# ----------------------------------------------------------- C-ABI mirrors

def stride_plan_create(grid: stride_grid_t, src_xyz, rec_xyz) -> ctypes.c_void_p:
    src = _coords(src_xyz, grid.ndim)
    rec = _coords(rec_xyz, grid.ndim)
    out = ctypes.c_void_p()
    _check(lib().stride_plan_create(ctypes.byref(grid), src.shape[0], _dp(src), rec.shape[0],
                                    _dp(rec), ctypes.byref(out)))
    return out


def stride_plan_destroy(plan) -> None:
    _check(lib().stride_plan_destroy(plan))


def stride_plan_padded_shape(plan):
    out = (ctypes.c_int64 * 3)()
    _check(lib().stride_plan_padded_shape(plan, out))
    return tuple(out)


def stride_workspace_bytes(plan, mode: int, budget_bytes: int = 0) -> int:
    out = ctypes.c_size_t()
    _check(lib().stride_workspace_bytes(plan, mode, budget_bytes, ctypes.byref(out)))
    return int(out.value)


def stride_workspace_query(grid: stride_grid_t, nsrc: int, nrec: int, mode: int,
                           budget_bytes: int = 0) -> int:
    out = ctypes.c_size_t()
    _check(lib().stride_workspace_query(ctypes.byref(grid), nsrc, nrec, mode, budget_bytes,
                                        ctypes.byref(out)))
    return int(out.value)


def stride_schedule_info(nt: int, fields: int):
    s = ctypes.c_int32()
    f = ctypes.c_int64()
    p = ctypes.c_int32()
    _check(lib().stride_schedule_info(nt, fields, ctypes.byref(s), ctypes.byref(f), ctypes.byref(p)))
    return int(s.value), int(f.value), int(p.value)


STRIDE_PATH_FULL_HISTORY = 0
STRIDE_PATH_SEGMENTED = 1
STRIDE_PATH_BINOMIAL = 2


def stride_gradient_path(grid, nrec: int, ws_bytes: int):
    """(path, forward steps per gradient, segments) of a gradient in a
    workspace of ws_bytes: path 0 full history, 1 segmented history, 2
    binomial checkpointing."""
    k = ctypes.c_int32()
    f = ctypes.c_int64()
    n = ctypes.c_int32()
    _check(lib().stride_gradient_path(ctypes.byref(grid), nrec, ws_bytes, ctypes.byref(k),
                                      ctypes.byref(f), ctypes.byref(n)))
    return int(k.value), int(f.value), int(n.value)


def stride_timing_enable(on: bool) -> None:
    _check(lib().stride_timing_enable(1 if on else 0))


def stride_check_finite(on: bool) -> None:
    """Scan solve outputs for NaN/Inf (STRIDE_E_NONFINITE) on this thread."""
    _check(lib().stride_check_finite(1 if on else 0))


def stride_timing_read():
    """(fwd_ms, fwd_steps, fwd_launches, adj_ms, adj_steps, adj_launches) since
    the last read."""
    f, a = ctypes.c_double(), ctypes.c_double()
    nf, lf, na, la = (ctypes.c_int64() for _ in range(4))
    _check(lib().stride_timing_read(ctypes.byref(f), ctypes.byref(nf), ctypes.byref(lf),
                                    ctypes.byref(a), ctypes.byref(na), ctypes.byref(la)))
    return f.value, int(nf.value), int(lf.value), a.value, int(na.value), int(la.value)


def stride_plan_forward(plan, vp, wavelet, traces, ws, stream=None):
    _check(lib().stride_plan_forward(plan, _dev(vp), _dev(wavelet), _dev(traces), _dev(ws),
                                     ws.numel(), _stream(stream)))


def stride_plan_forward_static(plan, vp, wavelet, traces, stream=None):
    """stride_plan_forward on the library's static device workspace (no
    allocation; STRIDE_STATIC_WORKSPACE_BYTES at most)."""
    _check(lib().stride_plan_forward_static(plan, _dev(vp), _dev(wavelet), _dev(traces),
                                            _stream(stream)))


STRIDE_STATIC_WORKSPACE_BYTES = 64 << 20


def stride_plan_forward_medium(plan, vp, rho, alpha0, att_power, wavelet, traces, ws, stream=None):
    _check(lib().stride_plan_forward_medium(plan, _dev(vp), _dev(rho), _dev(alpha0), int(att_power),
                                            _dev(wavelet), _dev(traces), _dev(ws), ws.numel(),
                                            _stream(stream)))


def stride_plan_gradient_medium(plan, vp, rho, alpha0, att_power, wavelet, observed, traces, misfit,
                                dvp, ws, stream=None):
    _check(lib().stride_plan_gradient_medium(plan, _dev(vp), _dev(rho), _dev(alpha0), int(att_power),
                                             _dev(wavelet), _dev(observed), _dev(traces),
                                             _dev(misfit), _dev(dvp), _dev(ws), ws.numel(),
                                             _stream(stream)))


def stride_lowpass(x, dt: float, f_max: float, out=None, stream=None):
    """Zero-phase low-pass of a [count][nt] float32 CUDA tensor (out may be x)."""
    import torch
    _dev(x, None, torch.float32, "signals")
    if out is None:
        out = torch.empty_like(x)
    nt = x.shape[-1]
    count = x.numel() // nt if nt else 0
    _check(lib().stride_lowpass(_dev(x), _dev(out), count, nt, float(dt), float(f_max),
                                _stream(stream)))
    return out


def stride_descent_step(vp, grad, step_size: float, vmin: float, vmax: float, work, mask=None,
                        stream=None):
    """vp = clamp(vp - step_size * m g / max|m g|, vmin, vmax) in place."""
    import torch
    _dev(vp, None, torch.float32, "vp")
    _dev(grad, tuple(vp.shape), torch.float32, "grad")
    if mask is not None:
        _dev(mask, tuple(vp.shape), torch.float32, "mask")
    _check(lib().stride_descent_step(_dev(vp), _dev(grad), _dev(mask), vp.numel(), float(step_size),
                                     float(vmin), float(vmax), _dev(work), _stream(stream)))


def stride_forward_save(plan, vp, wavelet, traces, ws, stream=None):
    _check(lib().stride_forward_save(plan, _dev(vp), _dev(wavelet), _dev(traces), _dev(ws),
                                     ws.numel(), _stream(stream)))


def stride_backward(plan, vp, wavelet, grad_traces, dvp, dwavelet, ws, stream=None):
    _check(lib().stride_backward(plan, _dev(vp), _dev(wavelet), _dev(grad_traces), _dev(dvp),
                                 _dev(dwavelet), _dev(ws), ws.numel(), _stream(stream)))


def stride_plan_gradient(plan, vp, wavelet, observed, traces, misfit, dvp, ws, stream=None):
    _check(lib().stride_plan_gradient(plan, _dev(vp), _dev(wavelet), _dev(observed), _dev(traces),
                                      _dev(misfit), _dev(dvp), _dev(ws), ws.numel(), _stream(stream)))


def stride_forward(grid: stride_grid_t, vp, wavelet, src_xyz, rec_xyz, traces, ws, stream=None):
    src = _coords(src_xyz, grid.ndim)
    rec = _coords(rec_xyz, grid.ndim)
    _check(lib().stride_forward(ctypes.byref(grid), _dev(vp), _dev(wavelet), src.shape[0], _dp(src),
                                rec.shape[0], _dp(rec), _dev(traces), _dev(ws), ws.numel(),
                                _stream(stream)))


def stride_gradient(grid: stride_grid_t, vp, wavelet, src_xyz, rec_xyz, observed, misfit, dvp, ws,
                    stream=None):
    src = _coords(src_xyz, grid.ndim)
    rec = _coords(rec_xyz, grid.ndim)
    _check(lib().stride_gradient(ctypes.byref(grid), _dev(vp), _dev(wavelet), src.shape[0], _dp(src),
                                 rec.shape[0], _dp(rec), _dev(observed), _dev(misfit), _dev(dvp),
                                 _dev(ws), ws.numel(), _stream(stream)))


def stride_engine_create(grid: stride_grid_t, max_slots: int, max_receivers: int, max_chunk: int,
                         use_graphs: bool) -> ctypes.c_void_p:
    out = ctypes.c_void_p()
    _check(lib().stride_engine_create(ctypes.byref(grid), max_slots, max_receivers, max_chunk,
                                      1 if use_graphs else 0, ctypes.byref(out)))
    return out


def stride_engine_destroy(engine) -> None:
    _check(lib().stride_engine_destroy(engine))


def stride_engine_attach(engine, plan, mode, vp, vp_max, wavelet, observed, traces, misfit, dvp,
                         ws, stream=None) -> int:
    slot = ctypes.c_int32(-1)
    _check(lib().stride_engine_attach(engine, plan, mode, _dev(vp), float(vp_max), _dev(wavelet),
                                      _dev(observed), _dev(traces), _dev(misfit), _dev(dvp), _dev(ws),
                                      ws.numel(), _stream(stream), ctypes.byref(slot)))
    return int(slot.value)


def stride_engine_run(engine, max_ticks: int, max_slots: int, stream=None):
    """(ticks enqueued, list of slots finished by this call)."""
    ticks = ctypes.c_int32(0)
    fin = (ctypes.c_int32 * max_slots)()
    _check(lib().stride_engine_run(engine, max_ticks, _stream(stream), ctypes.byref(ticks), fin))
    return int(ticks.value), [i for i in range(max_slots) if fin[i]]


def stride_engine_detach(engine, slot: int) -> None:
    _check(lib().stride_engine_detach(engine, slot))


def stride_engine_slot_ticks(engine, slot: int) -> int:
    out = ctypes.c_int64(0)
    _check(lib().stride_engine_slot_ticks(engine, slot, ctypes.byref(out)))
    return int(out.value)


def stride_accumulate(dst, src, stream=None) -> None:
    _check(lib().stride_accumulate(_dev(dst), _dev(src), dst.numel(), _stream(stream)))


# ------------------------------------------------------------- Plan object

class Plan:
    """A validated grid + shot geometry with its tap tables on the current device."""

    def __init__(self, shape, spacing, space_order, nb, vref, dt, nt, src_xyz, rec_xyz,
                 time_order: int = 2, interp: int = 0, boundary: int = 0, checkpointing: int = 0):
        self.grid = make_grid(shape, spacing, space_order, nb, vref, dt, nt, time_order, interp,
                              boundary, checkpointing)
        self.time_order = int(time_order)
        self.interp = int(interp)
        self.boundary = int(boundary)
        self.shape = tuple(int(s) for s in shape)
        self.ndim = len(self.shape)
        self.nt = int(nt)
        self.src_xyz = _coords(src_xyz, self.ndim)
        self.rec_xyz = _coords(rec_xyz, self.ndim)
        self.nsrc = self.src_xyz.shape[0]
        self.nrec = self.rec_xyz.shape[0]
        self.handle = stride_plan_create(self.grid, self.src_xyz, self.rec_xyz)

    @classmethod
    def from_workload(cls, w, src_xyz=None, rec_xyz=None, nt=None, time_order: int = 2,
                      interp: int = 0, boundary: int = 0, checkpointing: int = 0):
        return cls(w.shape, w.spacing, w.space_order, w.nb, w.vref, w.dt,
                   w.nt if nt is None else nt,
                   w.src_xyz if src_xyz is None else src_xyz,
                   w.rec_xyz if rec_xyz is None else rec_xyz, time_order, interp, boundary,
                   checkpointing)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            try:
                lib().stride_plan_destroy(h)
            except Exception:
                pass
            self.handle = None

    @property
    def padded_shape(self):
        return stride_plan_padded_shape(self.handle)[: self.ndim]

    def workspace_bytes(self, mode: int, budget_bytes: int = 0) -> int:
        return stride_workspace_bytes(self.handle, mode, budget_bytes)

    def gradient_path(self, ws_bytes: int):
        """(path, forward steps, segments) of a gradient in ws_bytes
        (STRIDE_PATH_*)."""
        return stride_gradient_path(self.grid, self.nrec, ws_bytes)

    def workspace(self, mode: int, budget_bytes: int = 0, device=None):
        import torch
        n = self.workspace_bytes(mode, budget_bytes)
        return torch.empty(n, dtype=torch.uint8, device=device or "cuda")

    # tensor checks ------------------------------------------------------
    def _vp(self, vp):
        import torch
        _dev(vp, self.shape, torch.float32, "vp")

    def _traces_like(self, t, name):
        import torch
        _dev(t, (self.nrec, self.nt), torch.float32, name)

    def _wavelet(self, w):
        import torch
        _dev(w, (self.nsrc, self.nt), torch.float32, "wavelet")

    # solves --------------------------------------------------------------
    def forward(self, vp, wavelet, traces=None, ws=None, stream=None):
        import torch
        self._vp(vp)
        self._wavelet(wavelet)
        if traces is None:
            traces = torch.empty((self.nrec, self.nt), dtype=torch.float32, device=vp.device)
        self._traces_like(traces, "traces")
        if ws is None:
            ws = self.workspace(STRIDE_MODE_FORWARD, device=vp.device)
        stride_plan_forward(self.handle, vp, wavelet, traces, ws, stream)
        return traces

    def forward_medium(self, vp, wavelet, rho=None, alpha0=None, att_power: int = 0, traces=None,
                       ws=None, stream=None):
        """Traces of a forward solve with variable density rho and power-law
        attenuation alpha0 * omega^att_power (att_power 0 or 2); None = constant
        density / no attenuation."""
        import torch
        self._vp(vp)
        self._wavelet(wavelet)
        for a, name in ((rho, "rho"), (alpha0, "alpha0")):
            if a is not None:
                _dev(a, self.shape, torch.float32, name)
        if traces is None:
            traces = torch.empty((self.nrec, self.nt), dtype=torch.float32, device=vp.device)
        self._traces_like(traces, "traces")
        if ws is None:
            ws = self.workspace(STRIDE_MODE_FORWARD_MEDIUM, device=vp.device)
        stride_plan_forward_medium(self.handle, vp, rho, alpha0, att_power, wavelet, traces, ws,
                                   stream)
        return traces

    def gradient_medium(self, vp, wavelet, observed, rho=None, alpha0=None, att_power: int = 0,
                        traces=None, ws=None, budget_bytes: int = 0, stream=None):
        """(misfit, dvp) of the shot gradient in the medium (rho, alpha0 fixed).
        The GRADIENT_MEDIUM workspace keeps every step's imaging factor; a
        smaller one (budget_bytes) checkpoints the forward states and
        recomputes the factors during the adjoint sweep."""
        import torch
        self._vp(vp)
        self._wavelet(wavelet)
        for a, name in ((rho, "rho"), (alpha0, "alpha0")):
            if a is not None:
                _dev(a, self.shape, torch.float32, name)
        self._traces_like(observed, "observed")
        if traces is not None:
            self._traces_like(traces, "traces")
        if ws is None:
            ws = self.workspace(STRIDE_MODE_GRADIENT_MEDIUM, budget_bytes, device=vp.device)
        misfit = torch.zeros(1, dtype=torch.float64, device=vp.device)
        dvp = torch.empty_like(vp)
        stride_plan_gradient_medium(self.handle, vp, rho, alpha0, att_power, wavelet, observed,
                                    traces, misfit, dvp, ws, stream)
        return misfit, dvp

    def gradient(self, vp, wavelet, observed, ws=None, budget_bytes: int = 0, traces=None,
                 stream=None):
        """(misfit [1] float64, dvp) for J = 1/2 sum (traces - observed)^2."""
        import torch
        self._vp(vp)
        self._wavelet(wavelet)
        self._traces_like(observed, "observed")
        if traces is not None:
            self._traces_like(traces, "traces")
        if ws is None:
            ws = self.workspace(STRIDE_MODE_GRADIENT, budget_bytes, device=vp.device)
        misfit = torch.zeros(1, dtype=torch.float64, device=vp.device)
        dvp = torch.empty_like(vp)
        stride_plan_gradient(self.handle, vp, wavelet, observed, traces, misfit, dvp, ws, stream)
        return misfit, dvp

    def forward_save(self, vp, wavelet, ws, traces=None, stream=None):
        import torch
        self._vp(vp)
        self._wavelet(wavelet)
        if traces is None:
            traces = torch.empty((self.nrec, self.nt), dtype=torch.float32, device=vp.device)
        stride_forward_save(self.handle, vp, wavelet, traces, ws, stream)
        return traces

    def backward(self, vp, wavelet, grad_traces, ws, want_dwavelet=False, stream=None):
        import torch
        self._vp(vp)
        self._wavelet(wavelet)
        self._traces_like(grad_traces, "grad_traces")
        dvp = torch.empty_like(vp)
        dwav = torch.empty_like(wavelet) if want_dwavelet else None
        stride_backward(self.handle, vp, wavelet, grad_traces, dvp, dwav, ws, stream)
        return dvp, dwav
