"""Plain FP64 CPU oracle for the acoustic FWI hot path (ctypes wrapper).

TEST INFRASTRUCTURE ONLY.  The product package never imports this module; only
the tests, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` do.  It shares no code with the HIP path.

The arithmetic lives in ``stride_oracle.c``; see its header for the scheme and
the readings of the paper (Sec. 2.2 adjoint-state gradient, Sec. 2.4 acoustic
equation, sponge and linear-interpolation taps).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np

from . import build as _build

_LIB = None


class _CGrid(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("shape", ctypes.c_long * 3),
        ("spacing", ctypes.c_double * 3),
        ("space_order", ctypes.c_int),
        ("nb", ctypes.c_int),
        ("vref", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("nt", ctypes.c_int),
        ("time_order", ctypes.c_int),
        ("interp", ctypes.c_int),
    ]


@dataclass
class Grid:
    """Physical grid, stencil order, sponge and time axis of one solve."""
    shape: Sequence[int]
    spacing: float | Sequence[float]
    space_order: int
    nb: int
    vref: float
    dt: float
    nt: int
    time_order: int = 2      # 4: leapfrog with the modified-equation correction
    interp: int = 0          # off-grid points: 0 linear, 1 Kaiser-windowed sinc
    ndim: int = field(init=False)

    def __post_init__(self):
        self.shape = tuple(int(s) for s in self.shape)
        self.ndim = len(self.shape)
        if np.isscalar(self.spacing):
            self.spacing = (float(self.spacing),) * self.ndim
        self.spacing = tuple(float(s) for s in self.spacing)

    def c(self) -> _CGrid:
        g = _CGrid()
        g.ndim = self.ndim
        for a in range(3):
            g.shape[a] = self.shape[a] if a < self.ndim else 1
            g.spacing[a] = self.spacing[a] if a < self.ndim else 1.0
        g.space_order = self.space_order
        g.nb = self.nb
        g.vref = self.vref
        g.dt = self.dt
        g.nt = self.nt
        g.time_order = self.time_order
        g.interp = self.interp
        return g

    @property
    def padded_shape(self):
        return tuple(s + 2 * self.nb for s in self.shape)


class OracleError(RuntimeError):
    pass


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        lp = ctypes.POINTER(ctypes.c_long)
        ip = ctypes.POINTER(ctypes.c_int)
        gp = ctypes.POINTER(_CGrid)
        L.oracle_fd_weights.argtypes = [ctypes.c_int, dp]
        L.oracle_padded_points.argtypes = [gp, lp]
        L.oracle_padded_points.restype = ctypes.c_long
        L.oracle_pad.argtypes = [gp, dp, dp]
        L.oracle_pad_transpose.argtypes = [gp, dp, dp]
        L.oracle_eta.argtypes = [gp, dp]
        L.oracle_taps.argtypes = [gp, ctypes.c_int, dp, lp, dp]
        L.oracle_laplacian.argtypes = [gp, dp, dp]
        L.oracle_forward.argtypes = [gp, dp, ctypes.c_int, dp, dp, ctypes.c_int, dp, dp,
                                     ctypes.c_int, ip, dp]
        L.oracle_adjoint.argtypes = [gp, dp, ctypes.c_int, dp, dp, ctypes.c_int, dp, dp,
                                     dp, dp, ctypes.c_int]
        L.oracle_gradient.argtypes = [gp, dp, ctypes.c_int, dp, dp, ctypes.c_int, dp, dp,
                                      dp, dp, dp, ctypes.c_int]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        L.oracle_fd1_weights.argtypes = [ctypes.c_int, dp]
        L.oracle_taps_per_point.argtypes = [gp]
        L.oracle_lowpass.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                     ctypes.c_double]
        L.oracle_taps_per_point.restype = ctypes.c_int
        L.oracle_medium_operator.argtypes = [gp, dp, dp, dp]
        L.oracle_forward_medium.argtypes = [gp, dp, dp, dp, ctypes.c_int, ctypes.c_int, dp, dp,
                                            ctypes.c_int, dp, dp]
        L.oracle_forward_pml.argtypes = [gp, dp, ctypes.c_int, dp, dp, ctypes.c_int, dp, dp]
        L.oracle_adjoint_medium.argtypes = [gp, dp, dp, dp, ctypes.c_int, ctypes.c_int, dp, dp,
                                            ctypes.c_int, dp, dp, dp, dp, ctypes.c_int]
        L.oracle_gradient_medium.argtypes = [gp, dp, dp, dp, ctypes.c_int, ctypes.c_int, dp, dp,
                                             ctypes.c_int, dp, dp, dp, dp, dp, ctypes.c_int]
        _LIB = L
    return _LIB


def _d(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a, shape=None) -> np.ndarray:
    out = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        out = out.reshape(shape)
    return out


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(f"{what} failed with code {rc}")


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the following oracle calls (timing only; results do not depend on it)."""
    lib().oracle_set_num_threads(int(n))


def fd_weights(space_order: int) -> np.ndarray:
    c = np.zeros(6)
    _check(lib().oracle_fd_weights(space_order, _d(c)), "fd_weights")
    return c[: space_order // 2 + 1].copy()


def pad(grid: Grid, phys) -> np.ndarray:
    phys = _f64(phys, grid.shape)
    out = np.zeros(grid.padded_shape)
    g = grid.c()
    _check(lib().oracle_pad(ctypes.byref(g), _d(phys), _d(out)), "pad")
    return out


def pad_transpose(grid: Grid, padded) -> np.ndarray:
    padded = _f64(padded, grid.padded_shape)
    out = np.zeros(grid.shape)
    g = grid.c()
    _check(lib().oracle_pad_transpose(ctypes.byref(g), _d(padded), _d(out)), "pad_transpose")
    return out


def eta(grid: Grid) -> np.ndarray:
    out = np.zeros(grid.padded_shape)
    g = grid.c()
    _check(lib().oracle_eta(ctypes.byref(g), _d(out)), "eta")
    return out


def taps(grid: Grid, xyz):
    """(idx, w): [npts][taps per point] flat padded indices and weights."""
    xyz = _f64(xyz).reshape(-1, grid.ndim)
    n = xyz.shape[0]
    g0 = grid.c()
    T = lib().oracle_taps_per_point(ctypes.byref(g0))
    _check(min(T, 0), "taps")
    idx = np.zeros((n, T), dtype=np.int64)
    w = np.zeros((n, T))
    g = grid.c()
    _check(lib().oracle_taps(ctypes.byref(g), n, _d(xyz),
                             idx.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _d(w)), "taps")
    return idx, w


def laplacian(grid: Grid, u) -> np.ndarray:
    u = _f64(u, grid.padded_shape)
    out = np.zeros(grid.padded_shape)
    g = grid.c()
    _check(lib().oracle_laplacian(ctypes.byref(g), _d(u), _d(out)), "laplacian")
    return out


def forward(grid: Grid, vp, src_xyz, wavelet, rec_xyz, snap_steps: Sequence[int] = ()):
    """Receiver traces [nrec][nt]; with snap_steps also u^n at those steps."""
    vp = _f64(vp, grid.shape)
    src = _f64(src_xyz).reshape(-1, grid.ndim)
    rec = _f64(rec_xyz).reshape(-1, grid.ndim)
    wav = _f64(wavelet).reshape(src.shape[0], grid.nt)
    traces = np.zeros((rec.shape[0], grid.nt))
    snaps = None
    steps = np.ascontiguousarray(np.asarray(snap_steps, dtype=np.int32))
    if len(steps):
        snaps = np.zeros((len(steps),) + grid.padded_shape)
    g = grid.c()
    rc = lib().oracle_forward(ctypes.byref(g), _d(vp), src.shape[0], _d(src), _d(wav),
                              rec.shape[0], _d(rec), _d(traces), len(steps),
                              steps.ctypes.data_as(ctypes.POINTER(ctypes.c_int)) if len(steps) else None,
                              _d(snaps))
    _check(rc, "forward")
    return (traces, snaps) if len(steps) else traces


def adjoint(grid: Grid, vp, src_xyz, wavelet, rec_xyz, grad_traces, seg: int = 0):
    """(dvp, dwavelet): the transpose of the forward Jacobian applied to grad_traces."""
    vp = _f64(vp, grid.shape)
    src = _f64(src_xyz).reshape(-1, grid.ndim)
    rec = _f64(rec_xyz).reshape(-1, grid.ndim)
    wav = _f64(wavelet).reshape(src.shape[0], grid.nt)
    gtr = _f64(grad_traces).reshape(rec.shape[0], grid.nt)
    dvp = np.zeros(grid.shape)
    dwav = np.zeros((src.shape[0], grid.nt))
    g = grid.c()
    rc = lib().oracle_adjoint(ctypes.byref(g), _d(vp), src.shape[0], _d(src), _d(wav),
                              rec.shape[0], _d(rec), _d(gtr), _d(dvp), _d(dwav), seg)
    _check(rc, "adjoint")
    return dvp, dwav


def gradient(grid: Grid, vp, src_xyz, wavelet, rec_xyz, observed, seg: int = 0):
    """(traces, misfit, dvp) for J = 1/2 sum (traces - observed)^2."""
    vp = _f64(vp, grid.shape)
    src = _f64(src_xyz).reshape(-1, grid.ndim)
    rec = _f64(rec_xyz).reshape(-1, grid.ndim)
    wav = _f64(wavelet).reshape(src.shape[0], grid.nt)
    obs = _f64(observed).reshape(rec.shape[0], grid.nt)
    traces = np.zeros((rec.shape[0], grid.nt))
    dvp = np.zeros(grid.shape)
    J = ctypes.c_double(0.0)
    g = grid.c()
    rc = lib().oracle_gradient(ctypes.byref(g), _d(vp), src.shape[0], _d(src), _d(wav),
                               rec.shape[0], _d(rec), _d(obs), _d(traces), ctypes.byref(J),
                               _d(dvp), seg)
    _check(rc, "gradient")
    return traces, float(J.value), dvp


def fd1_weights(space_order: int) -> np.ndarray:
    """[0, d_1 .. d_r]: centred first-derivative weights."""
    d = np.zeros(6)
    _check(lib().oracle_fd1_weights(space_order, _d(d)), "fd1_weights")
    return d[: space_order // 2 + 1].copy()


def medium_operator(grid: Grid, rho, u) -> np.ndarray:
    """L u + sum_a gamma_a D_a u on the padded grid (rho physical, None = 1)."""
    rho = None if rho is None else _f64(rho, grid.shape)
    u = _f64(u, grid.padded_shape)
    out = np.zeros(grid.padded_shape)
    g = grid.c()
    _check(lib().oracle_medium_operator(ctypes.byref(g), _d(rho), _d(u), _d(out)), "medium_operator")
    return out


def forward_medium(grid: Grid, vp, src_xyz, wavelet, rec_xyz, rho=None, alpha0=None,
                   att_power: int = 0):
    """Receiver traces [nrec][nt] in a medium with variable density (rho) and
    power-law attenuation alpha0 * omega^att_power, att_power 0 or 2."""
    vp = _f64(vp, grid.shape)
    rho = None if rho is None else _f64(rho, grid.shape)
    alpha0 = None if alpha0 is None else _f64(alpha0, grid.shape)
    src = _f64(src_xyz).reshape(-1, grid.ndim)
    rec = _f64(rec_xyz).reshape(-1, grid.ndim)
    wav = _f64(wavelet).reshape(src.shape[0], grid.nt)
    traces = np.zeros((rec.shape[0], grid.nt))
    g = grid.c()
    rc = lib().oracle_forward_medium(ctypes.byref(g), _d(vp), _d(rho), _d(alpha0), int(att_power),
                                     src.shape[0], _d(src), _d(wav), rec.shape[0], _d(rec),
                                     _d(traces))
    _check(rc, "forward_medium")
    return traces


def adjoint_medium(grid: Grid, vp, src_xyz, wavelet, rec_xyz, grad_traces, rho=None, alpha0=None,
                   att_power: int = 0, seg: int = 0):
    """(dvp, dwavelet): transpose of the medium forward's Jacobian applied to grad_traces."""
    vp = _f64(vp, grid.shape)
    rho = None if rho is None else _f64(rho, grid.shape)
    alpha0 = None if alpha0 is None else _f64(alpha0, grid.shape)
    src = _f64(src_xyz).reshape(-1, grid.ndim)
    rec = _f64(rec_xyz).reshape(-1, grid.ndim)
    wav = _f64(wavelet).reshape(src.shape[0], grid.nt)
    gtr = _f64(grad_traces).reshape(rec.shape[0], grid.nt)
    dvp = np.zeros(grid.shape)
    dwav = np.zeros((src.shape[0], grid.nt))
    g = grid.c()
    rc = lib().oracle_adjoint_medium(ctypes.byref(g), _d(vp), _d(rho), _d(alpha0), int(att_power),
                                     src.shape[0], _d(src), _d(wav), rec.shape[0], _d(rec), _d(gtr),
                                     _d(dvp), _d(dwav), seg)
    _check(rc, "adjoint_medium")
    return dvp, dwav


def gradient_medium(grid: Grid, vp, src_xyz, wavelet, rec_xyz, observed, rho=None, alpha0=None,
                    att_power: int = 0, seg: int = 0):
    """(traces, misfit, dvp) of J = 1/2 sum (traces - observed)^2 in the medium."""
    vp = _f64(vp, grid.shape)
    rho = None if rho is None else _f64(rho, grid.shape)
    alpha0 = None if alpha0 is None else _f64(alpha0, grid.shape)
    src = _f64(src_xyz).reshape(-1, grid.ndim)
    rec = _f64(rec_xyz).reshape(-1, grid.ndim)
    wav = _f64(wavelet).reshape(src.shape[0], grid.nt)
    obs = _f64(observed).reshape(rec.shape[0], grid.nt)
    traces = np.zeros((rec.shape[0], grid.nt))
    dvp = np.zeros(grid.shape)
    J = ctypes.c_double(0.0)
    g = grid.c()
    rc = lib().oracle_gradient_medium(ctypes.byref(g), _d(vp), _d(rho), _d(alpha0), int(att_power),
                                      src.shape[0], _d(src), _d(wav), rec.shape[0], _d(rec), _d(obs),
                                      _d(traces), ctypes.byref(J), _d(dvp), seg)
    _check(rc, "gradient_medium")
    return traces, float(J.value), dvp


def forward_pml(grid: Grid, vp, src_xyz, wavelet, rec_xyz):
    """Receiver traces [nrec][nt] with a perfectly matched layer in the
    grid's nb padded cells instead of the sponge (zeta from grid.vref)."""
    vp = _f64(vp, grid.shape)
    src = _f64(src_xyz).reshape(-1, grid.ndim)
    rec = _f64(rec_xyz).reshape(-1, grid.ndim)
    wav = _f64(wavelet).reshape(src.shape[0], grid.nt)
    traces = np.zeros((rec.shape[0], grid.nt))
    g = grid.c()
    rc = lib().oracle_forward_pml(ctypes.byref(g), _d(vp), src.shape[0], _d(src), _d(wav),
                                  rec.shape[0], _d(rec), _d(traces))
    _check(rc, "forward_pml")
    return traces


def lowpass(signals, dt: float, f_max: float) -> np.ndarray:
    """Zero-phase Hann-windowed-sinc low-pass of [count][nt] signals."""
    x = np.ascontiguousarray(np.asarray(signals, dtype=np.float64))
    shape = x.shape
    x = x.reshape(-1, shape[-1])
    out = np.zeros_like(x)
    rc = lib().oracle_lowpass(_d(x), _d(out), x.shape[0], x.shape[1], float(dt), float(f_max))
    _check(min(rc, 0), "lowpass")
    return out.reshape(shape)
