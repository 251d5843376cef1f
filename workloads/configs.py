"""Named workloads: the shapes, sizes and value ranges of the paper's
experiments at the sizes this implementation is measured on.

  config1  2D homogeneous forward, 200^2 at 0.2 mm, 8th order, 20-cell sponge,
           CFL 0.4, 500 steps, source at the centre node, 128 receivers on a
           15 mm ring (Sec. 3.1 validation setup: 500 kHz three-cycle burst,
           1500 m/s, homogeneous medium).
  config2  2D breast-like forward, one shot, 1024^2 at 0.2 mm, 40-cell sponge,
           2500 steps, 256-element ring of R = 90 mm (Sec. 3.2 breast setup:
           a ring of point transducers that all fire and record).
  config3  2D gradient, 512^2 at 0.2 mm, 40-cell sponge, 1500 steps, 256-element
           ring of R = 45 mm, 64 shots (elements 0, 4, ..., 252), true phantom for
           the observed data, 1500 m/s starting model (Sec. 3.2).
  config4  3D head-like forward + gradient, 256^3 at 0.5 mm, 10th order,
           30-cell sponge, 3000 steps, 1024 receivers on a Fibonacci hemisphere
           of R = 58 mm, source = element 0, skull-only starting model
           (Sec. 3.3).
In every config dt = 0.4 dx / max(vp) (3000 m/s in 3D) and the sponge
reference speed is the 1500 m/s background.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass
from typing import Optional

import numpy as np

from .geometry import fibonacci_hemisphere, ring
from .phantoms import breast_2d, head_3d, head_3d_skull_only, homogeneous
from .wavelets import tone_burst

CONFIG_NAMES = ("config1", "config2", "config3", "config4")


@dataclass
class Workload:
    name: str
    shape: tuple
    spacing: float
    space_order: int
    nb: int
    vref: float
    dt: float
    nt: int
    vp: np.ndarray              # model the forward runs on (float32)
    wavelet: np.ndarray         # [nsrc][nt] float32
    src_xyz: np.ndarray         # [nsrc][ndim] float64, metres
    rec_xyz: np.ndarray         # [nrec][ndim] float64, metres
    vp_true: Optional[np.ndarray] = None    # gradient configs: model of the observed data
    vp_start: Optional[np.ndarray] = None   # gradient configs: model the gradient is taken at
    shot_src_xyz: Optional[np.ndarray] = None  # [nshot][ndim] multi-shot configs

    @property
    def ndim(self):
        return len(self.shape)

    @property
    def padded_shape(self):
        return tuple(s + 2 * self.nb for s in self.shape)

    @property
    def padded_points(self):
        return int(np.prod(self.padded_shape))

    def grid_kwargs(self):
        return dict(shape=self.shape, spacing=self.spacing, space_order=self.space_order,
                    nb=self.nb, vref=self.vref, dt=self.dt, nt=self.nt)

    def with_nt(self, nt: int) -> "Workload":
        """Same workload truncated (or extended) to nt time samples."""
        wav = tone_burst(nt, self.dt, nsrc=self.wavelet.shape[0])
        return dataclasses.replace(self, nt=nt, wavelet=wav)

    def shot(self, i: int) -> "Workload":
        """Single-shot view firing shot i of a multi-shot workload."""
        assert self.shot_src_xyz is not None
        return dataclasses.replace(self, src_xyz=self.shot_src_xyz[i:i + 1].copy(),
                                   wavelet=tone_burst(self.nt, self.dt, nsrc=1))


def _dt(cfl, dx, vmax):
    return cfl * dx / vmax


def config1(cfl: float = 0.4, nt: int = 500) -> Workload:
    n, dx = 200, 0.2e-3
    vp = homogeneous((n, n), 1500.0)
    dt = _dt(cfl, dx, 1500.0)
    src = np.array([[100 * dx, 100 * dx]])
    rec = ring(128, 15e-3, src[0])
    return Workload("config1", (n, n), dx, 8, 20, 1500.0, dt, nt, vp,
                    tone_burst(nt, dt), src, rec)


def config2(nt: int = 2500, seed: int = 1) -> Workload:
    n, dx, R = 1024, 0.2e-3, 90e-3
    vp = breast_2d((n, n), dx, seed, R)
    dt = _dt(0.4, dx, float(vp.max()))
    c = ((n - 1) * dx / 2, (n - 1) * dx / 2)
    el = ring(256, R, c)
    return Workload("config2", (n, n), dx, 8, 40, 1500.0, dt, nt, vp,
                    tone_burst(nt, dt), el[0:1].copy(), el)


def config3(nt: int = 1500, seed: int = 2, nshots: int = 64) -> Workload:
    n, dx, R = 512, 0.2e-3, 45e-3
    vp_true = breast_2d((n, n), dx, seed, R)
    vp0 = homogeneous((n, n), 1500.0)
    dt = _dt(0.4, dx, float(vp_true.max()))
    c = ((n - 1) * dx / 2, (n - 1) * dx / 2)
    el = ring(256, R, c)
    shots = el[0:4 * nshots:4].copy()
    return Workload("config3", (n, n), dx, 8, 40, 1500.0, dt, nt, vp0,
                    tone_burst(nt, dt), shots[0:1].copy(), el,
                    vp_true=vp_true, vp_start=vp0, shot_src_xyz=shots)


def config4(nt: int = 3000, seed: int = 4, n: int = 256) -> Workload:
    dx, R = 0.5e-3, 58e-3
    shape = (n, n, n)
    vp_true = head_3d(shape, dx, seed)
    vp0 = head_3d_skull_only(shape, dx, seed)
    dt = _dt(0.4, dx, 3000.0)
    c = [(s - 1) * dx / 2 for s in shape]
    el = fibonacci_hemisphere(1024, R * n / 256, c)
    return Workload("config4", shape, dx, 10, 30, 1500.0, dt, nt, vp_true,
                    tone_burst(nt, dt), el[0:1].copy(), el,
                    vp_true=vp_true, vp_start=vp0)


def _smooth_random(shape, seed, amp):
    from scipy.ndimage import gaussian_filter
    rng = np.random.default_rng(seed)
    f = gaussian_filter(rng.standard_normal(shape), sigma=max(1.0, min(shape) / 8))
    f /= np.max(np.abs(f))
    return f * amp


def tiny_2d(n=(48, 56), nt: int = 120, space_order: int = 8, nb: int = 8, seed: int = 0,
            nsrc: int = 2, nrec: int = 7, vref: float = 1500.0, cfl: float = 0.4,
            dx: float = 0.2e-3) -> Workload:
    """Small heterogeneous 2D case with off-grid sources and receivers."""
    rng = np.random.default_rng(1000 + seed)
    vp = (1500.0 * (1.0 + _smooth_random(n, seed, 0.1))).astype(np.float32)
    dt = _dt(cfl, dx, float(vp.max()))
    ext = [(s - 1) * dx for s in n]
    src = np.stack([rng.uniform(0.2, 0.8, nsrc) * e for e in ext], axis=1)
    rec = np.stack([rng.uniform(0.05, 0.95, nrec) * e for e in ext], axis=1)
    # a short burst so that the signal fills the short time window
    wav = tone_burst(nt, dt, f0=1.5e6, nsrc=nsrc)
    wav *= rng.uniform(0.5, 1.5, size=(nsrc, 1)).astype(np.float32)
    return Workload("tiny_2d", tuple(n), dx, space_order, nb, vref, dt, nt, vp, wav, src, rec)


def tiny_3d(n=(20, 22, 24), nt: int = 60, space_order: int = 10, nb: int = 5, seed: int = 0,
            nsrc: int = 2, nrec: int = 9, vref: float = 1500.0, cfl: float = 0.35,
            dx: float = 0.5e-3) -> Workload:
    """Small heterogeneous 3D case with off-grid sources and receivers."""
    rng = np.random.default_rng(2000 + seed)
    vp = (1500.0 * (1.0 + _smooth_random(n, seed, 0.1))).astype(np.float32)
    dt = _dt(cfl, dx, float(vp.max()))
    ext = [(s - 1) * dx for s in n]
    src = np.stack([rng.uniform(0.3, 0.7, nsrc) * e for e in ext], axis=1)
    rec = np.stack([rng.uniform(0.05, 0.95, nrec) * e for e in ext], axis=1)
    wav = tone_burst(nt, dt, f0=0.6e6, nsrc=nsrc)
    wav *= rng.uniform(0.5, 1.5, size=(nsrc, 1)).astype(np.float32)
    return Workload("tiny_3d", tuple(n), dx, space_order, nb, vref, dt, nt, vp, wav, src, rec)


@dataclass
class RingSurvey:
    """A 2D ring survey for inversion runs: every transducer fires once and
    all record (Sec. 3.2 imaging setup, at a reduced size)."""
    shape: tuple
    spacing: float
    space_order: int
    nb: int
    vref: float
    dt: float
    nt: int
    vp_true: np.ndarray
    vp_start: np.ndarray
    positions: np.ndarray      # [n][2] transducers (sources and receivers)
    wavelet: np.ndarray        # [nt]
    roi: np.ndarray            # bool, the region inside the ring the inversion updates

    def grid_kwargs(self):
        return dict(shape=self.shape, spacing=self.spacing, space_order=self.space_order,
                    nb=self.nb, vref=self.vref, dt=self.dt, nt=self.nt)


def ring_survey_2d(n: int = 100, dx: float = 0.5e-3, ntrans: int = 16, seed: int = 0) -> RingSurvey:
    """n x n grid at dx; water 1500 m/s with a 1560 m/s disc (radius 8 mm)
    and a 1460 m/s disc (4 mm) whose centres are jittered by the seed;
    ntrans transducers on a ring of radius 0.44 n dx; 500 kHz 3-cycle burst;
    dt at CFL 0.3 of the fastest speed; records long enough to cross the ring
    and back out; the region of interest is the disc 4 mm inside the ring."""
    rng = np.random.default_rng(seed)
    X = np.meshgrid(np.arange(n) * dx, np.arange(n) * dx, indexing="ij")
    cen = (n - 1) * dx / 2
    vp = np.full((n, n), 1500.0)
    j = rng.uniform(-1e-3, 1e-3, size=4)
    vp[(X[0] - cen - 4e-3 - j[0]) ** 2 + (X[1] - cen + 2e-3 - j[1]) ** 2 < (8e-3) ** 2] = 1560.0
    vp[(X[0] - cen + 7e-3 - j[2]) ** 2 + (X[1] - cen - 6e-3 - j[3]) ** 2 < (4e-3) ** 2] = 1460.0
    R = 0.44 * n * dx
    ang = np.arange(ntrans) * 2 * np.pi / ntrans
    pos = np.stack([cen + R * np.cos(ang), cen + R * np.sin(ang)], axis=1)
    dt = 0.3 * dx / 1560.0
    nt = int((2 * R * 0.95 / 1500.0 + 8e-6) / dt)
    roi = (X[0] - cen) ** 2 + (X[1] - cen) ** 2 < (R - 4e-3) ** 2
    return RingSurvey((n, n), dx, 8, 16, 1500.0, dt, nt, vp.astype(np.float32),
                      np.full((n, n), 1500.0, dtype=np.float32), pos,
                      tone_burst(nt, dt, nsrc=1)[0], roi)
