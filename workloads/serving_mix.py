"""Seeded request streams for the solve server.

A request is one forward or gradient job of 1-16 shots on its own seeded
phantom and transducer geometry; arrivals follow a seeded Poisson process.
Grid classes follow the mix the server is measured on: 2D {256^2, 512^2,
1024^2} at 0.2 mm (order 8, 20-cell sponge) and 3D {128^3, 192^3, 256^3} at
0.5 mm (order 10, 30-cell sponge).  Each class has one dt (CFL 0.4 at the
class's maximum speed) so that shots of a class can share batched launches.
Observed data of gradient requests are seeded synthetic traces of the right
shape and scale (the server's cost does not depend on their values).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from .geometry import fibonacci_hemisphere, ring
from .phantoms import breast_2d, head_3d
from .wavelets import tone_burst

CLASSES_2D = (256, 512, 1024)
CLASSES_3D = (128, 192, 256)


@dataclass
class RequestSpec:
    rid: int
    kind: str                 # "forward" or "gradient"
    ndim: int
    n: int                    # physical points per axis
    nt: int
    nshots: int
    seed: int
    arrival: float            # seconds after the stream starts
    # filled by materialise()
    shape: tuple = ()
    spacing: float = 0.0
    space_order: int = 8
    nb: int = 20
    vref: float = 1500.0
    dt: float = 0.0
    vp: Optional[np.ndarray] = None
    wavelet: Optional[np.ndarray] = None      # [1][nt]
    src_xyz: Optional[np.ndarray] = None      # [nshots][ndim]
    rec_xyz: Optional[np.ndarray] = None      # [nrec][ndim]
    observed: List[np.ndarray] = field(default_factory=list)   # per shot [nrec][nt]

    @property
    def key(self):
        """Requests with equal keys share an engine (same padded grid)."""
        return (self.ndim, self.n, self.spacing, self.space_order, self.nb)

    def grid_kwargs(self):
        return dict(shape=self.shape, spacing=self.spacing, space_order=self.space_order,
                    nb=self.nb, vref=self.vref, dt=self.dt, nt=self.nt)


def class_params(ndim: int, n: int):
    if ndim == 2:
        dx = 0.2e-3
        return dict(shape=(n, n), spacing=dx, space_order=8, nb=20, vref=1500.0,
                    dt=0.4 * dx / 1700.0)
    dx = 0.5e-3
    return dict(shape=(n, n, n), spacing=dx, space_order=10, nb=30, vref=1500.0,
                dt=0.4 * dx / 3000.0)


def materialise(r: RequestSpec, nrec_2d: int = 128, nrec_3d: int = 256) -> RequestSpec:
    """Phantom, geometry, wavelet and observed data of one request."""
    p = class_params(r.ndim, r.n)
    r.shape, r.spacing, r.space_order = p["shape"], p["spacing"], p["space_order"]
    r.nb, r.vref, r.dt = p["nb"], p["vref"], p["dt"]
    rng = np.random.default_rng(10_000 + r.seed)
    ext = (r.n - 1) * r.spacing
    c = [ext / 2] * r.ndim
    if r.ndim == 2:
        R = 0.42 * ext
        r.vp = breast_2d(r.shape, r.spacing, r.seed, R)
        el = ring(nrec_2d, R, c)
    else:
        R = 0.45 * ext
        r.vp = head_3d(r.shape, r.spacing, r.seed)
        el = fibonacci_hemisphere(nrec_3d, R, c)
    r.rec_xyz = el
    pick = rng.choice(el.shape[0], size=r.nshots, replace=False)
    r.src_xyz = el[np.sort(pick)].copy()
    r.wavelet = tone_burst(r.nt, r.dt)
    if r.kind == "gradient":
        scale = 1e-3 if r.ndim == 2 else 1e-4
        r.observed = [(scale * rng.standard_normal((el.shape[0], r.nt))).astype(np.float32)
                      for _ in range(r.nshots)]
    return r


def request_stream(n_requests: int, seed: int, rate_hz: float, nt_range=(500, 3000),
                   shots_range=(1, 16), classes_2d=CLASSES_2D, classes_3d=CLASSES_3D,
                   frac_gradient: float = 0.3) -> List[RequestSpec]:
    """Seeded Poisson stream: grid class uniform over the classes given, nt
    uniform in nt_range, shots uniform in shots_range, 70/30 forward/gradient."""
    rng = np.random.default_rng(seed)
    classes = [(2, n) for n in classes_2d] + [(3, n) for n in classes_3d]
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate_hz)
        nd, n = classes[int(rng.integers(len(classes)))]
        out.append(RequestSpec(
            rid=i,
            kind="gradient" if rng.uniform() < frac_gradient else "forward",
            ndim=nd, n=n,
            nt=int(rng.integers(nt_range[0], nt_range[1] + 1)),
            nshots=int(rng.integers(shots_range[0], shots_range[1] + 1)),
            seed=int(rng.integers(1 << 30)),
            arrival=t))
    return out
