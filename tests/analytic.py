"""Closed-form homogeneous-medium solutions used to pin the oracle (the paper
validates its solver against the analytical solution for a homogeneous medium,
Sec. 3.1).

For (1/c^2) p_tt - lap p = delta(x) w(t):
  3D:  p(r, t) = w(t - r/c) / (4 pi r)
  2D:  p(r, t) = int_0^{t - r/c} w(tau) / (2 pi sqrt((t - tau)^2 - r^2/c^2)) dtau
       and with tau = t - r/c - s^2 this becomes the smooth integral
       (1/pi) int w(t - r/c - s^2) / sqrt(s^2 + 2 r / c) ds.
"""
import numpy as np
from scipy.integrate import quad


def green3d_trace(w, r: float, c: float, t: np.ndarray) -> np.ndarray:
    return w(t - r / c) / (4 * np.pi * r)


def green2d_trace(w, r: float, c: float, t: np.ndarray, support: float) -> np.ndarray:
    """support: w vanishes outside [0, support]."""
    out = np.zeros_like(t, dtype=np.float64)
    t0 = r / c
    for i, ti in enumerate(t):
        if ti <= t0:
            continue
        s_hi = np.sqrt(ti - t0)
        s_lo = np.sqrt(max(0.0, ti - t0 - support))
        val, _ = quad(lambda s: w(ti - t0 - s * s) / np.sqrt(s * s + 2 * t0),
                      s_lo, s_hi, epsabs=1e-14, epsrel=1e-11, limit=200)
        out[i] = val / np.pi
    return out


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
