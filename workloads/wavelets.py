"""Source signal: the three-cycle tone burst the paper fires in every experiment
(Sec. 3.1 validation, Sec. 3.2 breast, Sec. 3.3 head: three cycles centred at
500 kHz).  The window is a Hann window over the three cycles with a sine
carrier starting at t = 0, so the burst starts and ends smoothly and has zero
mean.
"""
import numpy as np


def tone_burst(nt: int, dt: float, f0: float = 500e3, cycles: int = 3,
               nsrc: int = 1, dtype=np.float32) -> np.ndarray:
    """Samples s^n = w(n dt), n = 0..nt-1, repeated for nsrc sources -> [nsrc][nt]."""
    t = np.arange(nt, dtype=np.float64) * dt
    dur = cycles / f0
    w = np.sin(2 * np.pi * f0 * t) * 0.5 * (1.0 - np.cos(2 * np.pi * f0 * t / cycles))
    w[t > dur] = 0.0
    return np.ascontiguousarray(np.tile(w, (nsrc, 1)).astype(dtype))


def tone_burst_fn(f0: float = 500e3, cycles: int = 3):
    """The continuous burst w(t) as a function (for closed-form comparisons)."""
    dur = cycles / f0

    def w(t):
        t = np.asarray(t, dtype=np.float64)
        v = np.sin(2 * np.pi * f0 * t) * 0.5 * (1.0 - np.cos(2 * np.pi * f0 * t / cycles))
        return np.where((t >= 0) & (t <= dur), v, 0.0)

    return w
