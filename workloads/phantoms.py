"""Seeded speed-of-sound phantoms (m/s, float32, C order).

They stand in for the paper's breast slice (Sec. 3.2, from an open breast
database) and MIDA-based head model (Sec. 3.3), neither of which is available:
only shapes and value ranges are taken, and every draw comes from
numpy.random.default_rng(seed).
"""
import numpy as np
from scipy.ndimage import gaussian_filter


def homogeneous(shape, vp: float = 1500.0) -> np.ndarray:
    return np.full(tuple(shape), vp, dtype=np.float32)


def breast_2d(shape, dx: float, seed: int, ring_radius: float,
              background: float = 1500.0, noise_sigma: float = 2e-3) -> np.ndarray:
    """Background 1500 m/s; 5-20 ellipses (centres within 0.6 R of the grid
    centre, semi-axes U(0.02, 0.28) R, random angle, vp U(1400, 1600)) painted in
    draw order; then x (1 + 0.01 n) with n Gaussian-smoothed (sigma 2 mm) white
    noise scaled to max |n| = 1."""
    rng = np.random.default_rng(seed)
    n0, n1 = shape
    vp = np.full((n0, n1), background, dtype=np.float64)
    c0, c1 = (n0 - 1) * dx / 2, (n1 - 1) * dx / 2
    x0 = np.arange(n0)[:, None] * dx - c0
    x1 = np.arange(n1)[None, :] * dx - c1
    R = ring_radius
    k = int(rng.integers(5, 21))
    for _ in range(k):
        rad = 0.6 * R * np.sqrt(rng.uniform())
        ang = rng.uniform(0, 2 * np.pi)
        e0, e1 = rad * np.cos(ang), rad * np.sin(ang)
        a = rng.uniform(0.02, 0.28) * R
        b = rng.uniform(0.02, 0.28) * R
        th = rng.uniform(0, np.pi)
        v = rng.uniform(1400.0, 1600.0)
        d0, d1 = x0 - e0, x1 - e1
        p = d0 * np.cos(th) + d1 * np.sin(th)
        q = -d0 * np.sin(th) + d1 * np.cos(th)
        vp[(p / a) ** 2 + (q / b) ** 2 <= 1.0] = v
    noise = gaussian_filter(rng.standard_normal((n0, n1)), sigma=noise_sigma / dx)
    noise /= np.max(np.abs(noise))
    vp *= 1.0 + 0.01 * noise
    return vp.astype(np.float32)


def _head_parts(shape, dx: float, seed: int):
    rng = np.random.default_rng(seed)
    n = shape
    cen = [(s - 1) * dx / 2 for s in n]
    axes = [np.arange(s) * dx - c for s, c in zip(n, cen)]
    X0 = axes[0][:, None, None]
    X1 = axes[1][None, :, None]
    X2 = axes[2][None, None, :]
    outer = np.array([38e-3, 46e-3, 49e-3]) * rng.uniform(0.95, 1.05, size=3)
    thick = rng.uniform(5e-3, 8e-3)
    inner = outer - thick
    v_skull = rng.uniform(2800.0, 3000.0)
    v_tissue = rng.uniform(1500.0, 1560.0)
    r_out = (X0 / outer[0]) ** 2 + (X1 / outer[1]) ** 2 + (X2 / outer[2]) ** 2
    r_in = (X0 / inner[0]) ** 2 + (X1 / inner[1]) ** 2 + (X2 / inner[2]) ** 2
    shell = (r_out <= 1.0) & (r_in > 1.0)
    brain = r_in <= 1.0
    incl = []
    for _ in range(int(rng.integers(3, 11))):
        c = rng.uniform(-0.5, 0.5, size=3) * inner
        ax = rng.uniform(0.05, 0.25, size=3) * inner
        v = rng.uniform(1500.0, 1560.0)
        incl.append((c, ax, v))
    return (X0, X1, X2), shell, brain, v_skull, v_tissue, incl


def head_3d(shape, dx: float, seed: int, background: float = 1500.0) -> np.ndarray:
    """Water 1500 m/s; ellipsoidal skull shell (outer semi-axes about
    (38, 46, 49) mm, thickness U(5, 8) mm, vp U(2800, 3000)) around tissue vp
    U(1500, 1560) with 3-10 inclusion ellipsoids of vp U(1500, 1560)."""
    (X0, X1, X2), shell, brain, v_skull, v_tissue, incl = _head_parts(shape, dx, seed)
    vp = np.full(tuple(shape), background, dtype=np.float32)
    vp[brain] = v_tissue
    for c, ax, v in incl:
        m = ((X0 - c[0]) / ax[0]) ** 2 + ((X1 - c[1]) / ax[1]) ** 2 + ((X2 - c[2]) / ax[2]) ** 2 <= 1.0
        vp[m & brain] = v
    vp[shell] = v_skull
    return vp


def head_3d_skull_only(shape, dx: float, seed: int, background: float = 1500.0) -> np.ndarray:
    """Starting model of the 3D inversion (Sec. 3.3 starts from the skull alone):
    the same skull shell in water."""
    _, shell, _, v_skull, _, _ = _head_parts(shape, dx, seed)
    vp = np.full(tuple(shape), background, dtype=np.float32)
    vp[shell] = v_skull
    return vp


def medium(vp: np.ndarray, dx: float, seed: int, att_power: int = 0, f0: float = 500e3,
           alpha_bone: float = 40.0):
    """Density (kg/m^3) and attenuation alpha0 for a speed model, float32.

    rho: 1000 where vp is within 1 m/s of 1500 (water), 1000 + 0.5 (vp - 1500)
    clipped to [950, 1100] for soft tissue (vp below 2500 m/s), 1900 for bone
    (vp >= 2500); then x (1 + 0.02 n), n Gaussian-smoothed (sigma 1 mm) white
    noise scaled to max |n| = 1.  Attenuation at f0: 0.5 Np/m water, 4 Np/m
    soft tissue, alpha_bone (default 40 Np/m) bone; alpha0 = alpha(f0) / (2 pi f0)^att_power, so
    that alpha0 omega^y is alpha(f0) at f0.  Only the value ranges follow
    tissue; the draws come from numpy.random.default_rng(seed)."""
    rng = np.random.default_rng(seed)
    vp = np.asarray(vp, dtype=np.float64)
    water = np.abs(vp - 1500.0) < 1.0
    bone = vp >= 2500.0
    rho = np.clip(1000.0 + 0.5 * (vp - 1500.0), 950.0, 1100.0)
    rho[water] = 1000.0
    rho[bone] = 1900.0
    noise = gaussian_filter(rng.standard_normal(vp.shape), sigma=1e-3 / dx)
    noise /= np.max(np.abs(noise))
    rho *= 1.0 + 0.02 * noise
    alpha = np.full(vp.shape, 4.0)
    alpha[water] = 0.5
    alpha[bone] = alpha_bone
    alpha0 = alpha / (2.0 * np.pi * f0) ** att_power
    return rho.astype(np.float32), alpha0.astype(np.float32)
