"""Transducer geometries (metres, origin at physical grid node 0, axis order of
the arrays).  Rings stand in for the 2D breast setup (Sec. 3.2: point
transducers around the model, all acting as sources and receivers); a
Fibonacci-spiral hemisphere stands in for the 3D head setup (Sec. 3.3, 1024
transducers; Sec. 3.1 distributes points by Fibonacci spirals).
"""
import numpy as np


def ring(n: int, radius: float, centre) -> np.ndarray:
    """n points at angles 2 pi j / n on a circle in the (axis0, axis1) plane."""
    th = 2 * np.pi * np.arange(n) / n
    c = np.asarray(centre, dtype=np.float64)
    return np.stack([c[0] + radius * np.cos(th), c[1] + radius * np.sin(th)], axis=1)


def grid_node_ring_2d(centre_node, radius_cells: int, dx: float) -> np.ndarray:
    """The 12 grid nodes at exactly radius_cells from centre_node when
    radius_cells is a multiple of 5 (3-4-5 triangle): (+-r,0), (0,+-r),
    (+-3r/5, +-4r/5), (+-4r/5, +-3r/5)."""
    r = radius_cells
    assert r % 5 == 0
    a, b = 3 * r // 5, 4 * r // 5
    offs = [(r, 0), (-r, 0), (0, r), (0, -r)]
    for s0 in (1, -1):
        for s1 in (1, -1):
            offs.append((s0 * a, s1 * b))
            offs.append((s0 * b, s1 * a))
    c = np.asarray(centre_node)
    return np.array([((c[0] + o0) * dx, (c[1] + o1) * dx) for o0, o1 in offs], dtype=np.float64)


def fibonacci_hemisphere(n: int, radius: float, centre) -> np.ndarray:
    """n points on the hemisphere axis0 >= centre[0], spread by the golden angle."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (i + 0.5) / n            # from the pole to the equator
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * np.pi * (3.0 - np.sqrt(5.0))
    c = np.asarray(centre, dtype=np.float64)
    return np.stack([c[0] + radius * z,
                     c[1] + radius * rho * np.cos(phi),
                     c[2] + radius * rho * np.sin(phi)], axis=1)
