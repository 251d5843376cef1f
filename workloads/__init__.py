"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package holds input generators only (phantoms, transducer geometries, the
source signal and the named workload shapes).  It contains none of the solver's
arithmetic, and it imports neither the HIP product package nor the oracle.
"""
from .wavelets import tone_burst
from .geometry import ring, fibonacci_hemisphere, grid_node_ring_2d
from .phantoms import homogeneous, breast_2d, head_3d, head_3d_skull_only, medium
from .configs import Workload, config1, config2, config3, config4, tiny_2d, tiny_3d, CONFIG_NAMES, RingSurvey, ring_survey_2d

__all__ = [
    "tone_burst", "ring", "fibonacci_hemisphere", "grid_node_ring_2d",
    "homogeneous", "breast_2d", "head_3d", "head_3d_skull_only",
    "Workload", "config1", "config2", "config3", "config4", "tiny_2d", "tiny_3d",
    "CONFIG_NAMES",
]
