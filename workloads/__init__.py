"""Seeded synthetic inputs for the cubed-sphere N-body sums.

This package only makes inputs: point sets on the unit sphere, cell areas,
spherical-harmonic fields and seeded random numbers. It holds none of the
method's arithmetic (no tree, no interpolation, no kernel), so both the
GPU library's tests and the CPU oracle can take their inputs from here.
"""

from .grid import cubed_sphere_grid, random_sphere_points
from .meshes import icosahedral_grid, latlon_grid
from .flows import rh_vorticity
from .sph import real_sph_harm_all, real_y43, real_y41, bandlimited_field
from .configs import CONFIGS, make_config, config_subset

__all__ = [
    "cubed_sphere_grid",
    "random_sphere_points",
    "icosahedral_grid",
    "latlon_grid",
    "rh_vorticity",
    "real_sph_harm_all",
    "real_y43",
    "real_y41",
    "bandlimited_field",
    "CONFIGS",
    "make_config",
    "config_subset",
]
