"""Seeded synthetic inputs for the GenEO two-level Schwarz / PCG path.

This package only *describes* problems: grid sizes, subdomain layout, the
per-element coefficient arrays and solver options.  It holds none of the
method's arithmetic (no assembly, no decomposition, no solver step), so the
CPU oracle and the HIP path can both read the same inputs without sharing
code.  Every random draw uses ``numpy.random.Generator(PCG64(seed))``.
"""
from .problems import (  # noqa: F401
    Problem,
    darcy_problem,
    elasticity_problem,
    channels_2d,
    grf_2d,
    layers_3d,
    laminate_3d,
    laminate_s20,
    layered_2d,
    CONFIGS,
)
from .fields import (  # noqa: F401
    channel_field,
    grf_exponential_2d,
    inclusions_2d,
    z_layers_3d,
    ply_stiffness,
    isotropic_stiffness,
    rotate_z90,
    voigt_upper,
)
