"""Seeded synthetic inputs for the PCEXP DG-Euler workloads.

This package generates *inputs only*: vertex/element arrays of the meshes,
analytic flow fields evaluated at caller-supplied points, seeded
perturbations and random directions.  It holds none of the method's
arithmetic (no quadrature, basis, flux, Jacobian, Krylov or time-stepping
code), so that both the FP64 CPU oracle and the HIP path can consume the
same inputs without sharing any part of the method.
"""

from .meshes import (MeshArrays, periodic_square, channel_bump, periodic_cube, box_cube,
                     stretched_square, BC_SLIP, BC_FARFIELD)
from .fields import (GAMMA, freestream_prim, prim_to_cons, isentropic_vortex,
                     uniform_state, perturbation, random_directions,
                     paper_vortex, random_unit_vector)
from .configs import CONFIGS, get_config, build_mesh

__all__ = [
    "MeshArrays", "periodic_square", "channel_bump", "periodic_cube", "box_cube",
    "stretched_square", "BC_SLIP", "BC_FARFIELD", "GAMMA", "freestream_prim",
    "prim_to_cons", "isentropic_vortex", "uniform_state", "perturbation",
    "random_directions", "random_unit_vector", "paper_vortex", "CONFIGS", "get_config", "build_mesh",
]
