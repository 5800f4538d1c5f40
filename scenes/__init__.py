"""Seeded synthetic voxel scenes shared by the tests, the oracle checks and the bench.

This module only draws and paints voxel grids (conductor ids and relative
permittivities).  It holds none of the solver's arithmetic: no panels, no
integrals, no linear algebra.  Every scene is a plain dict::

    {"name": str, "cond_id": int32[nx, ny, nz] (-1 = not a conductor),
     "eps_r": float64[nx, ny, nz] (relative permittivity of non-conductor voxels),
     "dv": float (voxel edge in metres), "eps_b": float (background outside the box),
     "meta": dict}

Arrays are C ordered with x slowest, z fastest (voxel (i, j, k) occupies
[i, i+1] x [j, j+1] x [k, k+1] in units of dv).
"""
from .generators import (  # noqa: F401
    cube, parallel_plates, random_boxes, meander, gradient_scene, random_small,
    coated_sphere, uneven_batch, by_name, CONFIG_NAMES,
)
