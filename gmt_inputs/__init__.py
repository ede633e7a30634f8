"""Seeded synthetic periodic voxel cells.

This module only produces inputs (binary voxel fields and random vectors).  It
holds none of the homogenization arithmetic, so both the GPU library's tests
and the CPU oracle may draw from it.

Voxel arrays are ``uint8`` of shape ``(N, N, N)`` indexed ``[z, y, x]`` so that
``arr.ravel()`` is the linear order ``x + N*(y + N*z)`` (x fastest).
"""

from .lattices import (  # noqa: F401
    FAMILIES,
    cell,
    cleanup_largest_component,
    diamond_sheet,
    gyroid_sheet,
    laminate,
    periodic_components,
    random_vectors,
    schwarz_p_sheet,
    spinodal,
    truss,
    uniform,
    winding_rank,
    workload_cell,
)
