"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This package holds only input generation: voxelised permittivity arrays for
the body families the paper studies (dielectric spheres, Pancharatnam-Berry
phase fin metasurfaces on a slab, random ellipsoid unions), incident
plane-wave channel descriptions and detector angle grids.  It contains none
of the method's arithmetic (no Green's function, no operator, no far field,
no correlation formula), so sharing it does not couple the oracle to the
HIP path.
"""

from .geometry import (  # noqa: F401
    Grid,
    default_origin,
    sphere,
    ellipsoid_union,
    random_ellipsoid_body,
    metasurface_fins,
    metasurface_family,
    pb_metasurface,
    paper_metasurface,
    cap_directions,
    uv_directions,
    pb_rotation_step,
    planewave,
    random_planewave,
    circular_pol_basis,
)
