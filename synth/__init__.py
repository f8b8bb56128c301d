"""Seeded synthetic workloads: triangle meshes and sun directions.

This package only generates geometry and random numbers.  It contains none
of the radiosity arithmetic (view factors, visibility, compression, matvec,
solve, insolation); both the library under test and the CPU reference
consume what it produces.
"""
from .meshes import (  # noqa: F401
    CapSpec, DemSpec, cap_mesh, dem_mesh, sun_directions, sun_grid_azimuth,
    CAP_SMALL, CAP_LARGE, DEM_256, DEM_512, instance_sizes, dem_instance, mlp_init,
    BodySpec, body_mesh,
)
