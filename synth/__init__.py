"""Seeded synthetic inputs for the ray-tracing radiative-transfer hot path.

This package builds point clouds, neighbour lists, opacity/emissivity tables,
velocities and frequency grids.  It holds none of the method's arithmetic (no
tracing, no direction sets, no transfer solve): both the CPU oracle and the HIP
library consume what it produces, and neither depends on the other.
"""
from .models import (  # noqa: F401
    Model,
    FreqGrid,
    concat_models,
    csr_from_edges,
    delaunay_csr,
    lattice_model,
    sphere_model,
    tiny_model,
    wind_model,
    octree_model,
    sph_cloud_model,
    sph_batch_models,
    to_fp32_tables,
)
