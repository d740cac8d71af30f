"""Seeded synthetic graph generators shared by the oracle tests and the GPU path.

This package holds input construction only: mesh topologies, seeded edge
weights and CSR assembly.  It contains none of the coarsening arithmetic
(no degrees, scores, ordering, merging or contraction), so that the oracle
and the HIP implementation can both consume the same inputs without sharing
any of the method's code.
"""
from .meshes import (  # noqa: F401
    Graph,
    grid2d,
    grid3d,
    trimesh,
    batch_sides,
    batch_trimeshes,
    random_graph,
    from_edges,
    powerlaw_graph,
    tie_permutation,
)
