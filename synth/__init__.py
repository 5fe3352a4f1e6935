"""Seeded synthetic inputs for the fast flow-based cartogram hot path.

The paper measures on real country maps (USA, India, China, Kensington and
Chelsea; main text, benchmarking sections) whose polygons and statistics are
not available here.  Seeded bounded Voronoi maps stand in for them: region
counts from 16 to 600 bracket the paper's maps, and polygon edges are
subdivided so that vertex counts reach the sizes of detailed borders.

This package holds only input synthesis.  It computes none of the method's
steps (areas, rasterisation, transforms, velocities, integration); both the
oracle and the HIP path consume its output unchanged.
"""
from .voronoi import (  # noqa: F401
    CartogramMap,
    make_map,
    workload,
    grid_nodes,
    warped_nodes,
    WORKLOADS,
)
