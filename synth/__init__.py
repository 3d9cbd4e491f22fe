"""Seeded synthetic point clouds shaped like the FEC paper's workloads.

This package holds input generators only: nothing in it computes distances
between points, neighbourhoods, components or labels.  Both the CPU oracle's
tests and the GPU path's tests/bench draw their inputs from here.
"""

from .clouds import (  # noqa: F401
    SensorModel,
    blobs_cloud,
    lidar_frame,
    lidar_map,
    map_trajectory,
    random_cloud,
    near_threshold_cloud,
    chain_cloud,
    blob_lattice,
    lidar_batch,
    serve_trace,
    voxel_clusters,
    SWEEPS,
    SWEEP_D,
    make_batch_config,
    CONFIGS,
    make_config,
)
