"""Seeded synthetic workloads for point-to-plane ICP and normal estimation.

This package only draws inputs: point clouds, rigid transforms and the
parameters that go with them.  It holds none of the method's arithmetic
(no neighbour search, no covariance, no normal equations), so both the CPU
oracle and the GPU path can consume it without sharing any method code.
"""
from .scenes import (  # noqa: F401
    CONFIGS,
    Workload,
    BatchWorkload,
    batch_workload,
    pose_pairs,
    pose_net_init,
    POSE_CONFIG,
    POSE_NET_SHAPES,
    make_workload,
    random_rigid,
    apply_rigid,
    sphere_plane,
    room_scan,
    street_scan,
    lattice_cloud,
    uniform_cloud,
    rng_for,
)
