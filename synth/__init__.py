"""Seeded synthetic inputs shared by the GPU path's tests/bench and the oracle.

This package holds no arithmetic of the method: it only draws closed
dislocation loops (segment end points and Burgers vectors).
"""
from .loops import (  # noqa: F401
    WORKLOADS,
    batch_sizes,
    make_batch,
    make_loops,
    make_workload,
    segment_subset,
)
