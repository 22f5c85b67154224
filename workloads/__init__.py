"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This package produces images and parameter sets only; it holds none of the
encoder's arithmetic (no dictionary, no pursuit, no quadtree logic).
"""
from .gen import (  # noqa: F401
    piecewise_image, gradient_edges_image, rgb_to_ycbcr, workload,
    C4_SIZES, sweep_trials, WORKLOADS,
)
