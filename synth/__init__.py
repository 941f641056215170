"""Seeded synthetic inputs shared by the oracle, the GPU path, the tests and the benchmark.

This package holds input recipes only: point clouds, their bandwidth rule and the
named workload configurations.  None of the method's arithmetic lives here.
"""
from .generators import (  # noqa: F401
    s_curve,
    mnist_shaped,
    gaussian_cloud,
    median_sq_dist_eps,
    two_clusters,
)
from .configs import CONFIGS, SERVING, SERVING_FAMILIES, SERVING_PATHS, get_config, tree_depth  # noqa: F401
