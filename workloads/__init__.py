"""Seeded synthetic inputs shared by the oracle side and the HIP side.

This package holds only input generation and file formats: random MLP
weights, random boxes, random sample points and the synthetic scalar fields
that stand in for the paper's datasets. It performs none of the range
analysis, uncertainty propagation, classification or marching-cubes
arithmetic; those live in ``oracle/`` (reference) and in the HIP library
(product), which never import each other.
"""

from .weights import MLPWeights, he_normal_mlp, read_weights, write_weights
from .cells import random_boxes, uniform_points

__all__ = [
    "MLPWeights",
    "he_normal_mlp",
    "read_weights",
    "write_weights",
    "random_boxes",
    "uniform_points",
]
