"""Seeded synthetic inputs shared by the CPU oracle tests and the HIP path.

This package only draws numbers.  It holds none of the k-NN method's arithmetic
(no distance evaluation used as a reference, no selection, no pivoting), so the
oracle and the HIP path remain independent of each other; both are handed the
arrays produced here.
"""
from .gen import (  # noqa: F401
    hash_u64,
    uniform01,
    normal,
    uniform_points,
    normal_points,
    gmm_points,
    sqdist_matrix_normal,
    adversarial_rows,
    SEEDS,
)
