"""Seeded synthetic inputs for the greedy D-optimal sensor-selection path.

This module only *makes inputs*: the dense data-space matrix
``K = F F^T / n_m + sigma^2 I`` of the linear-Gaussian inverse problem in its
data-space form (Sec. II-B, definition of K) with a synthetic parameter-to-
observable matrix ``F``.  It holds none of the selection method's arithmetic
(no Cholesky, no log-determinant, no Schur complement), so both the CPU oracle
and the HIP path can consume what it produces.
"""
from .synth import (  # noqa: F401
    TILE,
    tile_seed,
    f_tile,
    f_matrix,
    k_row_panels,
    make_K,
    make_K_lower_panels,
    make_K_sensor_noise,
    make_K_weighted_noise,
    k_sub_lower,
)
from .configs import CONFIGS, batched_instance_specs, Spec  # noqa: F401
