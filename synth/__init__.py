"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This package only draws inputs: skeleton samples (centre, ball radius, weight),
rotations and poses. It holds none of the method's arithmetic, so both the
FP64 oracle and the HIP path can consume it without sharing any computation.
"""

from .workloads import (  # noqa: F401
    Part,
    Assembly,
    ServingWorkload,
    polyline_part,
    shoemake_rotations,
    config_c1,
    config_c2,
    config_c3,
    config_c4,
    config_c5,
    random_part,
    lattice_poses,
    SIGMA,
    PENALTY,
)
