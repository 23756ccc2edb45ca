"""Seeded synthetic workloads for PI^2-RH with an LWPR dynamics model.

This package only draws inputs (model parameters, start states, goals,
obstacles, nominal controls).  It holds none of the method's arithmetic, so
both the FP64 CPU oracle and the HIP path consume exactly the same values.
"""
from .instances import (  # noqa: F401
    DYN_POINTMASS2D, DYN_QUAD12, DYN_QUAD_HYBRID, DYN_DIMS, DYN_D, OBS_INDICATOR, OBS_SMOOTH,
    W_COST_TO_GO, W_TRAJECTORY, LWPRModel, Problem,
    make_lwpr, make_problem, config, tiny_problem, batched_config, paper_shape,
)
