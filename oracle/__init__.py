"""FP64 CPU oracle of the milling-topography method (test infrastructure only).

A plain, slow, obviously correct restatement of the method, written in C (fsm_oracle.c) and
reached through ctypes.  It shares no code with the GPU library and is used only by the tests,
the smoke check and the benchmark's CPU-baseline leg.
"""
from .oracle import (  # noqa: F401
    build, lib, edge_points, plan, point, simulate, trajectory, cell_bounds, roughness,
    paper_trajectory_points, level, gauss_filter,
)
