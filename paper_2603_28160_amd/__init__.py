"""MI355X-native forward solution method (FSM) for milled 3D surface topography.

libfsm.so (HIP for gfx950, C ABI in include/fsm.h) does the work: edge discretisation, the
cutting-edge -> tool -> spindle -> workpiece kinematics at every time step, binning into the
workpiece grid, the per-cell minimum Z-map and its areal / profile roughness.  This package
is its thin Python binding; torch provides device memory and streams.

    from paper_2603_28160_amd import Context, workloads
    with Context(0) as ctx:
        zmap, rough = ctx.fsm_simulate(workloads.config2(), precision="f32")
"""
from ._abi import F32, F64, FsmError, TOOL_BALL, TOOL_ROUND  # noqa: F401
from .api import (Context, fsm_edge_points, fsm_plan, fsm_refine, fsm_serve_dry_run,  # noqa: F401
                  fsm_version)
from . import workloads  # noqa: F401
