"""ctypes mirror of include/fsm.h and the loader of libfsm.so.

Argument marshalling only: every step of the simulation runs inside libfsm (host planner and
HIP kernels).  The library must have been built (python -m paper_2603_28160_amd.build);
loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfsm.so")

FSM_ABI_VERSION = 2
MAXT = 8
MAX_EDGE = 4096

OK, EINVAL, ENOMEM, EDEVICE, EAGAIN, ENOTSUP = 0, -1, -2, -3, -4, -5
F64, F32 = 0, 1
TOOL_ROUND, TOOL_BALL = 0, 1
FLAG_SQ_ZERO, FLAG_NO_HIT, FLAG_LOW_COVERAGE = 1, 2, 4
OPT_ZMAP_STRATEGY, OPT_BUCKET_BYTES, OPT_GRAPHS = 1, 2, 3
OPT_TILE_SHAPE, OPT_TARGET_ROWS, OPT_AUTOTUNED = 4, 5, 6
FILTER_SMOOTH, FILTER_ROUGH = 0, 1
OPT_ASYNC_SLOTS, OPT_HBM_BUDGET, OPT_HIST_BYTES = 7, 8, 9
FSM_EAGAIN = -4
ZMAP_BINNED, ZMAP_SCATTER = 0, 1
# Z-map path of the last call (fsm_timings.zmap_path)
PATH_SCATTER, PATH_RUN, PATH_HIST, PATH_SUPER = 0, 1, 2, 3


class FsmTool(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_teeth", C.c_int32), ("n_edge", C.c_int32),
                ("uniform_pitch", C.c_int32), ("D", C.c_double), ("R_edge", C.c_double),
                ("helix", C.c_double), ("rake_radial", C.c_double), ("rake_axial", C.c_double),
                ("theta", C.c_double * MAXT), ("runout_ecc", C.c_double),
                ("runout_phase", C.c_double), ("eps_r", C.c_double * MAXT),
                ("eps_a", C.c_double * MAXT), ("tilt_lead", C.c_double),
                ("tilt_side", C.c_double)]


class FsmCut(C.Structure):
    _fields_ = [("f_z", C.c_double), ("a_p", C.c_double), ("a_e", C.c_double),
                ("phi0", C.c_double), ("steps_per_rev", C.c_int32), ("n_passes", C.c_int32),
                ("n_steps", C.c_int64), ("x_start", C.c_double), ("y_first", C.c_double),
                ("time_mode", C.c_int32), ("reserved", C.c_int32), ("v_c", C.c_double),
                ("dt", C.c_double), ("x_end", C.c_double)]


class FsmGrid(C.Structure):
    _fields_ = [("x0", C.c_double), ("y0", C.c_double), ("dd", C.c_double),
                ("nx", C.c_int64), ("ny", C.c_int64)]


class FsmPlanInfo(C.Structure):
    _fields_ = [("r_reach", C.c_double), ("x_start", C.c_double), ("y_first", C.c_double),
                ("n_passes", C.c_int64), ("n_steps", C.c_int64), ("n_evals", C.c_int64),
                ("n_cells", C.c_int64), ("zmap_bytes", C.c_int64),
                ("workspace_bytes", C.c_int64), ("zmap_path", C.c_int32), ("n_slices", C.c_int32)]


ROUGH_DOUBLES = ("Sa", "Sq", "Sp", "Sv", "Sz", "Ssk", "Sku", "Ra_feed", "Ra_pick", "mean",
                 "pos_err")
ROUGH_COUNTS = ("n_hit", "n_evals", "n_binned", "n_feed", "n_pick", "n_near")
NOALLOC_SCRATCH_BYTES = 64 << 20        # FSM_NOALLOC_SCRATCH_BYTES


class FsmRough(C.Structure):
    _fields_ = [(k, C.c_double) for k in ROUGH_DOUBLES] + \
               [(k, C.c_int64) for k in ROUGH_COUNTS] + \
               [("flags", C.c_uint32), ("reserved", C.c_uint32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}


class FsmTimings(C.Structure):
    _fields_ = [("upload_ms", C.c_float), ("fill_ms", C.c_float), ("scatter_ms", C.c_float),
                ("rough_ms", C.c_float), ("total_ms", C.c_float), ("count_ms", C.c_float),
                ("index_ms", C.c_float), ("write_ms", C.c_float), ("reduce_ms", C.c_float),
                ("n_slices", C.c_int32), ("valid", C.c_int32), ("zmap_path", C.c_int32),
                ("reserved", C.c_int32)]


class FsmJob(C.Structure):
    _fields_ = [("tool", C.POINTER(FsmTool)), ("cut", C.POINTER(FsmCut)),
                ("grid", C.POINTER(FsmGrid)), ("zmap_dev", C.c_void_p)]


class FsmTuneResult(C.Structure):
    _fields_ = [("strategy", C.c_int32), ("tile_shape", C.c_int32), ("target_rows", C.c_int32),
                ("n_tried", C.c_int32), ("best_ms", C.c_float), ("default_ms", C.c_float)]


class FsmTuneEntry(C.Structure):
    _fields_ = [("key", C.c_char * 64), ("strategy", C.c_int32), ("tile_shape", C.c_int32),
                ("target_rows", C.c_int32), ("reserved", C.c_int32)]


class FsmTextureSpec(C.Structure):
    _fields_ = [("lambda_s", C.c_double), ("lambda_c", C.c_double), ("trunc", C.c_double),
                ("level", C.c_int32), ("reserved", C.c_int32)]


class FsmRequest(C.Structure):
    _fields_ = [("tool", C.POINTER(FsmTool)), ("cut", C.POINTER(FsmCut)),
                ("grid", C.POINTER(FsmGrid)), ("arrival_s", C.c_double),
                ("zmap_dev", C.c_void_p)]


class FsmRequestResult(C.Structure):
    _fields_ = [("rough", FsmRough), ("admit_s", C.c_double), ("start_s", C.c_double),
                ("done_s", C.c_double), ("status", C.c_int32), ("batch", C.c_int32),
                ("slot", C.c_int32), ("pad", C.c_int32)]


class FsmServeConfig(C.Structure):
    _fields_ = [("precision", C.c_int32), ("n_slots", C.c_int32), ("max_batch", C.c_int32),
                ("realtime", C.c_int32), ("arena_bytes", C.c_int64), ("slot_bytes", C.c_int64)]


class FsmServeModel(C.Structure):
    _fields_ = [("launch_s", C.c_double), ("per_eval_s", C.c_double), ("per_cell_s", C.c_double)]


# every symbol include/fsm.h declares, with its ctypes signature
P = C.POINTER
SIGNATURES = {
    "fsm_version": ([], C.c_int),
    "fsm_strerror": ([C.c_int], C.c_char_p),
    "fsm_plan": ([P(FsmTool), P(FsmCut), P(FsmGrid), C.c_int, P(FsmPlanInfo)], C.c_int),
    "fsm_edge_points": ([P(FsmTool), P(FsmCut), P(C.c_double)], C.c_int),
    "fsm_refine": ([P(FsmTool), P(FsmCut), P(FsmGrid), C.c_double, P(FsmTool), P(FsmCut)], C.c_int),
    "fsm_ctx_create": ([P(C.c_void_p), C.c_int], C.c_int),
    "fsm_ctx_destroy": ([C.c_void_p], None),
    "fsm_last_error": ([C.c_void_p, C.c_char_p, C.c_size_t], C.c_int),
    "fsm_ctx_set_option": ([C.c_void_p, C.c_int, C.c_int64], C.c_int),
    "fsm_ctx_set_profiling": ([C.c_void_p, C.c_int], C.c_int),
    "fsm_last_timings": ([C.c_void_p, P(FsmTimings)], C.c_int),
    "fsm_simulate": ([C.c_void_p, P(FsmTool), P(FsmCut), P(FsmGrid), C.c_int, C.c_void_p,
                      P(FsmRough), C.c_void_p], C.c_int),
    "fsm_simulate_noalloc": ([C.c_void_p, P(FsmTool), P(FsmCut), P(FsmGrid), C.c_int,
                              C.c_void_p, P(FsmRough), C.c_void_p], C.c_int),
    "fsm_roughness": ([C.c_void_p, P(FsmGrid), C.c_int, C.c_void_p, P(FsmRough), C.c_void_p],
                      C.c_int),
    "fsm_level": ([C.c_void_p, P(FsmGrid), C.c_int, C.c_void_p, C.c_void_p, P(C.c_double),
                   C.c_void_p], C.c_int),
    "fsm_filter": ([C.c_void_p, P(FsmGrid), C.c_int, C.c_void_p, C.c_void_p, C.c_double,
                    C.c_double, C.c_int, C.c_void_p], C.c_int),
    "fsm_texture": ([C.c_void_p, P(FsmGrid), C.c_int, C.c_void_p, C.c_void_p, P(FsmTextureSpec),
                     P(FsmRough), P(C.c_double), C.c_void_p], C.c_int),
    "fsm_texture_batch": ([C.c_void_p, C.c_int, P(FsmGrid), C.c_int, P(C.c_void_p), P(C.c_void_p),
                           P(FsmTextureSpec), P(FsmRough), P(C.c_double), C.c_void_p], C.c_int),
    "fsm_batch_submit": ([C.c_void_p, C.c_int, P(FsmJob), C.c_int, C.c_void_p, P(C.c_uint64)],
                         C.c_int),
    "fsm_batch_poll": ([C.c_void_p, C.c_uint64, P(C.c_int)], C.c_int),
    "fsm_batch_wait": ([C.c_void_p, C.c_uint64, P(FsmRough)], C.c_int),
    "fsm_simulate_batch": ([C.c_void_p, C.c_int, P(FsmJob), C.c_int, P(FsmRough), C.c_void_p],
                           C.c_int),
    "fsm_trajectory": ([C.c_void_p, P(FsmTool), P(FsmCut), P(FsmGrid), C.c_int, C.c_void_p,
                        C.c_void_p, C.c_void_p], C.c_int),
    "fsm_autotune": ([C.c_void_p, C.c_int, P(FsmJob), C.c_int, P(FsmTuneResult), C.c_void_p],
                     C.c_int),
    "fsm_tune_get": ([C.c_void_p, P(FsmTuneEntry), C.c_int, P(C.c_int)], C.c_int),
    "fsm_tune_set": ([C.c_void_p, P(FsmTuneEntry), C.c_int], C.c_int),
    "fsm_serve_run": ([C.c_void_p, P(FsmServeConfig), C.c_int, P(FsmRequest),
                       P(FsmRequestResult)], C.c_int),
    "fsm_serve_dry_run": ([P(FsmServeConfig), P(FsmServeModel), C.c_int, P(FsmRequest),
                           P(FsmRequestResult), P(C.c_int64)], C.c_int),
}

_lock = threading.Lock()
_lib = None


class FsmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} [{code}]")
        self.code = code


def load() -> C.CDLL:
    """Load libfsm.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: build it with "
                                  "`python -m paper_2603_28160_amd.build`")
            lib = C.CDLL(LIB_PATH)
            for name, (args, res) in SIGNATURES.items():
                f = getattr(lib, name)
                f.argtypes = args
                f.restype = res
            if lib.fsm_version() != FSM_ABI_VERSION:
                raise ImportError("libfsm ABI version mismatch")
            _lib = lib
    return _lib


def tool_struct(t) -> FsmTool:
    o = FsmTool()
    o.kind = int(t.kind)
    o.n_teeth = int(t.n_teeth)
    o.n_edge = int(t.n_edge)
    o.uniform_pitch = 1 if t.theta is None else 0
    o.D = t.D
    o.R_edge = t.R_edge
    o.helix = t.helix
    o.rake_radial = t.rake_radial
    o.rake_axial = t.rake_axial
    if t.theta is not None:
        if len(t.theta) > MAXT:
            raise ValueError("too many tooth angles")
        for k, v in enumerate(t.theta):
            o.theta[k] = v
    o.runout_ecc = t.runout_ecc
    o.runout_phase = t.runout_phase
    for k, v in enumerate(t.eps_r[:MAXT]):
        o.eps_r[k] = v
    for k, v in enumerate(t.eps_a[:MAXT]):
        o.eps_a[k] = v
    o.tilt_lead = t.tilt_lead
    o.tilt_side = t.tilt_side
    return o


def cut_struct(c) -> FsmCut:
    return FsmCut(f_z=c.f_z, a_p=c.a_p, a_e=c.a_e, phi0=c.phi0,
                  steps_per_rev=int(c.steps_per_rev), n_passes=int(c.n_passes),
                  n_steps=int(c.n_steps), x_start=c.x_start, y_first=c.y_first,
                  time_mode=int(c.time_mode), v_c=c.v_c, dt=c.dt, x_end=c.x_end)


def grid_struct(g) -> FsmGrid:
    return FsmGrid(x0=g.x0, y0=g.y0, dd=g.dd, nx=int(g.nx), ny=int(g.ny))
