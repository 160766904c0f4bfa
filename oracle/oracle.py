"""ctypes shim over the FP64 CPU oracle (fsm_oracle.c).

TEST INFRASTRUCTURE ONLY.  Converts the parameter records of the workload module (any object
with the same attribute names) into the oracle's own C structures and calls it.  Nothing here
is shared with, or imported from, the GPU library.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fsm_oracle.c")
_HDR = os.path.join(_HERE, "fsm_oracle.h")
_LIB = os.path.join(_HERE, "liboracle.so")
# No contraction into fused multiply-adds and no compiler rewriting of libm calls: every
# operation is the one written in the source.
CFLAGS = ["-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-builtin",
          "-fno-fast-math", "-fPIC", "-shared", "-Wall"]

MAXT = 8


class OrTool(C.Structure):
    _fields_ = [("kind", C.c_int), ("n_teeth", C.c_int), ("n_edge", C.c_int),
                ("uniform_pitch", C.c_int), ("D", C.c_double), ("R_edge", C.c_double),
                ("helix", C.c_double), ("rake_f", C.c_double), ("rake_p", C.c_double),
                ("theta", C.c_double * MAXT), ("ecc", C.c_double), ("ecc_phase", C.c_double),
                ("eps_r", C.c_double * MAXT), ("eps_a", C.c_double * MAXT),
                ("tilt_lead", C.c_double), ("tilt_side", C.c_double)]


class OrCut(C.Structure):
    _fields_ = [("f_z", C.c_double), ("a_p", C.c_double), ("a_e", C.c_double),
                ("phi0", C.c_double), ("S", C.c_int), ("n_passes", C.c_int),
                ("n_steps", C.c_longlong), ("x_start", C.c_double), ("y_first", C.c_double),
                ("time_mode", C.c_int), ("v_c", C.c_double), ("dt", C.c_double),
                ("x_end", C.c_double)]


class OrGrid(C.Structure):
    _fields_ = [("x0", C.c_double), ("y0", C.c_double), ("dd", C.c_double),
                ("nx", C.c_longlong), ("ny", C.c_longlong)]


class OrPlan(C.Structure):
    _fields_ = [("r_reach", C.c_double), ("x_start", C.c_double), ("y_first", C.c_double),
                ("n_passes", C.c_longlong), ("n_steps", C.c_longlong),
                ("n_evals", C.c_longlong)]


class OrCounts(C.Structure):
    _fields_ = [("n_evals", C.c_longlong), ("n_binned", C.c_longlong)]


class OrRough(C.Structure):
    _fields_ = [(k, C.c_double) for k in
                ("Sa", "Sq", "Sp", "Sv", "Sz", "Ssk", "Sku", "Ra_feed", "Ra_pick", "mean")] + \
               [("n_hit", C.c_longlong), ("n_feed", C.c_longlong), ("n_pick", C.c_longlong)]


_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle into oracle/liboracle.so with gcc."""
    stale = (not os.path.exists(_LIB) or
             os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC), os.path.getmtime(_HDR)))
    if force or stale:
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _configure(L: C.CDLL) -> C.CDLL:
    P = C.POINTER
    L.or_edge_points.argtypes = [P(OrTool), P(OrCut), P(C.c_double), P(C.c_double)]
    L.or_plan.argtypes = [P(OrTool), P(OrCut), P(OrGrid), P(OrPlan)]
    L.or_point.argtypes = [P(OrTool), P(OrCut), P(OrGrid), C.c_longlong, C.c_longlong,
                           C.c_int, C.c_int, P(C.c_double)]
    L.or_simulate_window.argtypes = [P(OrTool), P(OrCut), P(OrGrid), C.c_longlong,
                                     C.c_longlong, C.c_longlong, C.c_longlong,
                                     P(C.c_double), P(C.c_longlong), P(OrCounts)]
    L.or_cell_bounds.argtypes = [P(OrTool), P(OrCut), P(OrGrid), C.c_double,
                                 P(C.c_double), P(C.c_double), P(C.c_double)]
    L.or_cell_bounds_window.argtypes = [P(OrTool), P(OrCut), P(OrGrid), C.c_double,
                                        C.c_longlong, C.c_longlong, C.c_longlong,
                                        C.c_longlong, P(C.c_double), P(C.c_double),
                                        P(C.c_double)]
    L.or_trajectory.argtypes = [P(OrTool), P(OrCut), P(OrGrid), P(C.c_double), P(C.c_int)]
    L.or_roughness.argtypes = [P(C.c_double), C.c_longlong, C.c_longlong, P(OrRough)]
    L.or_paper_trajectory_points.argtypes = [C.c_double, C.c_double, C.c_int,
                                             C.c_double, C.c_double, C.c_double]
    L.or_paper_trajectory_points.restype = C.c_longlong
    L.or_level.argtypes = [P(C.c_double), P(OrGrid), P(C.c_double), P(C.c_double)]
    L.or_gauss_filter.argtypes = [P(C.c_double), P(OrGrid), C.c_double, C.c_double, C.c_int,
                                  P(C.c_double)]
    L.or_gauss_filter_cells.argtypes = [P(C.c_double), P(OrGrid), C.c_double, C.c_double,
                                        C.c_int, P(C.c_longlong), C.c_longlong, P(C.c_double)]
    return L


def lib() -> C.CDLL:
    global _lib
    with _lock:
        if _lib is None:
            build()
            _lib = _configure(C.CDLL(_LIB))
    return _lib


@contextlib.contextmanager
def use_library(path: str):
    """Run the oracle's functions on another build of its source (a copy with a planted
    mistake, in the mutation tests) for the duration of the block."""
    global _lib
    lib()
    with _lock:
        saved = _lib
        _lib = _configure(C.CDLL(path))
    try:
        yield
    finally:
        with _lock:
            _lib = saved


def _tool(t) -> OrTool:
    o = OrTool()
    o.kind = int(t.kind)
    o.n_teeth = int(t.n_teeth)
    o.n_edge = int(t.n_edge)
    o.uniform_pitch = 1 if t.theta is None else 0
    o.D = t.D
    o.R_edge = t.R_edge
    o.helix = t.helix
    o.rake_f = t.rake_radial
    o.rake_p = t.rake_axial
    if t.theta is not None:
        for k, v in enumerate(t.theta):
            o.theta[k] = v
    o.ecc = t.runout_ecc
    o.ecc_phase = t.runout_phase
    for k, v in enumerate(t.eps_r):
        o.eps_r[k] = v
    for k, v in enumerate(t.eps_a):
        o.eps_a[k] = v
    o.tilt_lead = t.tilt_lead
    o.tilt_side = t.tilt_side
    return o


def _cut(c) -> OrCut:
    return OrCut(f_z=c.f_z, a_p=c.a_p, a_e=c.a_e, phi0=c.phi0, S=int(c.steps_per_rev),
                 n_passes=int(c.n_passes), n_steps=int(c.n_steps), x_start=c.x_start,
                 y_first=c.y_first, time_mode=int(c.time_mode), v_c=c.v_c, dt=c.dt,
                 x_end=c.x_end)


def _grid(g) -> OrGrid:
    return OrGrid(x0=g.x0, y0=g.y0, dd=g.dd, nx=int(g.nx), ny=int(g.ny))


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def edge_points(sim):
    """(pC [N,3], pT [z_n, N, 3]) of the discretised edge."""
    t = sim.tool
    pC = np.zeros((t.n_edge, 3))
    pT = np.zeros((t.n_teeth, t.n_edge, 3))
    rc = lib().or_edge_points(C.byref(_tool(t)), C.byref(_cut(sim.cut)), _dp(pC), _dp(pT))
    if rc:
        raise ValueError(f"or_edge_points: invalid parameters ({rc})")
    return pC, pT


def plan(sim) -> dict:
    p = OrPlan()
    rc = lib().or_plan(C.byref(_tool(sim.tool)), C.byref(_cut(sim.cut)),
                       C.byref(_grid(sim.grid)), C.byref(p))
    if rc:
        raise ValueError(f"or_plan: invalid parameters ({rc})")
    return {k: getattr(p, k) for k, _ in OrPlan._fields_}


def point(sim, q: int, s: int, K: int, p: int) -> np.ndarray:
    out = np.zeros(3)
    rc = lib().or_point(C.byref(_tool(sim.tool)), C.byref(_cut(sim.cut)),
                        C.byref(_grid(sim.grid)), q, s, K, p, _dp(out))
    if rc:
        raise ValueError(f"or_point: invalid parameters ({rc})")
    return out


def simulate(sim, window=None, winners: bool = False):
    """Per-cell-minimum Z-map (float64, +inf = empty) of the window (i0, i1, j0, j1), the
    whole grid by default.  Returns (Z, counts dict[, winner indices])."""
    g = sim.grid
    i0, i1, j0, j1 = window if window is not None else (0, g.nx, 0, g.ny)
    Z = np.empty((j1 - j0, i1 - i0))
    W = np.empty((j1 - j0, i1 - i0), dtype=np.int64) if winners else None
    cnt = OrCounts()
    rc = lib().or_simulate_window(
        C.byref(_tool(sim.tool)), C.byref(_cut(sim.cut)), C.byref(_grid(g)),
        i0, i1, j0, j1, _dp(Z),
        W.ctypes.data_as(C.POINTER(C.c_longlong)) if winners else None, C.byref(cnt))
    if rc:
        raise ValueError(f"or_simulate_window: invalid parameters ({rc})")
    counts = {"n_evals": cnt.n_evals, "n_binned": cnt.n_binned}
    return (Z, counts, W) if winners else (Z, counts)


def trajectory(sim):
    """(xyz [n_passes, n_steps, n_teeth, 3], edge index [n_passes, n_steps, n_teeth]) of the
    lowest edge point per time step and tooth."""
    p = plan(sim)
    shape = (p["n_passes"], p["n_steps"], sim.tool.n_teeth)
    xyz = np.empty(shape + (3,))
    idx = np.empty(shape, dtype=np.int32)
    rc = lib().or_trajectory(C.byref(_tool(sim.tool)), C.byref(_cut(sim.cut)),
                             C.byref(_grid(sim.grid)), _dp(xyz),
                             idx.ctypes.data_as(C.POINTER(C.c_int)))
    if rc:
        raise ValueError(f"or_trajectory: invalid parameters ({rc})")
    return xyz, idx


def cell_bounds(sim, delta: float, window=None):
    """(lo, hi, top) per cell when every evaluation may move by up to delta in x and y, over
    the whole grid or the cell window (i0, i1, j0, j1)."""
    g = sim.grid
    i0, i1, j0, j1 = window if window is not None else (0, g.nx, 0, g.ny)
    shape = (j1 - j0, i1 - i0)
    lo, hi, top = np.empty(shape), np.empty(shape), np.empty(shape)
    rc = lib().or_cell_bounds_window(C.byref(_tool(sim.tool)), C.byref(_cut(sim.cut)),
                                     C.byref(_grid(g)), float(delta), i0, i1, j0, j1,
                                     _dp(lo), _dp(hi), _dp(top))
    if rc:
        raise ValueError(f"or_cell_bounds: invalid parameters ({rc})")
    return lo, hi, top


def roughness(Z: np.ndarray) -> dict:
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    r = OrRough()
    rc = lib().or_roughness(_dp(Z), Z.shape[1], Z.shape[0], C.byref(r))
    if rc:
        raise ValueError("or_roughness: bad input")
    return {k: getattr(r, k) for k, _ in OrRough._fields_}


def paper_trajectory_points(v_c: float, f_z: float, z_n: int, D: float, L: float,
                            dt: float) -> int:
    return int(lib().or_paper_trajectory_points(v_c, f_z, z_n, D, L, dt))


def level(Z: np.ndarray, grid):
    """(Z minus its least-squares plane over the hit cells, (c0, c1, c2)) with the plane
    c0 + c1 x + c2 y in the grid's node coordinates."""
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    out = np.empty_like(Z)
    c = np.empty(3)
    rc = lib().or_level(_dp(Z), C.byref(_grid(grid)), _dp(out), _dp(c))
    if rc:
        raise ValueError(f"or_level: {'degenerate hit set' if rc == -2 else 'bad input'}")
    return out, tuple(float(v) for v in c)


def gauss_filter(Z: np.ndarray, grid, cutoff: float, trunc: float = 1.0, highpass: bool = False,
                 cells=None):
    """Areal Gaussian filter of the Z-map (+inf = empty): the weighted mean (S-filter) or, with
    highpass, Z minus it (L-filter).  cells: flat indices to evaluate (default: every cell)."""
    Z = np.ascontiguousarray(Z, dtype=np.float64)
    mode = 1 if highpass else 0
    if cells is None:
        out = np.empty_like(Z)
        rc = lib().or_gauss_filter(_dp(Z), C.byref(_grid(grid)), cutoff, trunc, mode, _dp(out))
    else:
        cells = np.ascontiguousarray(cells, dtype=np.int64)
        out = np.empty(cells.shape[0])
        rc = lib().or_gauss_filter_cells(_dp(Z), C.byref(_grid(grid)), cutoff, trunc, mode,
                                         cells.ctypes.data_as(C.POINTER(C.c_longlong)),
                                         cells.shape[0], _dp(out))
    if rc:
        raise ValueError("or_gauss_filter: bad input")
    return out


__all__ = ["build", "lib", "edge_points", "plan", "point", "simulate", "trajectory", "cell_bounds",
           "roughness", "paper_trajectory_points",
           "level", "gauss_filter"]
