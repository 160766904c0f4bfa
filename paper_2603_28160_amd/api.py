"""Python binding of libfsm: the C-ABI calls under the same names, with torch supplying the
device memory and the stream.

Only argument marshalling happens here; edge discretisation, kinematics, binning, the
per-cell minimum and the roughness all run inside libfsm.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Tuple

import numpy as np

from . import _abi

PRECISIONS = {"f64": _abi.F64, "f32": _abi.F32, _abi.F64: _abi.F64, _abi.F32: _abi.F32}


def _prec(p) -> int:
    try:
        return PRECISIONS[p]
    except KeyError:
        raise ValueError(f"precision must be 'f64' or 'f32', got {p!r}") from None


def _check(rc: int, what: str, ctx=None):
    if rc != _abi.OK:
        lib = _abi.load()
        msg = lib.fsm_strerror(rc).decode()
        if ctx is not None:
            buf = C.create_string_buffer(512)
            lib.fsm_last_error(ctx, buf, 512)
            if buf.value:
                msg += ": " + buf.value.decode()
        raise _abi.FsmError(rc, f"{what}: {msg}")


def fsm_version() -> int:
    return _abi.load().fsm_version()


def fsm_plan(sim, precision="f64") -> dict:
    """Resolved path and sizes of one simulation (host only)."""
    info = _abi.FsmPlanInfo()
    rc = _abi.load().fsm_plan(C.byref(_abi.tool_struct(sim.tool)), C.byref(_abi.cut_struct(sim.cut)),
                              C.byref(_abi.grid_struct(sim.grid)), _prec(precision), C.byref(info))
    _check(rc, "fsm_plan")
    return {k: getattr(info, k) for k, _ in info._fields_}


def fsm_edge_points(sim) -> np.ndarray:
    """Tool-frame edge points [n_teeth, n_edge, 3] (host only)."""
    t = sim.tool
    out = np.zeros((t.n_teeth, t.n_edge, 3))
    rc = _abi.load().fsm_edge_points(C.byref(_abi.tool_struct(t)), C.byref(_abi.cut_struct(sim.cut)),
                                     out.ctypes.data_as(C.POINTER(C.c_double)))
    _check(rc, "fsm_edge_points")
    return out


def fsm_refine(sim, spacing: float):
    """Coverage-complete planning: a copy of `sim` whose edge-point count and time step keep
    every pair of consecutive samples of the swept edge at most `spacing` apart."""
    import dataclasses
    t_in, c_in = _abi.tool_struct(sim.tool), _abi.cut_struct(sim.cut)
    t_out, c_out = _abi.FsmTool(), _abi.FsmCut()
    rc = _abi.load().fsm_refine(C.byref(t_in), C.byref(c_in), C.byref(_abi.grid_struct(sim.grid)),
                                float(spacing), C.byref(t_out), C.byref(c_out))
    _check(rc, "fsm_refine")
    tool = dataclasses.replace(sim.tool, n_edge=int(t_out.n_edge))
    cut = dataclasses.replace(sim.cut, steps_per_rev=int(c_out.steps_per_rev), dt=c_out.dt,
                              n_steps=int(c_out.n_steps))
    return sim.replace(tool=tool, cut=cut, name=(sim.name + "_refined") if sim.name else "")


def _torch():
    import torch
    return torch


def _stream_handle(stream, device: int) -> int:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return int(stream.cuda_stream)


def _requests(requests, precision, ctx=None):
    n = len(requests)
    reqs = (_abi.FsmRequest * n)()
    keep = []
    for k, (s, arrival, z) in enumerate(requests):
        if z is not None and ctx is not None:
            ctx._check_zmap(s.grid, precision, z)
        t, c, g = _abi.tool_struct(s.tool), _abi.cut_struct(s.cut), _abi.grid_struct(s.grid)
        keep += [t, c, g]
        reqs[k].tool = C.pointer(t)
        reqs[k].cut = C.pointer(c)
        reqs[k].grid = C.pointer(g)
        reqs[k].arrival_s = float(arrival)
        reqs[k].zmap_dev = None if z is None else (z if isinstance(z, int) else z.data_ptr())
    return reqs, keep


def _result(o) -> dict:
    return {"rough": o.rough.as_dict(), "status": o.status, "batch": o.batch, "slot": o.slot,
            "admit_s": o.admit_s, "start_s": o.start_s, "done_s": o.done_s}


def fsm_serve_dry_run(requests, precision="f32", n_slots=2, max_batch=16, realtime=True,
                      arena_bytes=1 << 30, slot_bytes=1 << 30, launch_s=50e-6,
                      per_eval_s=5e-12, per_cell_s=5e-11):
    """The serving scheduler on the host against a modelled device (no GPU): requests are
    (sim, arrival_s, zmap) with zmap None (server-held) or any non-None marker (caller-owned).
    Returns (per-request dicts, most arena bytes held at once)."""
    n = len(requests)
    cfg = _abi.FsmServeConfig(_prec(precision), n_slots, max_batch, 1 if realtime else 0,
                              int(arena_bytes), int(slot_bytes))
    model = _abi.FsmServeModel(launch_s, per_eval_s, per_cell_s)
    marked = [(s, a, None if z is None else 1) for s, a, z in requests]
    reqs, keep = _requests(marked, precision)
    out = (_abi.FsmRequestResult * max(n, 1))()
    peak = C.c_int64(0)
    rc = _abi.load().fsm_serve_dry_run(C.byref(cfg), C.byref(model), n, reqs, out, C.byref(peak))
    _check(rc, "fsm_serve_dry_run")
    del keep
    return [_result(out[k]) for k in range(n)], peak.value


class Context:
    """One libfsm context on one HIP device (fsm_ctx_create / fsm_ctx_destroy)."""

    def __init__(self, device: int = 0):
        self.device = int(device)
        self._lib = _abi.load()
        self._batches = {}   # asynchronous batch id -> number of simulations
        h = C.c_void_p()
        rc = self._lib.fsm_ctx_create(C.byref(h), self.device)
        _check(rc, "fsm_ctx_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.fsm_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def handle(self):
        return self._h

    def fsm_ctx_set_option(self, option: int, value: int):
        _check(self._lib.fsm_ctx_set_option(self._h, int(option), int(value)), "fsm_ctx_set_option", self._h)

    def set_strategy(self, name: str):
        """Z-map strategy: 'binned' (tile buckets + LDS reduction) or 'scatter'."""
        v = {"binned": _abi.ZMAP_BINNED, "scatter": _abi.ZMAP_SCATTER}[name]
        self.fsm_ctx_set_option(_abi.OPT_ZMAP_STRATEGY, v)

    def fsm_ctx_set_profiling(self, on: bool = True):
        _check(self._lib.fsm_ctx_set_profiling(self._h, 1 if on else 0), "fsm_ctx_set_profiling", self._h)

    def fsm_last_timings(self) -> dict:
        t = _abi.FsmTimings()
        _check(self._lib.fsm_last_timings(self._h, C.byref(t)), "fsm_last_timings", self._h)
        return {k: getattr(t, k) for k, _ in t._fields_}

    def new_zmap(self, grid, precision="f64"):
        torch = _torch()
        dt = torch.float64 if _prec(precision) == _abi.F64 else torch.float32
        return torch.empty((int(grid.ny), int(grid.nx)), dtype=dt, device=f"cuda:{self.device}")

    def _check_zmap(self, grid, precision, zmap):
        torch = _torch()
        dt = torch.float64 if _prec(precision) == _abi.F64 else torch.float32
        if (not isinstance(zmap, torch.Tensor) or zmap.dtype != dt or not zmap.is_cuda
                or zmap.device.index != self.device or not zmap.is_contiguous()
                or zmap.numel() != int(grid.nx) * int(grid.ny)):
            raise ValueError("zmap must be a contiguous device tensor of nx*ny elements of the "
                             "precision's dtype on the context's device")

    def fsm_simulate(self, sim, precision="f64", zmap=None, roughness: bool = True,
                     stream=None) -> Tuple[object, Optional[dict]]:
        """Run one simulation; returns (Z-map tensor [ny, nx], roughness dict or None)."""
        if zmap is None:
            zmap = self.new_zmap(sim.grid, precision)
        self._check_zmap(sim.grid, precision, zmap)
        out = _abi.FsmRough()
        rc = self._lib.fsm_simulate(
            self._h, C.byref(_abi.tool_struct(sim.tool)), C.byref(_abi.cut_struct(sim.cut)),
            C.byref(_abi.grid_struct(sim.grid)), _prec(precision), C.c_void_p(zmap.data_ptr()),
            C.byref(out) if roughness else None, C.c_void_p(_stream_handle(stream, self.device)))
        _check(rc, "fsm_simulate", self._h)
        return zmap, (out.as_dict() if roughness else None)

    def fsm_simulate_noalloc(self, sim, zmap, precision="f64", stream=None) -> dict:
        """fsm_simulate into the caller's Z-map tensor without any device or pinned-host
        allocation by the library (its scratch is a fixed per-GPU array); returns the
        roughness dict."""
        self._check_zmap(sim.grid, precision, zmap)
        out = _abi.FsmRough()
        rc = self._lib.fsm_simulate_noalloc(
            self._h, C.byref(_abi.tool_struct(sim.tool)), C.byref(_abi.cut_struct(sim.cut)),
            C.byref(_abi.grid_struct(sim.grid)), _prec(precision), C.c_void_p(zmap.data_ptr()),
            C.byref(out), C.c_void_p(_stream_handle(stream, self.device)))
        _check(rc, "fsm_simulate_noalloc", self._h)
        return out.as_dict()

    def fsm_trajectory(self, sim, precision="f64", stream=None):
        """Lowest edge point per (pass, step, tooth) in the workpiece frame: returns (xyz
        tensor [n_passes, n_steps, n_teeth, 3], edge-index tensor [n_passes, n_steps, n_teeth])."""
        torch = _torch()
        p = fsm_plan(sim, precision)
        shape = (int(p["n_passes"]), int(p["n_steps"]), int(sim.tool.n_teeth))
        dt = torch.float64 if _prec(precision) == _abi.F64 else torch.float32
        dev = f"cuda:{self.device}"
        xyz = torch.empty(shape + (3,), dtype=dt, device=dev)
        idx = torch.empty(shape, dtype=torch.int32, device=dev)
        rc = self._lib.fsm_trajectory(
            self._h, C.byref(_abi.tool_struct(sim.tool)), C.byref(_abi.cut_struct(sim.cut)),
            C.byref(_abi.grid_struct(sim.grid)), _prec(precision), C.c_void_p(xyz.data_ptr()),
            C.c_void_p(idx.data_ptr()), C.c_void_p(_stream_handle(stream, self.device)))
        _check(rc, "fsm_trajectory", self._h)
        return xyz, idx

    def fsm_roughness(self, grid, zmap, precision="f64", stream=None) -> dict:
        """Roughness of an existing device Z-map (+inf = empty cell)."""
        self._check_zmap(grid, precision, zmap)
        out = _abi.FsmRough()
        rc = self._lib.fsm_roughness(self._h, C.byref(_abi.grid_struct(grid)), _prec(precision),
                                     C.c_void_p(zmap.data_ptr()), C.byref(out),
                                     C.c_void_p(_stream_handle(stream, self.device)))
        _check(rc, "fsm_roughness", self._h)
        return out.as_dict()

    def _out_map(self, grid, precision, zmap, out):
        if out is None:
            out = self.new_zmap(grid, precision)
        self._check_zmap(grid, precision, zmap)
        self._check_zmap(grid, precision, out)
        return out

    def fsm_level(self, grid, zmap, precision="f64", out=None, stream=None):
        """Subtract the least-squares plane of the hit cells (F-operator); returns (levelled
        map, (c0, c1, c2)) with the plane c0 + c1 x + c2 y.  out may be zmap (in place)."""
        out = self._out_map(grid, precision, zmap, out)
        plane = (C.c_double * 3)()
        rc = self._lib.fsm_level(self._h, C.byref(_abi.grid_struct(grid)), _prec(precision),
                                 C.c_void_p(zmap.data_ptr()), C.c_void_p(out.data_ptr()), plane,
                                 C.c_void_p(_stream_handle(stream, self.device)))
        _check(rc, "fsm_level", self._h)
        return out, tuple(plane)

    def fsm_filter(self, grid, zmap, cutoff: float, precision="f64", highpass: bool = False,
                   trunc: float = 1.0, out=None, stream=None):
        """Areal Gaussian filter of cut-off `cutoff` mm: the weighted mean (S-filter) or, with
        highpass, the map minus it (L-filter).  out may be zmap (in place)."""
        out = self._out_map(grid, precision, zmap, out)
        rc = self._lib.fsm_filter(self._h, C.byref(_abi.grid_struct(grid)), _prec(precision),
                                  C.c_void_p(zmap.data_ptr()), C.c_void_p(out.data_ptr()),
                                  float(cutoff), float(trunc),
                                  _abi.FILTER_ROUGH if highpass else _abi.FILTER_SMOOTH,
                                  C.c_void_p(_stream_handle(stream, self.device)))
        _check(rc, "fsm_filter", self._h)
        return out

    def fsm_texture(self, grid, zmap, precision="f64", lambda_s: float = 0.01,
                    lambda_c: float = 0.8, level: bool = True, trunc: float = 1.0, out=None,
                    stream=None):
        """S-filter -> F-operator -> L-filter, then the roughness of the result (defaults: the
        paper's instrument, 10 um and 0.8 mm).  Returns (map, roughness dict, plane)."""
        out = self._out_map(grid, precision, zmap, out)
        spec = _abi.FsmTextureSpec(lambda_s=float(lambda_s), lambda_c=float(lambda_c),
                                   trunc=float(trunc), level=1 if level else 0)
        r = _abi.FsmRough()
        plane = (C.c_double * 3)()
        rc = self._lib.fsm_texture(self._h, C.byref(_abi.grid_struct(grid)), _prec(precision),
                                   C.c_void_p(zmap.data_ptr()), C.c_void_p(out.data_ptr()),
                                   C.byref(spec), C.byref(r), plane,
                                   C.c_void_p(_stream_handle(stream, self.device)))
        _check(rc, "fsm_texture", self._h)
        return out, r.as_dict(), tuple(plane)

    def fsm_texture_batch(self, grid, zmaps, precision="f64", lambda_s: float = 0.01,
                          lambda_c: float = 0.8, level: bool = True, trunc: float = 1.0,
                          outs=None, stream=None):
        """fsm_texture over many maps of one grid in one launch sequence; returns (maps,
        roughness dicts, planes), in the order of `zmaps`.  outs may be zmaps (in place)."""
        n = len(zmaps)
        if n == 0:
            return [], [], []
        if outs is None:
            outs = [self.new_zmap(grid, precision) for _ in range(n)]
        if len(outs) != n:
            raise ValueError("outs must hold one map per input map")
        for z, o in zip(zmaps, outs):
            self._check_zmap(grid, precision, z)
            self._check_zmap(grid, precision, o)
        spec = _abi.FsmTextureSpec(lambda_s=float(lambda_s), lambda_c=float(lambda_c),
                                   trunc=float(trunc), level=1 if level else 0)
        zin = (C.c_void_p * n)(*[z.data_ptr() for z in zmaps])
        zout = (C.c_void_p * n)(*[o.data_ptr() for o in outs])
        res = (_abi.FsmRough * n)()
        planes = (C.c_double * (3 * n))()
        rc = self._lib.fsm_texture_batch(self._h, n, C.byref(_abi.grid_struct(grid)), _prec(precision),
                                         zin, zout, C.byref(spec), res, planes,
                                         C.c_void_p(_stream_handle(stream, self.device)))
        _check(rc, "fsm_texture_batch", self._h)
        return outs, [r.as_dict() for r in res], [tuple(planes[3 * k:3 * k + 3]) for k in range(n)]

    def fsm_simulate_batch(self, sims, precision="f64", zmaps=None, stream=None):
        """Run many simulations in one launch sequence; returns (Z-map tensors, roughness
        dicts), both in the order of `sims`."""
        n = len(sims)
        if n == 0:
            return [], []
        if zmaps is None:
            zmaps = [self.new_zmap(s.grid, precision) for s in sims]
        keep = []
        jobs = (_abi.FsmJob * n)()
        for k, (s, z) in enumerate(zip(sims, zmaps)):
            self._check_zmap(s.grid, precision, z)
            t, c, g = _abi.tool_struct(s.tool), _abi.cut_struct(s.cut), _abi.grid_struct(s.grid)
            keep += [t, c, g]
            jobs[k].tool = C.pointer(t)
            jobs[k].cut = C.pointer(c)
            jobs[k].grid = C.pointer(g)
            jobs[k].zmap_dev = z.data_ptr()
        out = (_abi.FsmRough * n)()
        rc = self._lib.fsm_simulate_batch(self._h, n, jobs, _prec(precision), out,
                                          C.c_void_p(_stream_handle(stream, self.device)))
        _check(rc, "fsm_simulate_batch", self._h)
        return list(zmaps), [o.as_dict() for o in out]

    def fsm_batch_submit(self, sims, precision="f64", zmaps=None, stream=None):
        """Queue many simulations as one asynchronous batch on a slot of the context; returns
        (batch id, Z-map tensors).  The tensors must stay alive until fsm_batch_wait.  Raises
        FsmError with code FSM_EAGAIN when no slot (or HBM budget) is free."""
        n = len(sims)
        if n == 0:
            raise ValueError("an asynchronous batch needs at least one simulation")
        if zmaps is None:
            zmaps = [self.new_zmap(s.grid, precision) for s in sims]
        keep = []
        jobs = (_abi.FsmJob * n)()
        for k, (s, z) in enumerate(zip(sims, zmaps)):
            self._check_zmap(s.grid, precision, z)
            t, c, g = _abi.tool_struct(s.tool), _abi.cut_struct(s.cut), _abi.grid_struct(s.grid)
            keep += [t, c, g]
            jobs[k].tool = C.pointer(t)
            jobs[k].cut = C.pointer(c)
            jobs[k].grid = C.pointer(g)
            jobs[k].zmap_dev = z.data_ptr()
        bid = C.c_uint64(0)
        rc = self._lib.fsm_batch_submit(self._h, n, jobs, _prec(precision),
                                        C.c_void_p(_stream_handle(stream, self.device)), C.byref(bid))
        _check(rc, "fsm_batch_submit", self._h)
        self._batches[bid.value] = n
        return bid.value, list(zmaps)

    def fsm_batch_poll(self, batch_id: int) -> bool:
        """Whether the batch has finished on the device."""
        done = C.c_int(0)
        _check(self._lib.fsm_batch_poll(self._h, C.c_uint64(batch_id), C.byref(done)),
               "fsm_batch_poll", self._h)
        return bool(done.value)

    def fsm_batch_wait(self, batch_id: int):
        """Wait for the batch and free its slot; returns its roughness dicts in job order."""
        n = self._batches.get(batch_id, 0)
        out = (_abi.FsmRough * n)() if n else None   # a batch not submitted here gets no records
        rc = self._lib.fsm_batch_wait(self._h, C.c_uint64(batch_id), out)
        _check(rc, "fsm_batch_wait", self._h)
        self._batches.pop(batch_id, None)
        return [out[k].as_dict() for k in range(n)]

    def fsm_serve_run(self, requests, precision="f32", n_slots=2, max_batch=16, realtime=True,
                      arena_bytes=None, slot_bytes=1 << 30):
        """Serve requests [(sim, arrival_s, zmap tensor or None), ...] to completion with
        continuous batching; returns one dict per request (roughness, status, batch, slot and
        admit/start/done times in seconds after the start).  Requests without a Z-map tensor
        are held in a device arena sized to the largest of them times n_slots * max_batch
        unless arena_bytes is given."""
        n = len(requests)
        if n == 0:
            return []
        key = 8 if _prec(precision) == _abi.F64 else 4
        if arena_bytes is None:
            own = [int(s.grid.nx) * int(s.grid.ny) * key for s, _, z in requests if z is None]
            arena_bytes = 0 if not own else min(sum(own), max(own) * n_slots * max_batch) + (1 << 20)
        cfg = _abi.FsmServeConfig(_prec(precision), n_slots, max_batch, 1 if realtime else 0,
                                  int(arena_bytes), int(slot_bytes))
        reqs, keep = _requests(requests, precision, self)
        out = (_abi.FsmRequestResult * n)()
        rc = self._lib.fsm_serve_run(self._h, C.byref(cfg), n, reqs, out)
        _check(rc, "fsm_serve_run", self._h)
        del keep
        return [_result(o) for o in out]

    def fsm_autotune(self, sims, precision="f64", zmaps=None, stream=None) -> dict:
        """Time candidate launch parameters on `sims` run as one batch and keep the fastest for
        their workload class (later calls of that class use them).  Returns the kept
        parameters with the best and the default timings (ms)."""
        n = len(sims)
        if zmaps is None:
            zmaps = [self.new_zmap(s.grid, precision) for s in sims]
        keep = []
        jobs = (_abi.FsmJob * n)()
        for k, (s, z) in enumerate(zip(sims, zmaps)):
            self._check_zmap(s.grid, precision, z)
            t, c, g = _abi.tool_struct(s.tool), _abi.cut_struct(s.cut), _abi.grid_struct(s.grid)
            keep += [t, c, g]
            jobs[k].tool, jobs[k].cut, jobs[k].grid = C.pointer(t), C.pointer(c), C.pointer(g)
            jobs[k].zmap_dev = z.data_ptr()
        out = _abi.FsmTuneResult()
        rc = self._lib.fsm_autotune(self._h, n, jobs, _prec(precision), C.byref(out),
                                    C.c_void_p(_stream_handle(stream, self.device)))
        _check(rc, "fsm_autotune", self._h)
        return {k: getattr(out, k) for k, _ in out._fields_}

    def fsm_tune_get(self) -> list:
        """The context's tuning table: [{key, strategy, tile_shape, target_rows}, ...]."""
        n = C.c_int(0)
        _check(self._lib.fsm_tune_get(self._h, None, 0, C.byref(n)), "fsm_tune_get", self._h)
        buf = (_abi.FsmTuneEntry * max(1, n.value))()
        _check(self._lib.fsm_tune_get(self._h, buf, n.value, C.byref(n)), "fsm_tune_get", self._h)
        return [{"key": e.key.decode(), "strategy": e.strategy, "tile_shape": e.tile_shape,
                 "target_rows": e.target_rows} for e in buf[:n.value]]

    def fsm_tune_set(self, entries):
        """Add entries (dicts as fsm_tune_get returns them) to the context's tuning table."""
        n = len(entries)
        buf = (_abi.FsmTuneEntry * max(1, n))()
        for k, e in enumerate(entries):
            buf[k].key = e["key"].encode()
            buf[k].strategy = int(e["strategy"])
            buf[k].tile_shape = int(e["tile_shape"])
            buf[k].target_rows = int(e["target_rows"])
        _check(self._lib.fsm_tune_set(self._h, buf, n), "fsm_tune_set", self._h)

    def load_tuning(self, path) -> int:
        """Load a saved tuning table (JSON written by paper_2603_28160_amd.tune)."""
        import json
        with open(path) as f:
            entries = json.load(f)["entries"]
        self.fsm_tune_set(entries)
        return len(entries)

    def set_graphs(self, on: bool = True):
        """Capture launch sequences into HIP graphs and replay them per launch shape."""
        self.fsm_ctx_set_option(_abi.OPT_GRAPHS, 1 if on else 0)

    # short aliases
    simulate = fsm_simulate
    roughness = fsm_roughness
    simulate_batch = fsm_simulate_batch
    serve = fsm_serve_run
    trajectory = fsm_trajectory
    autotune = fsm_autotune
