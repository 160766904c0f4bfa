"""GPU parity: libfsm (HIP, through the C ABI) against the FP64 CPU oracle.

Double precision: identical hit masks, identical heights (|dZ| <= 1e-9 mm is the stated bar;
the kernels reproduce the oracle's arithmetic, so the test demands equality), identical
in-grid counts, roughness within 1e-4 relative.
Single precision: every cell inside the oracle's interval for a position error of a few ulps
and a height error of 2e-6 mm (f32_bounds); where no evaluation lies that close to a cell
boundary the interval is the double-precision height +- 2e-6 mm.  Roughness within 1e-4
relative plus the largest change the interval widths allow.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from paper_2603_28160_amd import workloads as W

import f32_bounds as FB

pytestmark = pytest.mark.gpu

ROUGH_KEYS = ("Sa", "Sq", "Sp", "Sv", "Sz", "Ssk", "Sku", "Ra_feed", "Ra_pick", "mean")
ROUGH_RTOL = 1e-4


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_28160_amd import Context
    c = Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module", params=["binned", "scatter"])
def sctx(request):
    """A context per Z-map strategy."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_28160_amd import Context
    c = Context(0)
    c.set_strategy(request.param)
    yield c
    c.close()


def run_gpu(ctx, sim, precision):
    print(f"[gpu] {sim.name or 'sim'} {precision} grid {sim.grid.nx}x{sim.grid.ny}", flush=True)
    z, r = ctx.fsm_simulate(sim, precision)
    return z.cpu().numpy().astype(np.float64), r


def check_rough(rg, ro, rtol=ROUGH_RTOL, abs_floor=1e-12):
    assert rg["n_hit"] == ro["n_hit"]
    assert rg["n_feed"] == ro["n_feed"] and rg["n_pick"] == ro["n_pick"]
    for k in ROUGH_KEYS:
        a, b = rg[k], ro[k]
        if math.isnan(b):
            assert math.isnan(a), k
        else:
            assert abs(a - b) <= rtol * abs(b) + abs_floor, (k, a, b)


def check_f64(ctx, sim):
    zg, rg = run_gpu(ctx, sim, "f64")
    zo, cnt = oracle.simulate(sim)
    assert rg["n_evals"] == cnt["n_evals"]
    assert rg["n_binned"] == cnt["n_binned"]
    assert np.array_equal(np.isfinite(zg), np.isfinite(zo))
    assert np.array_equal(zg, zo), float(np.nanmax(np.abs(np.where(np.isfinite(zo), zg - zo, 0))))
    check_rough(rg, oracle.roughness(zo))
    return zo


def check_f32(ctx, sim, zo=None, max_open=0.05, areal_bar=False):
    """Single precision against the oracle: every cell inside its interval, the library's own
    error statement (pos_err, n_near) consistent with the oracle's map, and every roughness
    parameter within 1e-4 relative plus the largest change the intervals allow (hit-state
    changes of the slack cells included).  Returns the map and the measured errors."""
    zg, rg = run_gpu(ctx, sim, "f32")
    if zo is None:
        zo, _ = oracle.simulate(sim)
    low, high, must_hit, must_miss = FB.f32_intervals(sim)
    # the interval is wide only where an evaluation lies near a cell boundary
    open_ = high - low > 2 * FB.F32_TOL + 1e-15
    assert open_.mean() <= max_open, open_.mean()
    FB.check_cells(zg, low, high, must_hit, must_miss)
    # the library's statement: its position bound is the operation-count bound, and a cell
    # differs from double precision by more than that only where a near-boundary evaluation
    # changed its cell (each such evaluation touches two cells)
    assert rg["pos_err"] == pytest.approx(FB.f32_delta(sim), rel=1e-12)
    hg, ho = np.isfinite(zg), np.isfinite(zo)
    with np.errstate(invalid="ignore"):
        moved = (hg != ho) | (hg & ho & (np.abs(zg - zo) > rg["pos_err"]))
    assert int(moved.sum()) <= 2 * rg["n_near"], (int(moved.sum()), rg["n_near"])
    assert rg["n_near"] <= rg["n_binned"]
    ro = oracle.roughness(zo)
    slack = np.sum(ho & ~must_hit) + np.sum(~ho & ~must_miss)
    assert abs(rg["n_hit"] - ro["n_hit"]) <= slack
    err = {"cells_moved": int(moved.sum()), "n_near": rg["n_near"], "open": float(open_.mean())}
    if ro["n_hit"] > 0:
        rb = FB.rough_bounds(zo, low, high, must_hit, must_miss, ro)
        for k in ("Sa", "Sq", "Sp", "Sv", "Sz", "Ssk", "Sku", "Ra_feed", "Ra_pick", "mean"):
            if math.isnan(ro[k]):
                continue
            e = abs(rg[k] - ro[k])
            err[k] = e / abs(ro[k]) if ro[k] else e
            assert e <= ROUGH_RTOL * abs(ro[k]) + rb[k] + 1e-12, (k, rg[k], ro[k], rb[k])
    if areal_bar:
        # the areal parameters average over every hit cell: the few cells a near-boundary
        # evaluation moves leave them inside the stated bar itself (a profile line has too
        # few cells for that and keeps the interval bound above)
        for k in ("Sa", "Sq", "Ssk", "Sku", "Sp", "Sv", "Sz", "mean"):
            assert abs(rg[k] - ro[k]) <= ROUGH_RTOL * abs(ro[k]), (k, rg[k], ro[k])
    print(f"[f32 vs oracle] {sim.name or 'sim'}: " +
          ", ".join(f"{k}={v:.3g}" if isinstance(v, float) else f"{k}={v}" for k, v in err.items()),
          flush=True)
    return zg, err


# --- double precision: bit-exact against the oracle ----------------------------------------

def test_config1_f64_exact(sctx):
    check_f64(sctx, W.config1())


def test_config2_reduced_f64_exact(sctx):
    # same tool and path rules as the 5000 x 5000 case on a ragged 777 x 613 grid
    check_f64(sctx, W.config2(nx=777, ny=613, dd=0.004))


@pytest.mark.parametrize("i", [0, 1, 2, 3, 5, 8])
def test_mix_sims_f64_exact(sctx, i):
    s = W.random_sim(3, i, side_max=300)
    s = s.replace(grid=dataclasses.replace(s.grid, dd=s.grid.dd * 4))
    check_f64(sctx, s)


def test_binned_slices_f64_exact(ctx):
    # a 1 MiB bucket budget forces the evaluation range into many slices, each folding its
    # tiles into the Z-map left by the previous one
    from paper_2603_28160_amd import _abi
    s = W.config2(nx=777, ny=613, dd=0.004)
    ctx.fsm_ctx_set_option(_abi.OPT_BUCKET_BYTES, 1 << 20)
    try:
        check_f64(ctx, s)
        check_f32(ctx, s)
    finally:
        ctx.fsm_ctx_set_option(_abi.OPT_BUCKET_BYTES, 2 << 30)


@pytest.mark.parametrize("shape", [0x77, 0x87])
def test_large_tiles_exact(ctx, shape):
    # tiles of 128 KiB (FP64 128 x 128, FP32 256 x 128): the reduction runs with eight waves
    # per block; the double-precision map stays bit-exact and the single one inside its bounds
    # (a shape too large for a precision falls back to that precision's default)
    from paper_2603_28160_amd import _abi
    s = W.config2(nx=777, ny=613, dd=0.004)
    ctx.fsm_ctx_set_option(_abi.OPT_AUTOTUNED, 0)
    try:
        ctx.fsm_ctx_set_option(_abi.OPT_TILE_SHAPE, shape)
        check_f64(ctx, s)
        check_f32(ctx, s)
    finally:
        ctx.fsm_ctx_set_option(_abi.OPT_TILE_SHAPE, 0)
        ctx.fsm_ctx_set_option(_abi.OPT_AUTOTUNED, 1)


def test_binned_slices_aligned_rows_exact(ctx):
    # rows a whole number of 16-byte vectors long: the tile reduction fills and drains its
    # tiles in vectors, and later slices fold into the map read back in vectors
    from paper_2603_28160_amd import _abi
    s = W.config2(nx=800, ny=613, dd=0.004)
    ctx.fsm_ctx_set_option(_abi.OPT_BUCKET_BYTES, 1 << 20)
    try:
        check_f64(ctx, s)
        check_f32(ctx, s)
    finally:
        ctx.fsm_ctx_set_option(_abi.OPT_BUCKET_BYTES, 2 << 30)


def last_path(ctx):
    t = ctx.fsm_last_timings()
    return t["zmap_path"], t["n_slices"]


@pytest.mark.parametrize("budget", [0, 96 << 20])
def test_super_tiles_exact(ctx, budget):
    # 16 x 16-cell tiles over 2100 x 2050 cells: 132 x 129 = 17 028 tiles, more than one row
    # histogram holds, so the rows count per super-tile of 2 x 2 tiles (the last super-tile
    # row half outside the grid) and a split pass sorts each super-tile's bucket into its
    # tiles; with a 96 MiB bucket budget the rows also run in many slices, each folding its
    # tiles into the map of the one before
    from paper_2603_28160_amd import _abi
    s = W.config2(nx=2100, ny=2050, dd=0.002)
    ctx.fsm_ctx_set_option(_abi.OPT_AUTOTUNED, 0)
    ctx.fsm_ctx_set_option(_abi.OPT_TILE_SHAPE, 0x44)
    # 0: the default budget, which holds every evaluation of this grid in one slice
    ctx.fsm_ctx_set_option(_abi.OPT_BUCKET_BYTES, budget or 16 << 30)
    ctx.fsm_ctx_set_profiling(True)
    try:
        check_f64(ctx, s)
        path, slices = last_path(ctx)
        assert path == _abi.PATH_SUPER
        assert (slices > 1) == bool(budget), slices
        check_f32(ctx, s)
        assert last_path(ctx)[0] == _abi.PATH_SUPER
    finally:
        ctx.fsm_ctx_set_profiling(False)
        ctx.fsm_ctx_set_option(_abi.OPT_BUCKET_BYTES, 2 << 30)
        ctx.fsm_ctx_set_option(_abi.OPT_TILE_SHAPE, 0)
        ctx.fsm_ctx_set_option(_abi.OPT_AUTOTUNED, 1)


def test_run_mode_exact(ctx):
    # no room for a row matrix: the binned strategy counts and claims with global atomics
    # per tile (run mode), over several slices
    from paper_2603_28160_amd import _abi
    s = W.config2(nx=777, ny=613, dd=0.004)
    ctx.fsm_ctx_set_option(_abi.OPT_HIST_BYTES, 0)
    ctx.fsm_ctx_set_option(_abi.OPT_BUCKET_BYTES, 16 << 20)
    ctx.fsm_ctx_set_profiling(True)
    try:
        check_f64(ctx, s)
        path, slices = last_path(ctx)
        assert path == _abi.PATH_RUN and slices > 1, (path, slices)
        check_f32(ctx, s)
    finally:
        ctx.fsm_ctx_set_profiling(False)
        ctx.fsm_ctx_set_option(_abi.OPT_BUCKET_BYTES, 2 << 30)
        ctx.fsm_ctx_set_option(_abi.OPT_HIST_BYTES, 1 << 30)


def test_paper_case2_tool_f64_exact(ctx):
    # the paper's own face-milling tool with rake and per-insert runout (Sec. 4.2)
    t = W.paper_case2_tool(eps_r=-0.026, eps_a=0.009, n_edge=30)
    s = W.Sim(t, W.Cut(f_z=0.4, a_p=0.4, steps_per_rev=500, a_e=4.0),
              W.centred_grid(301, 157, 0.01), name="paper_case2")
    check_f64(ctx, s)


@pytest.mark.parametrize("case", ["n1", "z1", "s1", "grid1x1", "nofeed", "odd", "sidetilt", "big_n",
                                  "tile_edges"])
def test_edge_cases_f64(sctx, case):
    base = W.config2(nx=90, ny=70, dd=0.02)
    t, c, g = base.tool, base.cut, base.grid
    if case == "n1":
        t = dataclasses.replace(t, n_edge=1)
    elif case == "z1":
        t = dataclasses.replace(t, n_teeth=1)
    elif case == "s1":
        c = dataclasses.replace(c, steps_per_rev=1)
    elif case == "grid1x1":
        g = W.centred_grid(1, 1, 0.05)
    elif case == "nofeed":
        c = dataclasses.replace(c, f_z=0.0, a_e=0.0, n_passes=1, x_start=0.0, y_first=0.0)
    elif case == "odd":
        g = W.centred_grid(77, 3, 0.013)       # 231 cells: odd, not a multiple of 4
    elif case == "sidetilt":
        t = dataclasses.replace(t, tilt_side=math.radians(-7.0), theta=(0.0, 1.5, 3.2, 4.6))
    elif case == "big_n":
        t = dataclasses.replace(t, n_edge=300, n_teeth=2)
    elif case == "tile_edges":
        g = W.centred_grid(129, 65, 0.02)      # one cell past whole tiles in both directions
    check_f64(sctx, W.Sim(t, c, g, name=case))


def test_empty_result(sctx):
    ctx = sctx
    # the path never reaches the grid: every cell stays +inf and every parameter is NaN
    s = W.config1()
    s = s.replace(cut=dataclasses.replace(s.cut, y_first=50.0))
    zg, rg = run_gpu(ctx, s, "f64")
    assert np.all(np.isinf(zg)) and rg["n_hit"] == 0 and rg["n_binned"] == 0
    assert rg["flags"] & 2 and math.isnan(rg["Sa"]) and math.isnan(rg["Ra_feed"])


def test_deterministic(ctx):
    s = W.config2(nx=400, ny=300, dd=0.003)
    for prec in ("f64", "f32"):
        z1, r1 = ctx.fsm_simulate(s, prec)
        a = z1.cpu().numpy().copy()
        z2, r2 = ctx.fsm_simulate(s, prec)
        assert np.array_equal(a, z2.cpu().numpy())
        assert r1 == r2 or all((r1[k] == r2[k]) or (math.isnan(r1[k]) and math.isnan(r2[k])) for k in r1)


# --- single precision: tolerance against the oracle --------------------------------------------

def test_config2_reduced_f32(sctx):
    check_f32(sctx, W.config2(nx=777, ny=613, dd=0.004))


@pytest.mark.parametrize("i", [0, 2, 5])
def test_mix_sims_f32(ctx, i):
    s = W.random_sim(3, i, side_max=300)
    s = s.replace(grid=dataclasses.replace(s.grid, dd=s.grid.dd * 4))
    check_f32(ctx, s)


# --- roughness entry point on given surfaces ------------------------------------------------------

@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [(64, 4), (101, 37), (1, 1), (5, 3)])
def test_roughness_entry(ctx, prec, shape):
    import torch
    nx, ny = shape
    rng = np.random.default_rng(nx * 31 + ny)
    Z = rng.normal(0.01, 0.003, size=(ny, nx))
    Z[rng.uniform(size=Z.shape) < 0.2] = np.inf
    if prec == "f32":
        Z = Z.astype(np.float32).astype(np.float64)
    dt = torch.float64 if prec == "f64" else torch.float32
    zt = torch.tensor(Z, dtype=dt, device="cuda:0")
    g = W.Grid(0.0, 0.0, 0.001, nx, ny)
    rg = ctx.fsm_roughness(g, zt, prec)
    ro = oracle.roughness(Z)
    check_rough(rg, ro, rtol=1e-10)
    # the surface is left untouched
    assert np.array_equal(zt.cpu().numpy().astype(np.float64), Z)


@pytest.mark.parametrize("strategy", ["binned", "scatter"])
def test_many_tiles_roughness(ctx, strategy):
    # 16 x 16-cell tiles over 3001 x 2000 cells (23 500 tiles): the binned strategy reduces
    # them in groups of eight with one partial per group, the scatter strategy's first pass
    # and the roughness entry point keep one per tile; every path sums to the oracle's values
    import torch
    from paper_2603_28160_amd import _abi
    ctx.fsm_ctx_set_option(_abi.OPT_AUTOTUNED, 0)
    ctx.fsm_ctx_set_option(_abi.OPT_TILE_SHAPE, 0x44)
    ctx.set_strategy(strategy)
    try:
        s = W.config2(nx=3001, ny=2000, dd=0.002)
        zo = check_f64(ctx, s)
        rg = ctx.fsm_roughness(s.grid, torch.tensor(zo, device="cuda:0"), "f64")
        check_rough(rg, oracle.roughness(zo), rtol=1e-10)
    finally:
        ctx.set_strategy("binned")
        ctx.fsm_ctx_set_option(_abi.OPT_TILE_SHAPE, 0)
        ctx.fsm_ctx_set_option(_abi.OPT_AUTOTUNED, 1)


def test_roughness_sinusoid_closed_form(ctx):
    import torch
    A = 0.3
    Z = np.tile(A * np.sin(2 * np.pi * np.arange(64) / 8), (4, 1))
    r = ctx.fsm_roughness(W.Grid(0, 0, 1e-3, 64, 4), torch.tensor(Z, device="cuda:0"), "f64")
    assert r["Sq"] == pytest.approx(A / math.sqrt(2), rel=1e-12)
    assert r["Sku"] == pytest.approx(1.5, rel=1e-12)
    assert r["Sa"] == pytest.approx(A * (1 + math.sqrt(2)) / 4, rel=1e-12)


# --- full-size workloads ------------------------------------------------------------------------------

@pytest.mark.parametrize("params", ["default", "tuned"])
def test_config2_full_f64_exact(ctx, params):
    # the 5000 x 5000 ball-end raster with the default launch parameters, and exactly as the
    # benchmark runs it (the shipped tuning table loaded)
    import os
    from paper_2603_28160_amd import _abi
    if params == "tuned":
        path = os.path.join(os.path.dirname(_abi.__file__), "tuning_mi355x.json")
        assert ctx.load_tuning(path) > 0
    else:
        ctx.fsm_ctx_set_option(_abi.OPT_AUTOTUNED, 0)
    try:
        print(f"[gpu] config2 full size, {params} launch parameters", flush=True)
        zo = check_f64(ctx, W.config2())
        check_f32(ctx, W.config2(), zo=zo, areal_bar=True)
    finally:
        ctx.fsm_ctx_set_option(_abi.OPT_AUTOTUNED, 1)
