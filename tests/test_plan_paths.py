"""The Z-map path and slicing the library's planner picks with a fresh context's launch
parameters (fsm_plan, host only): maps whose tiles fit one row histogram take the histogram
mode, larger ones count per super-tile, and only maps whose super-tiles still overflow a
histogram fall back to run mode.  The thresholds follow from the default tiles (64 x 64 cells
in double precision, 128 x 64 in single), 16 384 counters per histogram and super-tiles of at
most 64 tiles."""
import dataclasses
import math

import pytest

from paper_2603_28160_amd import _abi, fsm_plan, workloads as W


def with_grid(sim, n, dd=None):
    g = dataclasses.replace(sim.grid, nx=n, ny=n, dd=dd or sim.grid.dd)
    return dataclasses.replace(sim, grid=g)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_benchmark_fields(prec):
    p2 = fsm_plan(W.config2(), prec)
    assert p2["zmap_path"] == _abi.PATH_HIST and p2["n_slices"] == 1
    p5 = fsm_plan(W.config5(), prec)
    # 40 000^2 cells are 390 625 (FP64) or 195 313 (FP32) tiles: super-tiles, one slice
    assert p5["zmap_path"] == _abi.PATH_SUPER and p5["n_slices"] == 1


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_thresholds(prec):
    sx, sy = (6, 6) if prec == "f64" else (7, 6)
    base = W.config2()

    def tiles(n):
        return math.ceil(n / 2 ** sx) * math.ceil(n / 2 ** sy)

    # the largest square grid whose tiles fit one histogram, and the next one up
    n = max(k for k in range(64, 20000, 64) if tiles(k) <= 16384)
    assert fsm_plan(with_grid(base, n), prec)["zmap_path"] == _abi.PATH_HIST
    assert fsm_plan(with_grid(base, n + 64), prec)["zmap_path"] == _abi.PATH_SUPER
    # super-tiles of 64 tiles hold up to 64 * 16 384 tiles; beyond that, run mode
    big = with_grid(base, 160000, dd=0.001)
    assert tiles(160000) > 64 * 16384
    assert fsm_plan(big, prec)["zmap_path"] == _abi.PATH_RUN


def test_slices_follow_the_bucket_worst_case():
    # a simulation whose every evaluation could land in the grid needs more bucket bytes than
    # the 16 GiB default holds once its evaluations exceed about 1.6e9 (FP64 histogram mode,
    # 10 bytes per point): it runs in slices
    s = W.config2()
    p = fsm_plan(s, "f64")
    assert p["n_evals"] * 10 < 16 << 30 and p["n_slices"] == 1
    fine = dataclasses.replace(s, cut=dataclasses.replace(s.cut, steps_per_rev=s.cut.steps_per_rev * 10))
    q = fsm_plan(fine, "f64")
    assert q["n_evals"] * 10 > 16 << 30
    assert q["zmap_path"] == _abi.PATH_HIST and q["n_slices"] >= 2
