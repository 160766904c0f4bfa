"""CPU pins of the single-precision acceptance bounds (oracle.cell_bounds and the moment
bounds), checked against independent facts rather than against themselves:

* with no position error the interval collapses onto the oracle's own Z-map;
* moving the grid origin by s moves every evaluation by -s relative to the cells, so the
  Z-map of a shifted grid is a valid "perturbed" result and must fall inside the intervals;
* the roughness of randomly perturbed maps (oracle.roughness, the plain definitions) must stay
  within the moment bounds.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2603_28160_amd import workloads as W

import f32_bounds as FB


def small_sim():
    # the path is pinned explicitly: an automatic path follows the grid when the grid moves
    s = W.config2(nx=61, ny=47, dd=0.01)
    p = oracle.plan(s)
    cut = dataclasses.replace(s.cut, steps_per_rev=180, x_start=p["x_start"],
                              y_first=p["y_first"], n_passes=p["n_passes"],
                              n_steps=p["n_steps"] * 180 // s.cut.steps_per_rev)
    return s.replace(cut=cut, tool=dataclasses.replace(s.tool, n_edge=24))


def test_zero_delta_collapses_to_zmap():
    s = small_sim()
    zo, _ = oracle.simulate(s)
    lo, hi, top = oracle.cell_bounds(s, 0.0)
    assert np.array_equal(lo, zo)
    assert np.array_equal(hi, zo)
    hit = np.isfinite(zo)
    assert np.all(top[hit] >= zo[hit])
    assert np.all(np.isneginf(top[~hit]))


@pytest.mark.parametrize("shift", [(0.9, 0.0), (-0.9, 0.5), (0.3, -0.9), (-0.7, -0.7)])
def test_shifted_grid_falls_inside_intervals(shift):
    s = small_sim()
    delta = 0.3 * s.grid.dd
    low, high, must_hit, must_miss = FB.f32_intervals(s, delta=delta, tol=0.0)
    g = s.grid
    moved = s.replace(grid=dataclasses.replace(g, x0=g.x0 + shift[0] * delta,
                                               y0=g.y0 + shift[1] * delta))
    zs, _ = oracle.simulate(moved)
    zo, _ = oracle.simulate(s)
    assert not np.array_equal(zs, zo)          # the shift changes cells: the check has teeth
    FB.check_cells(zs, low, high, must_hit, must_miss)


def test_intervals_reject_a_wrong_map():
    s = small_sim()
    low, high, must_hit, must_miss = FB.f32_intervals(s, delta=0.3 * s.grid.dd, tol=0.0)
    zo, _ = oracle.simulate(s)
    bad = zo.copy()
    k = np.argwhere(np.isfinite(zo))[len(zo) // 2]
    bad[tuple(k)] -= 0.01                       # deeper than any evaluation reaching the cell
    with pytest.raises(AssertionError):
        FB.check_cells(bad, low, high, must_hit, must_miss)


@pytest.mark.parametrize("seed", range(6))
def test_moment_bounds_hold_for_perturbed_maps(seed):
    rng = np.random.default_rng([28160, 77, seed])
    ny, nx = 37, 53
    Z = rng.normal(0.0, 0.01, (ny, nx)) + 0.004 * np.sin(np.arange(nx) / 3.0)[None, :]
    Z[rng.random((ny, nx)) < 0.05] = np.inf
    w = rng.uniform(0.0, 2e-3, (ny, nx)) * (rng.random((ny, nx)) < 0.3)
    r = oracle.roughness(Z)
    b = FB.moment_bounds(Z, w, r)
    for trial in range(20):
        u = rng.choice([-1.0, 1.0], (ny, nx)) if trial % 2 else rng.uniform(-1, 1, (ny, nx))
        Zp = np.where(np.isfinite(Z), Z + w * u, np.inf)
        rp = oracle.roughness(Zp)
        for k, bound in b.items():
            assert abs(rp[k] - r[k]) <= bound * (1 + 1e-12) + 1e-15, (k, rp[k], r[k], bound)


def test_moment_bounds_are_tight_for_a_shift():
    # a uniform shift by c moves the mean by exactly c and leaves the centred parameters alone
    rng = np.random.default_rng([28160, 78])
    Z = rng.normal(0.0, 0.01, (20, 30))
    w = np.full(Z.shape, 1e-3)
    r = oracle.roughness(Z)
    b = FB.moment_bounds(Z, w, r)
    rp = oracle.roughness(Z + 1e-3)
    assert abs(rp["mean"] - r["mean"]) == pytest.approx(b["mean"], rel=1e-9)
    assert abs(rp["Sq"] - r["Sq"]) <= 1e-15


def test_window_equals_full_grid_slice():
    s = small_sim()
    delta = 0.3 * s.grid.dd
    full = oracle.cell_bounds(s, delta)
    win = oracle.cell_bounds(s, delta, window=(7, 40, 5, 31))
    for a, b in zip(full, win):
        assert np.array_equal(a[5:31, 7:40], b)
