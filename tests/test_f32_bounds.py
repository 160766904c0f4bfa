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


ROUGH_KEYS = ("mean", "Sa", "Sq", "Sp", "Sv", "Sz", "Ssk", "Sku", "Ra_feed", "Ra_pick")


def random_intervals(rng, ny, nx, p_slack):
    """An oracle-like map with per-cell intervals, some cells forced hit, some forced empty
    and a fraction p_slack whose hit state is open (empty in the oracle or not)."""
    Z = rng.normal(-0.2, 0.05, (ny, nx)) + 0.01 * np.sin(np.arange(nx) / 4.0)[None, :]
    empty = rng.random((ny, nx)) < 0.15
    Z[empty] = np.inf
    slack = rng.random((ny, nx)) < p_slack
    w = rng.uniform(0.0, 2e-3, (ny, nx)) * (rng.random((ny, nx)) < 0.3)
    centre = np.where(empty, rng.normal(-0.2, 0.05, (ny, nx)), Z)
    low = centre - w - rng.uniform(0, 1e-4, (ny, nx))
    high = centre + w + rng.uniform(0, 1e-4, (ny, nx))
    must_hit = ~empty & ~slack
    must_miss = empty & ~slack
    return Z, low, high, must_hit, must_miss


def allowed_map(rng, Z, low, high, must_hit, must_miss):
    """A map the intervals allow: forced cells as forced, slack cells hit or empty at random,
    every hit cell at a random height of its interval (often at an end)."""
    slack = ~must_hit & ~must_miss
    hit = must_hit | (slack & (rng.random(Z.shape) < 0.5))
    t = rng.uniform(0, 1, Z.shape)
    t = np.where(rng.random(Z.shape) < 0.5, np.round(t), t)
    return np.where(hit, low + t * (high - low), np.inf)


@pytest.mark.parametrize("seed", range(6))
def test_rough_bounds_hold_with_hit_state_changes(seed):
    rng = np.random.default_rng([28160, 79, seed])
    Z, low, high, mh, mm = random_intervals(rng, 41, 57, p_slack=[0.0, 0.01, 0.05][seed % 3])
    r = oracle.roughness(Z)
    b = FB.rough_bounds(Z, low, high, mh, mm, r)
    for trial in range(30):
        Zp = allowed_map(rng, Z, low, high, mh, mm)
        rp = oracle.roughness(Zp)
        for k in ROUGH_KEYS:
            assert abs(rp[k] - r[k]) <= b[k] * (1 + 1e-12) + 1e-15, (k, rp[k], r[k], b[k])


def test_rough_bounds_cover_a_dropped_extreme_cell():
    # dropping the highest cell (a slack cell) moves Sp by the gap to the next one: the bound
    # must reach that far, which a bound over fixed hit sets does not
    Z = np.full((5, 6), -0.3)
    Z[2, 3] = -0.1
    low, high = Z - 1e-6, Z + 1e-6
    mh = np.isfinite(Z)
    mh[2, 3] = False
    mm = np.zeros_like(mh)
    r = oracle.roughness(Z)
    b = FB.rough_bounds(Z, low, high, mh, mm, r)
    Zp = Z.copy()
    Zp[2, 3] = np.inf
    rp = oracle.roughness(Zp)
    for k in ("mean", "Sa", "Sq", "Sp", "Sz"):
        assert abs(rp[k] - r[k]) <= b[k], k
    assert abs(rp["Sp"] - r["Sp"]) > 0.1
    mb = FB.moment_bounds(Z, FB.interval_widths(Z, low, high), r)
    assert abs(rp["Sa"] - r["Sa"]) > mb["Sa"]


@pytest.mark.parametrize("shift", [(0.9, 0.0), (-0.7, -0.7)])
def test_shifted_grid_roughness_inside_rough_bounds(shift):
    # a grid moved by less than the position error is an allowed result, hit-state changes
    # included: its roughness must lie inside the bounds of the unmoved grid's intervals
    s = small_sim()
    s = s.replace(grid=dataclasses.replace(s.grid, dd=0.003))   # 79 % coverage
    delta = 0.3 * s.grid.dd
    low, high, mh, mm = FB.f32_intervals(s, delta=delta, tol=0.0)
    g = s.grid
    moved = s.replace(grid=dataclasses.replace(g, x0=g.x0 + shift[0] * delta,
                                               y0=g.y0 + shift[1] * delta))
    zs, _ = oracle.simulate(moved)
    zo, _ = oracle.simulate(s)
    assert not np.array_equal(np.isfinite(zs), np.isfinite(zo))   # hit states do change
    r = oracle.roughness(zo)
    b = FB.rough_bounds(zo, low, high, mh, mm, r)
    rs = oracle.roughness(zs)
    for k in ROUGH_KEYS:
        assert abs(rs[k] - r[k]) <= b[k] * (1 + 1e-12) + 1e-15, (k, rs[k], r[k], b[k])


def test_f32_delta_from_operation_count():
    # 16 single-precision rounding units of the farthest edge point from the tool origin
    s = W.config2()
    _, pts = oracle.edge_points(s)
    R = float(np.max(np.linalg.norm(pts, axis=-1)))
    assert FB.f32_delta(s) == 16.0 * 2.0 ** -24 * R
    assert 2.0 < R < 3.1                      # ball R3: points on the engaged meridian
