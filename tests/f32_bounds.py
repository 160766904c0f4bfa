"""Acceptance bounds for single-precision results, derived from the FP64 oracle.

A single-precision evaluation differs from the double-precision one by a small position error
(at most `f32_delta(sim)` along x and y) and a small height error (at most F32_TOL).  The
oracle's per-cell interval (oracle.cell_bounds) then bounds every cell of a correct
single-precision Z-map, and the interval widths bound how far the areal parameters may move.
Nothing here reads a GPU result to set a bound.
"""
import math

import numpy as np

import oracle

F32_TOL = 2e-6       # mm, height error of a single-precision evaluation


def f32_delta(sim):
    """Bound on the single-precision error of a workpiece-frame position: a few ulps of the
    largest tool-local coordinate (the tool-centre offset is split off in double precision)."""
    pl = oracle.plan(sim)
    return 16.0 * 2.0 ** -24 * (pl["r_reach"] + sim.cut.a_p + 1.0)


def f32_intervals(sim, delta=None, tol=F32_TOL, window=None):
    """Per-cell acceptance interval [low, high] (mm), the cells that must be hit and the cells
    that must stay empty, for a single-precision Z-map of `sim` (or its cell window
    (i0, i1, j0, j1))."""
    lo, hi, top = oracle.cell_bounds(sim, f32_delta(sim) if delta is None else delta, window)
    must_hit = np.isfinite(hi)
    must_miss = ~np.isfinite(lo)
    low = lo - tol
    high = np.minimum(hi, top) + tol
    return low, high, must_hit, must_miss


def check_cells(zg, low, high, must_hit, must_miss):
    """Every hit cell inside its interval; hit/empty where the interval forces it."""
    hit = np.isfinite(zg)
    assert not np.any(must_hit & ~hit), int(np.sum(must_hit & ~hit))
    assert not np.any(must_miss & hit), int(np.sum(must_miss & hit))
    bad = hit & ((zg < low) | (zg > high))
    assert not np.any(bad), (int(bad.sum()), np.argwhere(bad)[:5].tolist())


def moment_bounds(Z, w, r):
    """Largest change of the areal parameters of Z (oracle roughness r) when every hit cell c
    moves by at most w[c] and the set of hit cells stays the same.

    Centring is an orthogonal projection: it never lengthens the perturbation in the 2-norm
    and at most doubles it in the 1-norm.  Hence |dmean| <= |w|_1/n, |dSq| <= |w|_2/sqrt(n),
    |dSa| <= 2|w|_1/n; for the third and fourth central moments |a^k - b^k| <= k R^(k-1) |a - b|
    with R bounding every centred value of either map (the range Sz grown by 2 max w)."""
    hit = np.isfinite(Z)
    n = int(hit.sum())
    wv = np.asarray(w, dtype=np.float64)[hit]
    l1 = float(wv.sum()) / n
    l2 = math.sqrt(float((wv * wv).sum()) / n)
    out = {"mean": l1, "Sq": l2, "Sa": 2.0 * l1}
    R = r["Sz"] + 2.0 * float(wv.max(initial=0.0))
    sq = r["Sq"]
    sq_lo = sq - l2
    if sq_lo <= 0.0:
        out["Ssk"] = out["Sku"] = math.inf
        return out
    m3 = r["Ssk"] * sq ** 3
    m4 = r["Sku"] * sq ** 4
    dm3 = 3.0 * R * R * 2.0 * l1
    dm4 = 4.0 * R ** 3 * 2.0 * l1
    # |m'/s'^k - m/s^k| <= |m' - m|/s_lo^k + |m| (1/s_lo^k - 1/s^k)
    out["Ssk"] = dm3 / sq_lo ** 3 + abs(m3) * (sq_lo ** -3 - sq ** -3)
    out["Sku"] = dm4 / sq_lo ** 4 + abs(m4) * (sq_lo ** -4 - sq ** -4)
    return out


def interval_widths(Z, low, high):
    """Per-cell bound on |Z' - Z| for any Z' inside [low, high] (zero off the hit cells)."""
    with np.errstate(invalid="ignore"):
        w = np.maximum(Z - low, high - Z)
    return np.where(np.isfinite(Z) & np.isfinite(w), w, 0.0)
