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

F32_TOL = 2e-6       # mm, height tolerance of a single-precision Z-map (the stated bar)
U32 = 2.0 ** -24     # unit roundoff of single precision


def f32_delta(sim):
    """Bound on the single-precision error of a workpiece-frame position, from an operation
    count.  The single-precision path rounds the tool-frame point and the spindle cos/sin to
    float and turns the point by Eq. (3), then by the lead and the side tilt, each coordinate
    with one product and one fused multiply-add per rotation.  Every intermediate is a
    coordinate of a rotated edge point, so no value exceeds R = the largest distance of an edge
    point from the tool origin, and each rounding errs by at most U32 * R.  Counting the
    roundings along the longest chain (the y coordinate after both tilts, which carries the z
    error of the lead tilt) gives 13 U32 R; 16 U32 R covers the second-order terms and the
    double-precision reference's own roundings.  The tool-centre offset is added in double."""
    _, pts = oracle.edge_points(sim)
    return 16.0 * U32 * float(np.sqrt((pts * pts).sum(axis=-1)).max())


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


def rough_bounds(Z, low, high, must_hit, must_miss, r):
    """Largest change of every roughness parameter over all maps Z' the intervals allow:
    cells that must be hit lie in [low, high], cells neither forced hit nor forced empty (the
    slack cells) may be empty or lie in [low, high], forced-empty cells stay empty.  Z is the
    oracle's map and r its roughness.

    With H the oracle's hit set (n cells, mean mu), removed cells Rm and added cells Ad:
      sum over H' of (z' - mu) = sum over the kept cells of (z' - z) - sum over Rm of (z - mu)
                                 + sum over Ad of (z' - mu),
    so |mean' - mu| <= B1 / n_lo, B1 bounding each cell's largest possible term and n_lo the
    fewest cells H' can have.  The same split bounds the sums of |d|, d^3 and d^4 (|a^k - b^k|
    <= k Rr^(k-1) |a - b| for |a|, |b| <= Rr), and the 2-norm of the centred vector changes by
    at most the 2-norm of the per-cell changes (Sq).  Extremes come from the intervals
    directly.  The profiles are bounded like Sa over their own line."""
    hit = np.isfinite(Z)
    n = int(hit.sum())
    out = {}
    if n == 0:
        return {k: math.inf for k in ("mean", "Sa", "Sq", "Sp", "Sv", "Sz", "Ssk", "Sku",
                                      "Ra_feed", "Ra_pick")}
    slack = ~must_hit & ~must_miss
    mu = r["mean"]
    with np.errstate(invalid="ignore"):
        w = np.where(hit, np.maximum(Z - low, high - Z), 0.0)
        dev = np.where(hit, np.abs(Z - mu), 0.0)
        ext = np.maximum(np.abs(low - mu), np.abs(high - mu))
    keep = hit & ~slack            # stays hit
    rem = hit & slack              # may be dropped
    add = ~hit & slack             # may be added
    n_lo = n - int(rem.sum())
    dn = max(int(rem.sum()), int(add.sum()))
    if n_lo <= 0:
        return {k: math.inf for k in ("mean", "Sa", "Sq", "Sp", "Sv", "Sz", "Ssk", "Sku",
                                      "Ra_feed", "Ra_pick")}
    b1 = float(w[keep].sum() + np.maximum(w[rem], dev[rem]).sum() + ext[add].sum())
    dmu = b1 / n_lo
    out["mean"] = dmu
    out["Sa"] = 2.0 * b1 / n_lo + r["Sa"] * dn / n_lo
    b2 = math.sqrt(float(((w[keep] + dmu) ** 2).sum()
                         + np.maximum((w[rem] + dmu) ** 2, dev[rem] ** 2).sum()
                         + ((ext[add] + dmu) ** 2).sum()))
    sq = r["Sq"]
    n_hi = n + int(add.sum())
    out["Sq"] = b2 / math.sqrt(n_lo) + sq * max(math.sqrt(n / n_lo) - 1.0, 1.0 - math.sqrt(n / n_hi))
    cand = hit | add
    rr = float(max(dev.max(), ext[cand].max())) + dmu
    for k, key in ((3, "Ssk"), (4, "Sku")):
        bk = float((k * rr ** (k - 1) * (w[keep] + dmu)).sum()
                   + np.maximum(k * rr ** (k - 1) * (w[rem] + dmu), dev[rem] ** k).sum()
                   + ((ext[add] + dmu) ** k).sum())
        sq_lo = sq - out["Sq"]
        if not sq > 0.0 or sq_lo <= 0.0 or math.isnan(r[key]):
            out[key] = math.inf
            continue
        mk = r[key] * sq ** k
        dmk = bk / n_lo + abs(mk) * dn / n_lo
        out[key] = dmk / sq_lo ** k + abs(mk) * (sq_lo ** -k - sq ** -k)
    zmax, zmin = float(Z[hit].max()), float(Z[hit].min())
    max_hi = float(high[cand].max())
    min_lo = float(low[cand].min())
    forced = must_hit
    max_lo = float(low[forced].max()) if forced.any() else -math.inf
    min_hi = float(high[forced].min()) if forced.any() else math.inf
    dmax = max(max_hi - zmax, zmax - max_lo)
    dmin = max(zmin - min_lo, min_hi - zmin)
    out["Sp"] = dmax + dmu
    out["Sv"] = dmin + dmu
    out["Sz"] = dmax + dmin
    ny, nx = Z.shape
    for key, sel in (("Ra_feed", (ny // 2, slice(None))), ("Ra_pick", (slice(None), nx // 2))):
        zl, lo_l, hi_l = Z[sel], low[sel], high[sel]
        mh, mm = must_hit[sel], must_miss[sel]
        hl = np.isfinite(zl)
        nl = int(hl.sum())
        if nl == 0 or math.isnan(r[key]):
            out[key] = math.inf
            continue
        ml = float(zl[hl].mean())
        sl = ~mh & ~mm
        with np.errstate(invalid="ignore"):
            wl = np.where(hl, np.maximum(zl - lo_l, hi_l - zl), 0.0)
            dl = np.where(hl, np.abs(zl - ml), 0.0)
            el = np.maximum(np.abs(lo_l - ml), np.abs(hi_l - ml))
        kl, rl, al = hl & ~sl, hl & sl, ~hl & sl
        nl_lo = nl - int(rl.sum())
        if nl_lo <= 0:
            out[key] = math.inf
            continue
        bl = float(wl[kl].sum() + np.maximum(wl[rl], dl[rl]).sum() + el[al].sum())
        out[key] = 2.0 * bl / nl_lo + r[key] * max(int(rl.sum()), int(al.sum())) / nl_lo
    return out
