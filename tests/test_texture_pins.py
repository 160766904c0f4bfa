"""Pins of the oracle's surface-texture operators (the F-operator plane and the areal Gaussian
S-/L-filter of the measurement practice in Sec. 4.1.1), checked against what mathematics fixes:
exact planes and moment-free patterns, orthogonality of least-squares residuals, the Gaussian
filter's defining 50 % transmission at the cut-off wavelength, its transmission at other
wavelengths, invariance of constants and planes, holes, symmetry under mirroring and
transposition, linearity, and scipy's Gaussian filter on the interior.  CPU only."""
import math

import numpy as np
import pytest

import oracle
from paper_2603_28160_amd import workloads as W


def grid(nx, ny, dd, x0=0.0, y0=0.0):
    return W.Grid(x0=x0, y0=y0, dd=dd, nx=nx, ny=ny)


def nodes(g):
    x = g.x0 + np.arange(g.nx) * g.dd
    y = g.y0 + np.arange(g.ny) * g.dd
    return np.meshgrid(x, y)


# --- F-operator: least-squares plane ---------------------------------------------------------

def test_level_removes_an_exact_plane():
    g = grid(37, 23, 0.01, x0=-0.2, y0=0.3)
    X, Y = nodes(g)
    Z = 0.013 - 0.4 * X + 0.07 * Y
    out, c = oracle.level(Z, g)
    assert np.allclose(c, (0.013, -0.4, 0.07), rtol=0, atol=1e-13)
    assert np.abs(out).max() < 1e-14


def test_level_keeps_a_pattern_without_first_moments():
    # a checkerboard on an even grid has zero sum and zero x- and y-moments: the fitted plane
    # is exactly the added one and the residual is the checkerboard
    g = grid(40, 30, 0.005)
    X, Y = nodes(g)
    J, I = np.mgrid[0:g.ny, 0:g.nx]
    pat = 0.002 * (-1.0) ** (I + J)
    out, c = oracle.level(pat + 0.5 + 0.1 * X - 0.3 * Y, g)
    assert np.allclose(c, (0.5, 0.1, -0.3), rtol=0, atol=1e-13)
    assert np.allclose(out, pat, rtol=0, atol=1e-14)


def test_level_residual_is_orthogonal_and_matches_lstsq():
    rng = np.random.default_rng(5)
    g = grid(50, 41, 0.002, x0=1.0, y0=-0.5)
    X, Y = nodes(g)
    Z = rng.normal(0.0, 1e-3, (g.ny, g.nx)) + 0.02 * X
    Z[rng.random(Z.shape) < 0.3] = np.inf            # holes are ignored
    out, c = oracle.level(Z, g)
    hit = np.isfinite(Z)
    assert np.array_equal(np.isfinite(out), hit)
    r = out[hit]
    for m in (np.ones_like(r), X[hit], Y[hit]):
        assert abs(np.dot(m, r)) < 1e-12 * np.sqrt(len(r))
    A = np.stack([np.ones(hit.sum()), X[hit], Y[hit]], axis=1)
    ref = np.linalg.lstsq(A, Z[hit], rcond=None)[0]
    assert np.allclose(c, ref, rtol=1e-9, atol=1e-12)


def test_level_rejects_degenerate_hit_sets():
    g = grid(10, 10, 0.01)
    Z = np.full((10, 10), np.inf)
    Z[4, :] = 1.0                                    # one row: the y slope is undetermined
    with pytest.raises(ValueError):
        oracle.level(Z, g)
    Z[:] = np.inf
    Z[0, 0] = Z[3, 3] = 0.0
    with pytest.raises(ValueError):
        oracle.level(Z, g)


# --- areal Gaussian filter ---------------------------------------------------------------------

ALPHA = math.sqrt(math.log(2.0) / math.pi)


def transmission_x(lam, cutoff, dd=0.002, trunc=1.0, highpass=False):
    """Amplitude ratio of a cosine of wavelength lam along x after the filter, measured in the
    interior where the whole window lies in the grid."""
    R = int(math.floor(trunc * cutoff / dd + 1e-9))
    nx = 2 * R + int(round(2 * lam / dd)) + 1
    g = grid(nx, 2 * R + 3, dd)
    X, _ = nodes(g)
    Z = np.cos(2 * math.pi * X / lam)
    out = oracle.gauss_filter(Z, g, cutoff, trunc, highpass=highpass)
    mid = g.ny // 2
    # a cosine through a symmetric filter stays a cosine of the same phase: ratio at the peaks
    i0 = R + int(np.argmax(Z[mid, R:nx - R]))
    return out[mid, i0] / Z[mid, i0]


@pytest.mark.parametrize("ratio", [1.0, 2.0, 0.5])
def test_gaussian_transmission(ratio):
    # the weighting function's spectrum is exp(-pi (alpha cutoff / lam)^2): 50 % at the cut-off
    cutoff = 0.08
    lam = ratio * cutoff
    want = math.exp(-math.pi * (ALPHA * cutoff / lam) ** 2)
    if ratio == 1.0:
        assert want == pytest.approx(0.5, abs=1e-15)
    got = transmission_x(lam, cutoff)
    assert got == pytest.approx(want, abs=2e-5)
    assert transmission_x(lam, cutoff, highpass=True) == pytest.approx(1.0 - want, abs=2e-5)


def test_gaussian_acts_on_each_axis_by_its_own_wavelength():
    # z = cos(2 pi x / l1) + cos(2 pi y / l2): each term keeps its own transmission
    cutoff, dd = 0.05, 0.0025
    R = int(math.floor(cutoff / dd + 1e-9))
    l1, l2 = 0.1, 0.05
    g = grid(2 * R + 81, 2 * R + 61, dd)
    X, Y = nodes(g)
    Z = np.cos(2 * math.pi * X / l1) + np.cos(2 * math.pi * Y / l2)
    out = oracle.gauss_filter(Z, g, cutoff)
    t1 = math.exp(-math.pi * (ALPHA * cutoff / l1) ** 2)
    t2 = math.exp(-math.pi * (ALPHA * cutoff / l2) ** 2)
    want = t1 * np.cos(2 * math.pi * X / l1) + t2 * np.cos(2 * math.pi * Y / l2)
    inner = (slice(R, g.ny - R), slice(R, g.nx - R))
    assert np.abs(out[inner] - want[inner]).max() < 5e-5


def test_gaussian_keeps_constants_and_interior_planes():
    g = grid(60, 45, 0.01)
    X, Y = nodes(g)
    c = np.full((g.ny, g.nx), -0.25)
    assert np.abs(oracle.gauss_filter(c, g, 0.08) + 0.25).max() < 1e-14
    assert np.abs(oracle.gauss_filter(c, g, 0.08, highpass=True)).max() < 1e-14
    P = 0.1 + 0.3 * X - 0.2 * Y
    out = oracle.gauss_filter(P, g, 0.08)
    R = 8
    inner = (slice(R, g.ny - R), slice(R, g.nx - R))
    assert np.abs(out[inner] - P[inner]).max() < 1e-14
    # near the border the window is one-sided: the mean there is no longer the plane
    assert abs(out[0, 0] - P[0, 0]) > 5e-4


def test_gaussian_ignores_holes_and_keeps_them():
    rng = np.random.default_rng(9)
    g = grid(40, 40, 0.01)
    Z = np.full((40, 40), 0.7)
    holes = rng.random(Z.shape) < 0.2
    Z[holes] = np.inf
    for hp, want in ((False, 0.7), (True, 0.0)):
        out = oracle.gauss_filter(Z, g, 0.1, highpass=hp)
        assert np.array_equal(np.isinf(out), holes)
        assert np.abs(out[~holes] - want).max() < 1e-14


def test_gaussian_interior_equals_scipy():
    ndimage = pytest.importorskip("scipy.ndimage")
    rng = np.random.default_rng(3)
    dd, cutoff = 0.004, 0.05
    R = int(math.floor(cutoff / dd + 1e-9))
    g = grid(70, 52, dd)
    Z = rng.normal(0.0, 1.0, (g.ny, g.nx))
    out = oracle.gauss_filter(Z, g, cutoff)
    # exp(-pi r^2 / (alpha cutoff)^2) is the normal density of sigma = alpha cutoff / sqrt(2 pi)
    sigma = ALPHA * cutoff / math.sqrt(2 * math.pi) / dd
    ref = ndimage.gaussian_filter(Z, sigma, truncate=R / sigma, mode="constant")
    inner = (slice(R, g.ny - R), slice(R, g.nx - R))
    assert np.abs(out[inner] - ref[inner]).max() < 1e-13


def test_gaussian_commutes_with_flips_and_transposition():
    # symmetric weights, renormalised over the hit cells of a square window: mirroring the map
    # (holes included) mirrors the result, and so does swapping the axes
    rng = np.random.default_rng(12)
    g = grid(37, 23, 0.01)
    Z = rng.normal(size=(g.ny, g.nx))
    Z[rng.random(Z.shape) < 0.15] = np.inf
    for hp in (False, True):
        out = oracle.gauss_filter(Z, g, 0.06, highpass=hp)
        pairs = ((oracle.gauss_filter(Z[:, ::-1], g, 0.06, highpass=hp), out[:, ::-1]),
                 (oracle.gauss_filter(Z[::-1, :], g, 0.06, highpass=hp), out[::-1, :]),
                 (oracle.gauss_filter(Z.T, grid(g.ny, g.nx, g.dd), 0.06, highpass=hp), out.T))
        for a, b in pairs:
            assert np.array_equal(np.isinf(a), np.isinf(b))
            m = np.isfinite(b)
            assert np.abs(a[m] - b[m]).max() < 1e-13


def test_gaussian_is_linear_for_one_hole_set():
    rng = np.random.default_rng(13)
    g = grid(31, 26, 0.01)
    holes = rng.random((g.ny, g.nx)) < 0.1
    Z1, Z2 = rng.normal(size=(2, g.ny, g.nx))
    mix = 2.5 * Z1 - 0.75 * Z2
    for Z in (Z1, Z2, mix):
        Z[holes] = np.inf
    for hp in (False, True):
        lhs = oracle.gauss_filter(mix, g, 0.05, highpass=hp)
        f1, f2 = (oracle.gauss_filter(Z, g, 0.05, highpass=hp)[~holes] for Z in (Z1, Z2))
        assert np.array_equal(np.isinf(lhs), holes)
        assert np.abs(lhs[~holes] - (2.5 * f1 - 0.75 * f2)).max() < 1e-13


def test_level_residual_ignores_an_added_plane():
    # the least-squares residual of Z + plane is that of Z, and the fitted plane moves by it
    rng = np.random.default_rng(14)
    g = grid(25, 19, 0.02, x0=-0.3, y0=0.1)
    X, Y = nodes(g)
    Z = rng.normal(0.0, 0.01, (g.ny, g.nx))
    Z[rng.random(Z.shape) < 0.2] = np.inf
    r0, c0 = oracle.level(Z, g)
    r1, c1 = oracle.level(Z + (0.4 - 0.7 * X + 0.2 * Y), g)
    m = np.isfinite(Z)
    assert np.array_equal(np.isfinite(r1), m)
    assert np.abs(r1[m] - r0[m]).max() < 1e-13
    np.testing.assert_allclose(np.subtract(c1, c0), [0.4, -0.7, 0.2], atol=1e-12)


def test_gaussian_cells_variant_and_zero_radius():
    rng = np.random.default_rng(4)
    g = grid(33, 29, 0.01)
    Z = rng.normal(size=(29, 33))
    Z[rng.random(Z.shape) < 0.1] = np.inf
    full = oracle.gauss_filter(Z, g, 0.07, highpass=True)
    cells = rng.integers(0, Z.size, 50)
    assert np.array_equal(oracle.gauss_filter(Z, g, 0.07, highpass=True, cells=cells),
                          full.ravel()[cells])
    # a window smaller than one cell keeps every value
    assert np.array_equal(oracle.gauss_filter(Z, g, 0.005), Z)
    with pytest.raises(ValueError):
        oracle.gauss_filter(Z, g, -1.0)


# --- Latin hypercube sampling of the dataset generator --------------------------------------

def test_lhs_puts_one_point_in_every_stratum():
    ranges = {"a": (0.0, 1.0), "b": (-3.0, 5.0), "c": (10.0, 10.5)}
    n = 97
    pts = W.lhs(n, ranges, seed=3)
    assert len(pts) == n
    for name, (lo, hi) in ranges.items():
        v = np.array([p[name] for p in pts])
        assert np.all((v >= lo) & (v < hi))
        strata = np.floor((v - lo) / (hi - lo) * n).astype(int)
        assert sorted(strata) == list(range(n))
    # the pairing differs between parameters and the draw is seeded
    sa = np.argsort([p["a"] for p in pts])
    sb = np.argsort([p["b"] for p in pts])
    assert not np.array_equal(sa, sb)
    assert W.lhs(n, ranges, seed=3) == pts and W.lhs(n, ranges, seed=4) != pts


def test_dataset_sims_share_one_grid():
    sims = W.dataset_sims(12, side=256, dd=0.004)
    assert len({(s.grid.nx, s.grid.ny, s.grid.dd, s.grid.x0) for s in sims}) == 1
    assert sorted({s.tool.n_teeth for s in sims}) == [2, 3, 4]
    assert len({s.cut.f_z for s in sims}) == 12
