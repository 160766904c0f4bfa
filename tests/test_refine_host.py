"""Coverage-complete planning (fsm_refine, host only), checked with the oracle's own
kinematics: after refinement, neighbouring edge points and consecutive time steps of every edge
point lie within the requested spacing, and the swept band of a small face-milling pass is
covered completely where the unrefined plan leaves holes."""
import math

import numpy as np
import pytest

import oracle
from paper_2603_28160_amd import _abi, fsm_refine, workloads as W


def small_face_mill():
    tool = W.Tool(kind=W.ROUND, n_teeth=2, n_edge=12, D=2.0, R_edge=1.0, helix=0.3,
                  runout_ecc=0.002, runout_phase=0.7)
    cut = W.Cut(f_z=0.05, a_p=0.2, steps_per_rev=90, n_passes=1, y_first=0.0)
    return W.Sim(tool, cut, W.centred_grid(60, 60, 0.01))


def test_refined_samples_are_within_spacing():
    s = small_face_mill()
    spacing = 0.005
    r = fsm_refine(s, spacing)
    assert r.tool.n_edge >= s.tool.n_edge and r.cut.steps_per_rev >= s.cut.steps_per_rev
    assert r.cut.n_steps == 0
    _, pT = oracle.edge_points(r)
    gaps = np.linalg.norm(np.diff(pT, axis=1), axis=2)
    assert gaps.max() <= spacing
    # consecutive steps of the outermost edge points, at several places along the pass
    radius = np.hypot(pT[..., 0], pT[..., 1])
    for K in range(r.tool.n_teeth):
        for p in (int(np.argmax(radius[K])), 0, r.tool.n_edge - 1):
            for st in (0, 17, 1000, 5000):
                a = oracle.point(r, 0, st, K, p)
                b = oracle.point(r, 0, st + 1, K, p)
                assert math.hypot(*(b - a)[:2]) <= spacing


def test_refinement_closes_the_holes():
    s = small_face_mill()
    z0, _ = oracle.simulate(s)
    assert np.isfinite(z0).mean() < 0.9            # the coarse plan leaves cells empty
    r = fsm_refine(s, s.grid.dd / 2)
    z1, _ = oracle.simulate(r)
    assert np.isfinite(z1).all()                   # the refined one samples every cell
    assert np.all(z1[np.isfinite(z0)] <= z0[np.isfinite(z0)])   # more samples never raise a cell


def test_fixed_step_mode_refines_dt():
    # the paper's 0.4 us step already moves the insert rim by ~1.5 um per step at 230 m/min:
    # a 1.2 um spacing needs a finer step, a 10 um one keeps it
    s = W.paper_mode(7, dd=0.05)
    assert fsm_refine(s, 0.01).cut.dt == s.cut.dt
    r = fsm_refine(s, 0.0012)
    assert r.cut.dt < s.cut.dt and r.tool.n_edge > s.tool.n_edge
    _, pT = oracle.edge_points(r)
    p = int(np.argmax(np.hypot(pT[0, :, 0], pT[0, :, 1])))
    p0, p1 = oracle.point(r, 0, 100, 0, p), oracle.point(r, 0, 101, 0, p)
    assert math.hypot(*(p1 - p0)[:2]) <= 0.0012


def test_refine_rejects_bad_requests():
    s = small_face_mill()
    for spacing in (0.0, -1.0, float("nan")):
        with pytest.raises(_abi.FsmError):
            fsm_refine(s, spacing)
    with pytest.raises(_abi.FsmError):          # would need more than 4096 edge points
        fsm_refine(W.config2(), 0.0005)


hyp = pytest.importorskip("hypothesis")
from hypothesis import HealthCheck, given, settings, strategies as st  # noqa: E402


@settings(max_examples=60, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow])
@given(st.integers(0, 10_000), st.floats(0.002, 0.05), st.booleans())
def test_spacing_bound_holds_on_drawn_tools(index, spacing, fixed_step):
    # the bound of the refined plan for any drawn tool of the batch mix (round or ball, helix,
    # eccentric runout, lead tilt) or of the paper's fixed-step conditions, with the oracle's
    # own kinematics: neighbouring edge points, and one step of the outermost and end points
    s = W.paper_mode(1 + index % 9, dd=0.05) if fixed_step else W.random_sim(3, index)
    try:
        r = fsm_refine(s, spacing)
    except _abi.FsmError as e:
        assert e.code == _abi.EINVAL                # beyond 4096 edge points or 2^24 steps
        hyp.event("refused")
        return
    hyp.event("refined")
    _, pT = oracle.edge_points(r)
    assert np.linalg.norm(np.diff(pT, axis=1), axis=2).max() <= spacing
    radius = np.hypot(pT[..., 0], pT[..., 1])
    S = r.cut.steps_per_rev
    for K in range(r.tool.n_teeth):
        for p in {int(np.argmax(radius[K])), 0, r.tool.n_edge - 1}:
            for st_ in (0, 1, S // 3, S + 7):
                a = oracle.point(r, 0, st_, K, p)
                b = oracle.point(r, 0, st_ + 1, K, p)
                assert math.hypot(*(b - a)[:2]) <= spacing, (K, p, st_)
