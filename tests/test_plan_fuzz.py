"""Property test of the host planner at the C ABI: over drawn tool, cut and grid parameters
(valid ones and edge values: zero, negative, non-finite), fsm_plan and fsm_edge_points return
a status code and never crash.  Every draw inside the documented ranges is accepted; what the
library accepts the oracle accepts too, and there the plan and the edge points agree bit for
bit.  The library checks more than the oracle (finiteness of every value, angle bounds), so an
edge value the oracle lets through may still be rejected."""
import dataclasses
import math

import numpy as np
import pytest

hyp = pytest.importorskip("hypothesis")
from hypothesis import HealthCheck, given, settings, strategies as st  # noqa: E402

import oracle  # noqa: E402
from paper_2603_28160_amd import _abi, fsm_edge_points, fsm_plan, workloads as W  # noqa: E402

EDGE = st.sampled_from([0.0, -1.0, math.nan, math.inf])


@st.composite
def sims(draw):
    clean = [True]

    def val(lo, hi, edge=True):
        s = st.floats(lo, hi, allow_nan=False, allow_infinity=False)
        if not edge:
            return draw(s)
        v = draw(EDGE) if draw(st.integers(0, 15)) == 0 else draw(s)
        clean[0] &= math.isfinite(v) and lo <= v <= hi
        return v

    def count(lo, hi, valid_lo):
        v = draw(st.integers(lo, hi))
        clean[0] &= v >= valid_lo
        return v

    kind = draw(st.sampled_from([W.ROUND, W.BALL]))
    z_n = count(1, 9, 1)
    clean[0] &= z_n <= 8
    D = val(0.5, 20.0)
    pitch = draw(st.booleans())
    theta = None
    if not pitch and 1 <= z_n <= 8:
        theta = tuple(sorted(draw(st.lists(st.floats(0.0, 6.28), min_size=z_n, max_size=z_n))))
    tool = W.Tool(kind=kind, n_teeth=z_n, n_edge=count(0, 80, 1), D=D,
                  R_edge=val(0.01, 10.0), helix=val(0.0, 1.2),
                  rake_radial=val(-0.3, 0.3, edge=False), theta=theta,
                  runout_ecc=val(0.0, 0.02), runout_phase=val(0.0, 6.3, edge=False),
                  tilt_lead=val(-0.5, 0.5), tilt_side=val(-0.5, 0.5, edge=False))
    cut = W.Cut(f_z=val(0.001, 0.5), a_p=val(0.01, 2.0), a_e=val(0.05, 3.0),
                steps_per_rev=count(-1, 2000, 1), n_passes=count(0, 6, 0),
                n_steps=count(-1, 3000, 0))
    nx, ny = count(-1, 400, 1), count(-1, 400, 1)
    grid = W.centred_grid(max(nx, 1), max(ny, 1), draw(st.floats(0.001, 0.05)))
    grid = dataclasses.replace(grid, nx=nx, ny=ny)
    return W.Sim(tool, cut, grid), clean[0]


@settings(max_examples=500, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow])
@given(sims())
def test_planner_accepts_valid_draws_and_agrees_with_the_oracle(drawn):
    s, clean = drawn
    try:
        want = oracle.plan(s)
    except ValueError:
        want = None
    try:
        got = fsm_plan(s)
    except _abi.FsmError as e:
        assert e.code == _abi.EINVAL, e
        got = None
    hyp.event("accepted" if got is not None else "rejected")
    if clean:
        assert got is not None, s
    if got is None:
        return
    assert want is not None, s
    for k in want:
        assert got[k] == want[k] or (math.isnan(got[k]) and math.isnan(want[k])), k
    _, b = oracle.edge_points(s)
    assert np.array_equal(fsm_edge_points(s), b)
