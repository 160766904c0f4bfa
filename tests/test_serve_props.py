"""Property test of the serving scheduler on the host (fsm_serve_dry_run) over drawn mixes:
request sizes, arrival times in any order, server-held and caller-owned maps, slot counts,
batch limits and arena sizes.  Every drawn run must keep the loop's rules: each request ends
once, a request that fits the arena runs and one that cannot is rejected alone, admission and
starts follow arrival order, no batch exceeds max_batch or runs on two slots, never more
batches in flight than slots, and the server-held maps in flight never exceed the arena."""
import pytest

hyp = pytest.importorskip("hypothesis")
from hypothesis import HealthCheck, given, settings, strategies as st  # noqa: E402

from paper_2603_28160_amd import _abi, fsm_serve_dry_run, workloads as W  # noqa: E402

SIDES = (16, 48, 96, 160)


def sim(i, side):
    s = W.random_sim(4, 700 + i, side_max=256)
    return s.replace(grid=W.centred_grid(side, side, s.grid.dd))


@st.composite
def runs(draw):
    n = draw(st.integers(1, 24))
    reqs = []
    for i in range(n):
        side = draw(st.sampled_from(SIDES))
        arrival = draw(st.sampled_from([0.0, 0.001, 0.002]) | st.floats(0.0, 0.02))
        owned = draw(st.integers(0, 3)) == 0
        reqs.append((sim(i, side), arrival, 1 if owned else None))
    big = max(SIDES) ** 2 * 4
    arena = draw(st.sampled_from([0, big // 3, big, big + 4096, 3 * big, 64 << 20]))
    cfg = dict(n_slots=draw(st.integers(1, 4)), max_batch=draw(st.integers(1, 6)),
               arena_bytes=arena, realtime=draw(st.booleans()))
    return reqs, cfg


@settings(max_examples=150, deadline=None, derandomize=True,
          suppress_health_check=[HealthCheck.too_slow])
@given(runs())
def test_scheduler_rules_hold_on_drawn_mixes(run):
    reqs, cfg = run
    res, peak = fsm_serve_dry_run(reqs, **cfg)
    arena, rt = cfg["arena_bytes"], cfg["realtime"]
    held = [(s.grid.nx * s.grid.ny * 4 if z is None else 0) for s, _, z in reqs]
    for (s, a, z), r, h in zip(reqs, res, held):
        if h > arena:
            assert r["status"] == _abi.ENOMEM and r["batch"] == -1
            continue
        if h <= arena - 256 or h == 0:
            assert r["status"] == 0, (h, arena, r)
        if r["status"] != 0:
            continue
        assert r["done_s"] >= r["start_s"] >= r["admit_s"] >= 0.0
        if rt:
            assert r["admit_s"] >= a - 1e-12
    ok = [k for k, r in enumerate(res) if r["status"] == 0]
    # first come, first served in the order of the stated arrivals, ties in request order
    # (offline runs, where every request arrives at 0, queue in that order too)
    order = sorted(ok, key=lambda k: (reqs[k][1], k))
    for key in ("admit_s", "start_s", "batch"):
        seq = [res[k][key] for k in order]
        assert seq == sorted(seq), key
    # batches: within max_batch, one slot and one start each
    b = {}
    for k in ok:
        b.setdefault(res[k]["batch"], []).append(k)
    for idx in b.values():
        assert len(idx) <= cfg["max_batch"]
        assert len({res[k]["slot"] for k in idx}) == 1
        assert len({res[k]["start_s"] for k in idx}) == 1
    iv = [(res[i[0]]["start_s"], res[i[0]]["done_s"], res[i[0]]["slot"]) for i in b.values()]
    for t0, _, _ in iv:
        live = [sl for a, d, sl in iv if a <= t0 < d]
        assert len(live) <= cfg["n_slots"] and len(set(live)) == len(live)
    hyp.event("some rejected" if len(ok) < len(reqs) else "all ran")
    hyp.event("batches of several" if max(map(len, b.values()), default=0) > 1 else "batches of one")
    # the arena: what is held from admission to the end never exceeds it
    assert 0 <= peak <= arena
    for k in ok:
        t = res[k]["admit_s"]
        assert sum(held[q] for q in ok if res[q]["admit_s"] <= t < res[q]["done_s"]) <= arena
