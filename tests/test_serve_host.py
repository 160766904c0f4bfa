"""The serving loop's scheduler on the host (fsm_serve_dry_run): the same admission, batching and
slot rules as fsm_serve_run, against a simulated clock.  Checked here: every request finishes
once, first come first served, no start before arrival, batches within max_batch, never more
batches in flight than slots, the arena never overcommitted, continuous batching (a request
that arrives while a batch runs starts before it ends), rejection of oversized and invalid
requests without stalling the rest."""
import dataclasses

import numpy as np
import pytest

from paper_2603_28160_amd import _abi, fsm_plan, fsm_serve_dry_run, workloads as W


def small(i, side=96):
    s = W.random_sim(4, i, side_max=256)
    return s.replace(grid=W.centred_grid(side, side, s.grid.dd))


def zbytes(s, prec="f32"):
    return s.grid.nx * s.grid.ny * (4 if prec == "f32" else 8)


def batches(res):
    out = {}
    for k, r in enumerate(res):
        if r["batch"] >= 0:
            out.setdefault(r["batch"], []).append(k)
    return out


def check_common(reqs, res, max_batch, n_slots, realtime=True):
    for (s, a, _), r in zip(reqs, res):
        if r["status"] != 0:
            continue
        assert r["done_s"] >= r["start_s"] >= r["admit_s"]
        if realtime:
            assert r["admit_s"] >= a - 1e-12
    b = batches(res)
    for idx in b.values():
        assert len(idx) <= max_batch
        assert len({res[k]["slot"] for k in idx}) == 1
        assert len({res[k]["start_s"] for k in idx}) == 1
    # never more batches in flight than slots, and one batch per slot at a time
    iv = sorted((res[idx[0]]["start_s"], res[idx[0]]["done_s"], res[idx[0]]["slot"]) for idx in b.values())
    for t0, _, _ in iv:
        live = [(a, d, sl) for a, d, sl in iv if a <= t0 < d]
        assert len(live) <= n_slots
        assert len({sl for _, _, sl in live}) == len(live)


def test_every_request_runs_once_in_arrival_order():
    rng = np.random.default_rng(1)
    arrivals = np.sort(rng.uniform(0, 0.05, 40))
    reqs = [(small(i), float(a), None) for i, a in enumerate(arrivals)]
    res, peak = fsm_serve_dry_run(reqs, n_slots=2, max_batch=4, arena_bytes=64 << 20)
    assert all(r["status"] == 0 for r in res)
    check_common(reqs, res, 4, 2)
    # first come first served: start order follows arrival order
    starts = [r["start_s"] for r in res]
    assert starts == sorted(starts)
    b = [r["batch"] for r in res]
    assert b == sorted(b)
    assert 0 < peak <= 64 << 20


def test_burst_forms_full_batches_and_slots_overlap():
    reqs = [(small(i), 0.0, None) for i in range(20)]
    res, _ = fsm_serve_dry_run(reqs, n_slots=2, max_batch=4, arena_bytes=1 << 30,
                               launch_s=1e-3)
    sizes = sorted(len(v) for v in batches(res).values())
    assert sizes == [4] * 5
    check_common(reqs, res, 4, 2)
    slots = {r["slot"] for r in res}
    assert slots == {0, 1}


def test_continuous_batching_joins_while_others_run():
    # a long request first, then short ones arriving while it runs: they must start (on the
    # other slot) before the long one finishes
    big = small(0, side=512)
    reqs = [(big, 0.0, None)] + [(small(i + 1), 0.001 * (i + 1), None) for i in range(6)]
    res, _ = fsm_serve_dry_run(reqs, n_slots=2, max_batch=8, arena_bytes=1 << 30,
                               per_eval_s=1e-10)
    long_done = res[0]["done_s"]
    assert any(r["start_s"] < long_done for r in res[1:])
    assert all(r["slot"] == 1 for r in res[1:] if r["start_s"] < long_done)
    check_common(reqs, res, 8, 2)


def test_arena_bounds_admission():
    reqs = [(small(i, side=128), 0.0, None) for i in range(12)]
    arena = 3 * zbytes(reqs[0][0]) + 4096        # three maps at a time
    res, peak = fsm_serve_dry_run(reqs, n_slots=4, max_batch=8, arena_bytes=arena)
    assert all(r["status"] == 0 for r in res)
    assert peak <= arena
    # never more than three requests admitted and unfinished at once
    for r in res:
        t = r["admit_s"]
        held = [q for q in res if q["admit_s"] <= t < q["done_s"]]
        assert len(held) <= 3
    check_common(reqs, res, 8, 4)


def test_oversized_and_invalid_requests_are_rejected_alone():
    ok = small(1)
    huge = ok.replace(grid=W.centred_grid(4096, 4096, ok.grid.dd))
    bad = ok.replace(tool=dataclasses.replace(ok.tool, n_teeth=0))
    reqs = [(ok, 0.0, None), (huge, 0.0, None), (bad, 0.0, None), (small(2), 0.0, None)]
    res, _ = fsm_serve_dry_run(reqs, n_slots=2, max_batch=4, arena_bytes=8 << 20)
    assert [r["status"] for r in res] == [0, _abi.ENOMEM, _abi.EINVAL, 0]
    assert res[1]["batch"] == -1 and res[2]["batch"] == -1


def test_caller_owned_maps_take_no_arena():
    reqs = [(small(i), 0.0, 1) for i in range(6)]
    res, peak = fsm_serve_dry_run(reqs, n_slots=2, max_batch=3, arena_bytes=0)
    assert all(r["status"] == 0 for r in res)
    assert peak == 0


def test_slot_workspace_limits_batches():
    reqs = [(small(0, side=256), 0.0, 1)] * 6     # six copies: one fits exactly as well as another

    def alone_fits(slot):
        r, _ = fsm_serve_dry_run(reqs[:1], n_slots=1, max_batch=6, arena_bytes=0, slot_bytes=slot)
        return r[0]["status"] == 0

    # the smallest slot one request fits (its bucket sliced down to one binning item)
    lo, hi = 4096, fsm_plan(reqs[0][0], "f32")["workspace_bytes"]
    assert alone_fits(hi) and not alone_fits(lo)
    while hi - lo > 4096:
        mid = (lo + hi) // 2
        lo, hi = (lo, mid) if alone_fits(mid) else (mid, hi)
    res, _ = fsm_serve_dry_run(reqs, n_slots=2, max_batch=6, arena_bytes=0,
                               slot_bytes=int(hi * 1.5))
    assert all(r["status"] == 0 for r in res)
    assert max(len(v) for v in batches(res).values()) < 6
    # far too small a slot: every request is rejected, none stalls the loop
    res, _ = fsm_serve_dry_run(reqs, n_slots=2, max_batch=6, arena_bytes=0, slot_bytes=lo)
    assert all(r["status"] == _abi.ENOMEM for r in res)


def test_offline_mode_ignores_arrival_times():
    reqs = [(small(i), 10.0 + i, None) for i in range(5)]
    res, _ = fsm_serve_dry_run(reqs, realtime=False, n_slots=1, max_batch=5, arena_bytes=1 << 30)
    assert all(r["start_s"] == 0.0 for r in res)
    assert len(batches(res)) == 1


@pytest.mark.parametrize("bad", [dict(n_slots=0), dict(n_slots=17), dict(max_batch=0),
                                 dict(slot_bytes=0), dict(arena_bytes=-1)])
def test_bad_configuration(bad):
    kw = dict(n_slots=2, max_batch=4, arena_bytes=1 << 20, slot_bytes=1 << 30)
    kw.update(bad)
    with pytest.raises(_abi.FsmError):
        fsm_serve_dry_run([(small(0), 0.0, None)], **kw)
