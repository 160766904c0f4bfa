"""GPU checks of the asynchronous batches: a submitted batch gives the maps and roughness of
the synchronous batch bit for bit, batches overlap on the context's slots, admission refuses
(FSM_EAGAIN, nothing queued) when every slot holds a batch not yet waited for or the HBM
budget is too small, work queued later on the caller's stream sees the finished maps, and
unknown ids are refused."""
import dataclasses

import numpy as np
import pytest

from paper_2603_28160_amd import _abi, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture()
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_28160_amd import Context
    c = Context(0)
    yield c
    c.close()


def small_mix(k0, n, side=300):
    sims = [W.random_sim(3, k0 + i, side_max=side) for i in range(n)]
    return [s.replace(grid=dataclasses.replace(s.grid, dd=s.grid.dd * 4)) for s in sims]


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_async_equals_sync(ctx, prec):
    a, b = small_mix(0, 5), small_mix(10, 3)
    za, ra = ctx.fsm_simulate_batch(a, prec)
    zb, rb = ctx.fsm_simulate_batch(b, prec)
    print(f"[gpu] async batches {prec}", flush=True)
    ida, ma = ctx.fsm_batch_submit(a, prec)
    idb, mb = ctx.fsm_batch_submit(b, prec)
    assert ida != idb
    ra2 = ctx.fsm_batch_wait(ida)
    rb2 = ctx.fsm_batch_wait(idb)
    for ref, got, rr, rg in ((za, ma, ra, ra2), (zb, mb, rb, rb2)):
        assert len(rg) == len(ref)
        for k in range(len(ref)):
            assert np.array_equal(ref[k].cpu().numpy(), got[k].cpu().numpy()), k
            assert rg[k] == rr[k], k


def test_admission_and_errors(ctx):
    import torch
    a, b, c = small_mix(20, 2), small_mix(30, 2), small_mix(40, 2)
    ctx.fsm_ctx_set_option(_abi.OPT_ASYNC_SLOTS, 2)
    ida, _ = ctx.fsm_batch_submit(a, "f32")
    idb, _ = ctx.fsm_batch_submit(b, "f32")
    with pytest.raises(_abi.FsmError) as e:          # both slots are held until waited for
        ctx.fsm_batch_submit(c, "f32")
    assert e.value.code == _abi.FSM_EAGAIN
    with pytest.raises(_abi.FsmError) as e:          # no change of slots while batches fly
        ctx.fsm_ctx_set_option(_abi.OPT_ASYNC_SLOTS, 4)
    assert e.value.code == _abi.FSM_EAGAIN
    torch.cuda.synchronize()
    assert ctx.fsm_batch_poll(ida) and ctx.fsm_batch_poll(idb)
    ctx.fsm_batch_wait(ida)
    idc, _ = ctx.fsm_batch_submit(c, "f32")          # a waited-for slot is free again
    ctx.fsm_batch_wait(idb)
    ctx.fsm_batch_wait(idc)
    for bad in (0, ida, 10 ** 9):
        with pytest.raises(_abi.FsmError):
            ctx.fsm_batch_wait(bad)
        with pytest.raises(_abi.FsmError):
            ctx.fsm_batch_poll(bad)
    # a budget below one batch's workspace refuses it; the existing slot workspaces count
    ctx.fsm_ctx_set_option(_abi.OPT_ASYNC_SLOTS, 1)
    ctx.fsm_ctx_set_option(_abi.OPT_HBM_BUDGET, 1 << 20)
    with pytest.raises(_abi.FsmError) as e:
        ctx.fsm_batch_submit(small_mix(50, 2), "f64")
    assert e.value.code == _abi.FSM_EAGAIN
    ctx.fsm_ctx_set_option(_abi.OPT_HBM_BUDGET, 0)
    idd, _ = ctx.fsm_batch_submit(small_mix(50, 2), "f64")
    ctx.fsm_batch_wait(idd)
    for bad in (0, 17):
        with pytest.raises(_abi.FsmError):
            ctx.fsm_ctx_set_option(_abi.OPT_ASYNC_SLOTS, bad)


def test_caller_stream_is_ordered_after_the_batch(ctx):
    import torch
    sims = small_mix(60, 3)
    ref_maps, ref_rough = ctx.fsm_simulate_batch(sims, "f64")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        bid, maps = ctx.fsm_batch_submit(sims, "f64", stream=s)
        # queued on the same stream without waiting: runs after the batch's kernels
        r = ctx.fsm_roughness(sims[0].grid, maps[0], "f64", stream=s)
    # the stand-alone estimator may sum its tiles in another order: last bits only
    assert r["n_hit"] == ref_rough[0]["n_hit"]
    assert r["Sq"] == pytest.approx(ref_rough[0]["Sq"], rel=1e-12)
    assert r["Sa"] == pytest.approx(ref_rough[0]["Sa"], rel=1e-12)
    got = ctx.fsm_batch_wait(bid)
    assert got == ref_rough
    assert np.array_equal(maps[2].cpu().numpy(), ref_maps[2].cpu().numpy())
