"""GPU tests of the batched form: many uneven simulations in one launch sequence.

Each result of a batch must equal the same simulation run alone (bit for bit: every kernel
computes a simulation's points, tiles and reductions independently of its neighbours), and
the double-precision results must equal the CPU oracle.  Graph replays are checked against
the eager result after eager work on the same context in between.
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from paper_2603_28160_amd import _abi, workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_28160_amd import Context
    return Context


def small_mix(n, seed_cfg=3, scale=4):
    sims = []
    for i in range(n):
        s = W.random_sim(seed_cfg, i, side_max=320)
        sims.append(s.replace(grid=dataclasses.replace(s.grid, dd=s.grid.dd * scale)))
    return sims


def same_rough(a, b):
    for k, v in a.items():
        w = b[k]
        if isinstance(v, float) and math.isnan(v):
            assert math.isnan(w), k
        else:
            assert v == w, (k, v, w)


def np_maps(zs):
    return [z.cpu().numpy().astype(np.float64) for z in zs]


@pytest.mark.parametrize("strategy", ["binned", "scatter"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_batch_equals_alone(Ctx, strategy, prec):
    sims = small_mix(7)
    with Ctx(0) as ctx:
        ctx.set_strategy(strategy)
        print(f"[gpu] batch of {len(sims)} {strategy} {prec}", flush=True)
        zb, rb = ctx.fsm_simulate_batch(sims, prec)
        mb = np_maps(zb)
        for k, s in enumerate(sims):
            z1, r1 = ctx.fsm_simulate(s, prec)
            assert np.array_equal(mb[k], z1.cpu().numpy().astype(np.float64)), k
            same_rough(rb[k], r1)


def test_batch_f64_matches_oracle(Ctx):
    sims = small_mix(5)
    with Ctx(0) as ctx:
        zb, rb = ctx.fsm_simulate_batch(sims, "f64")
        mb = np_maps(zb)
    for k, s in enumerate(sims):
        zo, cnt = oracle.simulate(s)
        assert np.array_equal(mb[k], zo), k
        assert rb[k]["n_binned"] == cnt["n_binned"]
        assert rb[k]["n_evals"] == cnt["n_evals"]
        ro = oracle.roughness(zo)
        for key in ("Sa", "Sq", "Sz", "Ssk", "Sku", "Ra_feed", "Ra_pick"):
            if math.isnan(ro[key]):
                assert math.isnan(rb[k][key])
            else:
                assert abs(rb[k][key] - ro[key]) <= 1e-4 * abs(ro[key]) + 1e-12, (k, key)


def test_batch_slices_equal_unsliced(Ctx):
    sims = small_mix(6)
    with Ctx(0) as ctx:
        za, ra = ctx.fsm_simulate_batch(sims, "f64")
        ma = np_maps(za)
        ctx.fsm_ctx_set_option(_abi.OPT_BUCKET_BYTES, 1 << 20)
        zb, rb = ctx.fsm_simulate_batch(sims, "f64")
        mb = np_maps(zb)
    for k in range(len(sims)):
        assert np.array_equal(ma[k], mb[k]), k
        same_rough(ra[k], rb[k])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_graph_replays_match_eager(Ctx, prec):
    import torch
    sims = small_mix(5)
    with Ctx(0) as eager:
        ze, re_ = eager.fsm_simulate_batch(sims, prec)
        me = np_maps(ze)
    with Ctx(0) as ctx:
        ctx.set_graphs(True)
        zmaps = [ctx.new_zmap(s.grid, prec) for s in sims]
        for rep in range(4):
            for z in zmaps:
                z.fill_(123.0)            # stale contents must be fully overwritten
            print(f"[gpu] graph replay {rep} {prec}", flush=True)
            zg, rg = ctx.fsm_simulate_batch(sims, prec, zmaps=zmaps)
            mg = np_maps(zg)
            for k in range(len(sims)):
                assert np.array_equal(mg[k], me[k]), (rep, k)
                same_rough(rg[k], re_[k])
            # eager work of the program between replays
            one, _ = ctx.fsm_simulate(sims[rep % len(sims)], prec)
            torch.cuda.synchronize()
            assert np.array_equal(one.cpu().numpy().astype(np.float64), me[rep % len(sims)])


@pytest.mark.parametrize("strategy", ["binned", "scatter"])
def test_graph_replay_fresh_maps_and_parameters(Ctx, strategy):
    # A captured launch sequence is reused only for a set that lays out the same way: fresh
    # Z-maps on every call and members whose parameters (so item and row counts) change while
    # every grid stays the same must each give the eager result.  The small bucket budget
    # splits the histogram work into several slices whose tile ranges depend on the members'
    # row counts; swapping the members keeps every total but moves those ranges.
    import torch
    mix = small_mix(3)
    g = mix[0].grid
    a, b, c = [s.replace(grid=g) for s in mix]
    sets = [[a, b, c], [c, b, a], [b, a, c]]
    with Ctx(0) as eager:
        eager.set_strategy(strategy)
        eager.fsm_ctx_set_option(_abi.OPT_BUCKET_BYTES, 1 << 20)
        eager.fsm_ctx_set_profiling(True)
        want = []
        for s in sets:
            z, r = eager.fsm_simulate_batch(s, "f64")
            want.append([np_maps(z), r])
            if strategy == "binned":
                assert eager.fsm_last_timings()["n_slices"] > 1
    with Ctx(0) as ctx:
        ctx.set_strategy(strategy)
        ctx.fsm_ctx_set_option(_abi.OPT_BUCKET_BYTES, 1 << 20)
        ctx.set_graphs(True)
        for rep in range(2):
            for k, s in enumerate(sets):
                print(f"[gpu] graph {strategy} set {k} replay {rep}", flush=True)
                zg, rg = ctx.fsm_simulate_batch(s, "f64")
                torch.cuda.synchronize()
                for m, (zm, r) in enumerate(zip(np_maps(zg), rg)):
                    assert np.array_equal(zm, want[k][0][m]), (rep, k, m)
                    same_rough(r, want[k][1][m])
    for s, zm in zip(sets[0], want[0][0]):
        zo, _ = oracle.simulate(s)
        assert np.array_equal(zm, zo)


def test_batch_with_empty_and_tiny_members(Ctx):
    base = W.config2(nx=90, ny=70, dd=0.02)
    far = base.replace(cut=dataclasses.replace(base.cut, n_passes=1, y_first=80.0, a_e=0.0))
    tiny = base.replace(grid=W.centred_grid(1, 1, 0.05))
    sims = [base, far, tiny, W.config1()]
    with Ctx(0) as ctx:
        zb, rb = ctx.fsm_simulate_batch(sims, "f64")
        mb = np_maps(zb)
    assert np.all(np.isinf(mb[1])) and rb[1]["n_hit"] == 0 and rb[1]["flags"] & _abi.FLAG_NO_HIT
    for k in (0, 2, 3):
        zo, _ = oracle.simulate(sims[k])
        assert np.array_equal(mb[k], zo), k


def test_overlapping_maps_rejected(Ctx):
    # the jobs' Z-maps of one call are written by the same launches: a shared byte is an
    # error found on the host before anything is queued; disjoint views of one buffer are fine
    torch = pytest.importorskip("torch")
    sims = small_mix(2)
    sims = [sims[0], sims[0].replace(name="copy")]
    g = sims[0].grid
    cells = g.nx * g.ny
    with Ctx(0) as ctx:
        buf = torch.empty(2 * cells + 1, dtype=torch.float64, device="cuda:0")
        a = buf[:cells].view(g.ny, g.nx)
        b = buf[cells - 1:2 * cells - 1].view(g.ny, g.nx)      # shares a's last cell
        for call in (ctx.fsm_simulate_batch, ctx.fsm_batch_submit):
            with pytest.raises(_abi.FsmError, match="jobs 0 and 1: Z-maps overlap") as e:
                call(sims, "f64", zmaps=[a, b])
            assert e.value.code == _abi.EINVAL
        with pytest.raises(_abi.FsmError, match="overlap"):
            ctx.fsm_simulate_batch(sims, "f64", zmaps=[a, a])
        c = buf[cells:2 * cells].view(g.ny, g.nx)
        zs, rs = ctx.fsm_simulate_batch(sims, "f64", zmaps=[a, c])
        assert np.array_equal(zs[0].cpu().numpy(), zs[1].cpu().numpy())
        same_rough(rs[0], rs[1])


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_super_mode_batch_equals_alone(Ctx, prec):
    # one member with more 16 x 16-cell tiles than a row histogram holds (132 x 129): the whole
    # batch counts per super-tile, each member's found through the super-tile bases, and
    # splits them into tiles; every member must equal its run alone (the small ones alone take
    # the histogram mode), with the default bucket budget and with a small one (more slices)
    big = W.config2(nx=2100, ny=2050, dd=0.002)
    mix = small_mix(3)
    sims = [mix[0], big, mix[1], mix[2]]
    slices = []
    with Ctx(0) as ctx:
        ctx.fsm_ctx_set_option(_abi.OPT_AUTOTUNED, 0)
        ctx.fsm_ctx_set_option(_abi.OPT_TILE_SHAPE, 0x44)
        for budget in (16 << 30, 256 << 20):
            ctx.fsm_ctx_set_option(_abi.OPT_BUCKET_BYTES, budget)
            print(f"[gpu] super-mode batch {prec}, bucket budget {budget >> 20} MiB", flush=True)
            ctx.fsm_ctx_set_profiling(True)
            zb, rb = ctx.fsm_simulate_batch(sims, prec)
            t = ctx.fsm_last_timings()
            ctx.fsm_ctx_set_profiling(False)
            assert t["zmap_path"] == _abi.PATH_SUPER, t
            slices.append(t["n_slices"])
            mb = np_maps(zb)
            for k, s in enumerate(sims):
                z1, r1 = ctx.fsm_simulate(s, prec)
                assert np.array_equal(mb[k], z1.cpu().numpy().astype(np.float64)), (budget, k)
                same_rough(rb[k], r1)
    assert slices[1] > slices[0], slices
