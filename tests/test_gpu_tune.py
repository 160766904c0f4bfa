"""GPU tests of the launch parameters and the autotuner: tile shapes and rows per launch change
how the work is cut, never the Z-map (bit-exact against the oracle in double precision and
against the default parameters in both), and change roughness only in the last bits (the
order of the tile partial sums).  The autotuner's choice is used by later calls of the same
workload class and can be switched off."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
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


def close_rough(a, b, rtol=1e-12):
    for k, v in a.items():
        w = b[k]
        if isinstance(v, float):
            if math.isnan(v):
                assert math.isnan(w), k
            else:
                assert abs(v - w) <= rtol * abs(w) + 1e-15, (k, v, w)
        else:
            assert v == w, (k, v, w)


SIM = W.config2(nx=777, ny=613, dd=0.004)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("shape", [0x44, 0x55, 0x56, 0x65, 0x66, 0x75, 0x76, 0x77, 0x86, 0x88])
def test_tile_shapes_keep_the_zmap(ctx, prec, shape):
    # the option holds for both precisions; a tile whose keys exceed 64 KiB in this precision
    # falls back to the default tile, one too large for both is refused
    cells = 1 << ((shape >> 4) + (shape & 15))
    if 4 * cells > 65536:
        with pytest.raises(_abi.FsmError):
            ctx.fsm_ctx_set_option(_abi.OPT_TILE_SHAPE, shape)
        return
    z0, r0 = ctx.fsm_simulate(SIM, prec)
    ctx.fsm_ctx_set_option(_abi.OPT_TILE_SHAPE, shape)
    print(f"[gpu] tile shape {shape:#x} {prec}", flush=True)
    z1, r1 = ctx.fsm_simulate(SIM, prec)
    assert np.array_equal(z0.cpu().numpy(), z1.cpu().numpy())
    close_rough(r1, r0)
    if prec == "f64":
        zo, _ = oracle.simulate(SIM)
        assert np.array_equal(z1.cpu().numpy(), zo)


@pytest.mark.parametrize("rows", [256, 1024, 16384, 65536])
def test_rows_per_launch_keep_the_zmap(ctx, rows):
    z0, r0 = ctx.fsm_simulate(SIM, "f64")
    ctx.fsm_ctx_set_option(_abi.OPT_TARGET_ROWS, rows)
    z1, r1 = ctx.fsm_simulate(SIM, "f64")
    assert np.array_equal(z0.cpu().numpy(), z1.cpu().numpy())
    close_rough(r1, r0)


def test_bad_options_rejected(ctx):
    for opt, val in ((_abi.OPT_TILE_SHAPE, 0x33), (_abi.OPT_TILE_SHAPE, 0x99),
                     (_abi.OPT_TARGET_ROWS, 100), (_abi.OPT_TARGET_ROWS, 1 << 20), (99, 1)):
        with pytest.raises(_abi.FsmError):
            ctx.fsm_ctx_set_option(opt, val)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_autotune_choice_is_used_and_exact(ctx, prec):
    sims = [W.random_sim(3, i, side_max=320) for i in range(4)]
    sims = [s.replace(grid=dataclasses.replace(s.grid, dd=s.grid.dd * 4)) for s in sims]
    z_ref, r_ref = ctx.fsm_simulate_batch(sims, prec)
    ref = [z.cpu().numpy() for z in z_ref]
    print(f"[gpu] autotune batch of {len(sims)} {prec}", flush=True)
    t = ctx.fsm_autotune(sims, prec)
    assert t["n_tried"] >= 5 and t["best_ms"] > 0 and t["best_ms"] <= t["default_ms"]
    assert t["strategy"] in (_abi.ZMAP_BINNED, _abi.ZMAP_SCATTER)
    assert 256 <= t["target_rows"] <= 65536
    z_t, r_t = ctx.fsm_simulate_batch(sims, prec)
    for k in range(len(sims)):
        assert np.array_equal(z_t[k].cpu().numpy(), ref[k]), k
        close_rough(r_t[k], r_ref[k])
    # switched off, the context's own options apply again: same maps
    ctx.fsm_ctx_set_option(_abi.OPT_AUTOTUNED, 0)
    z_o, _ = ctx.fsm_simulate_batch(sims, prec)
    for k in range(len(sims)):
        assert np.array_equal(z_o[k].cpu().numpy(), ref[k]), k
    if prec == "f64":
        for k, s in enumerate(sims):
            zo, _ = oracle.simulate(s)
            assert np.array_equal(ref[k], zo), k


def test_tuning_table_round_trip(ctx):
    import json
    import os
    entries = [{"key": "0/0/18/22", "strategy": _abi.ZMAP_BINNED, "tile_shape": 0x67, "target_rows": 2048},
               {"key": "1/0/18/22", "strategy": _abi.ZMAP_SCATTER, "tile_shape": 0, "target_rows": 4096}]
    ctx.fsm_tune_set(entries)
    got = {e["key"]: e for e in ctx.fsm_tune_get()}
    for e in entries:
        assert got[e["key"]] == e
    for bad in ({"key": "", "strategy": 0, "tile_shape": 0, "target_rows": 4096},
                {"key": "x", "strategy": 7, "tile_shape": 0, "target_rows": 4096},
                {"key": "x", "strategy": 0, "tile_shape": 0x99, "target_rows": 4096},
                {"key": "x", "strategy": 0, "tile_shape": 0, "target_rows": 10}):
        with pytest.raises(_abi.FsmError):
            ctx.fsm_tune_set([bad])
    # the shipped table loads and keeps the maps of its workload classes
    path = os.path.join(os.path.dirname(_abi.__file__), "tuning_mi355x.json")
    if os.path.exists(path):
        z0, r0 = ctx.fsm_simulate(SIM, "f64")
        n = ctx.load_tuning(path)
        assert n == len(json.load(open(path))["entries"])
        z1, r1 = ctx.fsm_simulate(SIM, "f64")
        assert np.array_equal(z0.cpu().numpy(), z1.cpu().numpy())
