"""The large single field at its full size: a D = 12 mm four-flute round-edge mill over
40000 x 40000 cells at 0.5 um (1.6e9 cells, 5.7e8 edge-point evaluations), the launch the
benchmark's large-field leg times.  Its 98 125 (FP64) or 49 141 (FP32) tiles per map are
more than one row histogram holds, so the binned strategy counts per super-tile and splits
the super-tile buckets into the tiles (super mode).

Double precision: the whole 12.8 GB Z-map equals the oracle's, bit for bit, with identical
in-grid counts and roughness within 1e-4.  Single precision: sampled windows inside the
oracle's per-cell intervals.  The oracle calls run in parallel threads (ctypes releases the
interpreter lock)."""
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle
from paper_2603_28160_amd import workloads as W

import f32_bounds as FB

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import os
    from paper_2603_28160_amd import Context, _abi
    c = Context(0)
    # the benchmark's launch parameters: the shipped tuning table (its single-precision entry
    # covers this field; double precision keeps the defaults)
    c.load_tuning(os.path.join(os.path.dirname(_abi.__file__), "tuning_mi355x.json"))
    yield c
    c.close()


def test_config5_f64_full_field_exact(ctx):
    import torch
    s = W.config5()
    with ThreadPoolExecutor(1) as pool:
        fut = pool.submit(oracle.simulate, s)
        print("[gpu] config5 f64 40000x40000", flush=True)
        ctx.fsm_ctx_set_profiling(True)
        z, r = ctx.fsm_simulate(s, "f64")
        torch.cuda.synchronize()
        t = ctx.fsm_last_timings()
        ctx.fsm_ctx_set_profiling(False)
        from paper_2603_28160_amd import _abi
        assert t["zmap_path"] == _abi.PATH_SUPER and t["n_slices"] == 1, t
        zg = z.cpu().numpy()
        del z
        torch.cuda.empty_cache()
        zo, cnt = fut.result()
    assert r["n_evals"] == cnt["n_evals"]
    assert r["n_binned"] == cnt["n_binned"]
    assert np.array_equal(zg, zo)
    ro = oracle.roughness(zo)
    assert r["n_hit"] == ro["n_hit"]
    for k in ("Sa", "Sq", "Sp", "Sv", "Sz", "Ssk", "Sku", "Ra_feed", "Ra_pick", "mean"):
        assert abs(r[k] - ro[k]) <= 1e-4 * abs(ro[k]) + 1e-12, (k, r[k], ro[k])


def test_config5_f32_windows(ctx):
    import torch
    s = W.config5()
    n = s.grid.nx
    rng = np.random.default_rng([28160, 5, 1])
    windows = [(n // 2 - 48, n // 2 + 48, n // 2 - 48, n // 2 + 48),
               (0, 64, n - 64, n)]
    i0, j0 = (int(v) for v in rng.integers(0, n - 128, 2))
    windows.append((i0, i0 + 128, j0, j0 + 96))
    with ThreadPoolExecutor(len(windows)) as pool:
        futs = [pool.submit(FB.f32_intervals, s, None, FB.F32_TOL, w) for w in windows]
        print("[gpu] config5 f32 40000x40000", flush=True)
        z, r = ctx.fsm_simulate(s, "f32")
        torch.cuda.synchronize()
        parts = [z[b:e, a:c].cpu().numpy().astype(np.float64) for a, c, b, e in windows]
        del z
        torch.cuda.empty_cache()
        for f, zg in zip(futs, parts):
            low, high, must_hit, must_miss = f.result()
            FB.check_cells(zg, low, high, must_hit, must_miss)
    assert r["n_evals"] == oracle.plan(s)["n_evals"]
