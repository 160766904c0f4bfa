"""The benchmark's bookkeeping on the host (no GPU): the FLOP model per evaluation, the
roofline of the dominant stage with the counter traffic that is read only while the committed
summary was taken on the current kernel source, the per-stage kernel names of each Z-map path,
and the refusal of several GPUs."""
import dataclasses
import os
import subprocess
import sys

import pytest

import bench
from paper_2603_28160_amd import fsm_plan, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def fake_prof(path=2, n_slices=1):
    return {"count_ms": 0.12, "index_ms": 0.04, "write_ms": 0.20, "reduce_ms": 0.17,
            "rough_ms": 0.05, "scatter_ms": 0.0, "fill_ms": 0.0, "n_slices": n_slices,
            "zmap_path": path, "rough": {"n_binned": 48_000_000}}


def test_flop_per_eval_follows_the_tilts():
    t = W.config2().tool
    assert bench.flop_per_eval(t) == 20                       # lead tilt only
    assert bench.flop_per_eval(dataclasses.replace(t, tilt_lead=0.0)) == 14
    assert bench.flop_per_eval(dataclasses.replace(t, tilt_side=0.1)) == 29


def test_roofline_of_the_dominant_stage():
    s = W.config2()
    plan = fsm_plan(s)
    r = bench.roofline(s, plan, "f64", fake_prof())
    assert r["kernel"] == "hist_write<f64>" and r["bound"] == "alu"
    want = 20 * plan["n_evals"] / 0.20e-3 / 1e12
    assert r["achieved"] == pytest.approx(want) and r["frac"] == pytest.approx(want / 78.6)
    # the committed summary was taken on this kernel source
    assert r["traffic"] == bench.stored_traffic("hist_write", "f64") and r["traffic"] > 0


def test_traffic_is_dropped_for_another_kernel_source(tmp_path, monkeypatch):
    other = tmp_path / "fsm_kernels.hip"
    other.write_text("// not the source the counters were taken on\n")
    monkeypatch.setattr(bench, "KERNEL_SRC", str(other))
    assert bench.stored_traffic("hist_write", "f64") is None


@pytest.mark.parametrize("path, write_kernel", [(1, "bin_points<f64,true>"), (2, "hist_write<f64>"),
                                                (3, "hist_write<f64> + split_super")])
def test_stage_names_follow_the_path(path, write_kernel):
    s = W.config2()
    st = bench.stage_rooflines(s, fsm_plan(s), "f64", fake_prof(path))
    assert st["write"]["kernel"] == write_kernel
    assert st["reduce"]["kernel"] == "tile_reduce<f64>" and st["reduce"]["bound"] == "hbm"
    cells = s.grid.nx * s.grid.ny
    assert st["reduce"]["bytes_per_launch"] == 48_000_000 * 10 + cells * 8


def test_several_gpus_are_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stdout + p.stderr
