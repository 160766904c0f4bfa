"""The shipped tuning table (paper_2603_28160_amd/tuning_mi355x.json, written by
paper_2603_28160_amd.tune on an MI355X): it parses, its entries carry parameters the library
accepts (strategy, tile shape code, rows per launch) with one entry per workload class, and
the benchmark's workloads still fall into classes it holds.  CPU only: the class key is the
library's rule (precision / orders of two of simulations, cells and evaluations), formed
here from fsm_plan's host-side sizes."""
import json
import math
import os

import pytest

from paper_2603_28160_amd import _abi, fsm_plan, workloads as W

TABLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                     "paper_2603_28160_amd", "tuning_mi355x.json")


def order2(v):
    return 0 if v < 1.0 else int(math.floor(math.log2(v) + 0.5))


def class_key(sims, prec):
    cells = sum(float(s.grid.nx) * float(s.grid.ny) for s in sims)
    evals = sum(float(fsm_plan(s, prec)["n_evals"]) for s in sims)
    p = _abi.F64 if prec == "f64" else _abi.F32
    return f"{p}/{order2(len(sims))}/{order2(cells)}/{order2(evals)}"


@pytest.fixture(scope="module")
def table():
    with open(TABLE) as f:
        return json.load(f)


def test_entries_are_valid(table):
    entries = table["entries"]
    assert entries
    keys = [e["key"] for e in entries]
    assert len(keys) == len(set(keys))
    for e in entries:
        prec = int(e["key"].split("/")[0])
        assert prec in (_abi.F64, _abi.F32)
        assert e["strategy"] in (0, 1)
        assert 256 <= e["target_rows"] <= 65536
        code = e["tile_shape"]
        if code:
            sx, sy = code >> 4, code & 15
            assert code >> 8 == 0 and 4 <= sx <= 8 and 4 <= sy <= 8
            # the tile's keys fit the LDS of one workgroup on gfx950 (160 KiB)
            assert (8 if prec == _abi.F64 else 4) << (sx + sy) <= 163840


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_benchmark_workloads_have_entries(table, prec):
    keys = {e["key"] for e in table["entries"]}
    assert class_key([W.config2()], prec) in keys
    assert class_key(W.config3(256), prec) in keys
    # the large field and the latency workload are timed with the table as well
    assert class_key([W.config5()], prec) in keys
    assert class_key([W.config1()], prec) in keys
