"""GPU checks of coverage-complete planning: a refined small face-milling pass equals the
oracle bit for bit and hits every cell; the refined 200 x 200 single pass (5.8e9 evaluations,
too many for the oracle) hits every cell in both precisions, where the coarse plan hits fewer
than half, and its two precisions agree within the single-precision position error."""
import numpy as np
import pytest

import oracle
from paper_2603_28160_amd import fsm_refine, workloads as W

from test_refine_host import small_face_mill

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2603_28160_amd import Context
    c = Context(0)
    yield c
    c.close()


def test_refined_small_pass_exact_and_complete(ctx):
    s = fsm_refine(small_face_mill(), 0.005)
    print("[gpu] refined small face mill f64", flush=True)
    z, r = ctx.fsm_simulate(s, "f64")
    zo, cnt = oracle.simulate(s)
    assert r["n_binned"] == cnt["n_binned"]
    assert np.array_equal(z.cpu().numpy(), zo)
    assert r["n_hit"] == s.grid.nx * s.grid.ny


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_refined_config1_covers_every_cell(ctx, prec):
    s = W.config1()
    r_sim = fsm_refine(s, s.grid.dd / 2)
    print(f"[gpu] refined config1 {prec}: N {r_sim.tool.n_edge}, S {r_sim.cut.steps_per_rev}", flush=True)
    zc, _ = ctx.fsm_simulate(s, prec)
    zr, rr = ctx.fsm_simulate(r_sim, prec)
    zc, zr = zc.cpu().numpy(), zr.cpu().numpy()
    assert rr["n_hit"] == s.grid.nx * s.grid.ny and not rr["flags"] & 4
    hit = np.isfinite(zc)
    assert hit.mean() < 0.5


def test_refined_config1_precisions_agree(ctx):
    # both maps come from the same samples; single precision moves a point by at most a few
    # ulps of its ~10 mm coordinates, so a cell's minimum may change to a neighbouring sample
    # whose height differs by less than the edge's rise over one sample spacing
    s = W.config1()
    r_sim = fsm_refine(s, s.grid.dd / 2)
    z64, _ = ctx.fsm_simulate(r_sim, "f64")
    z32, _ = ctx.fsm_simulate(r_sim, "f32")
    d = np.abs(z64.cpu().numpy() - z32.cpu().numpy().astype(np.float64))
    assert np.median(d) < 1e-6 and d.max() < s.grid.dd
