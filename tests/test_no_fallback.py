"""Without libfsm.so the binding fails loudly: every entry point that computes raises
ImportError naming the missing library, and nothing falls back to a CPU path.  Run in a child
process with the library path pointed at a file that does not exist.  CPU only."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROBE = r"""
import sys
sys.path.insert(0, sys.argv[1])
import paper_2603_28160_amd as pkg
from paper_2603_28160_amd import _abi, workloads as W
_abi.LIB_PATH = "/nonexistent/libfsm.so"
_abi._lib = None
sim = W.config1()
calls = {
    "fsm_version": lambda: pkg.fsm_version(),
    "fsm_plan": lambda: pkg.fsm_plan(sim),
    "fsm_edge_points": lambda: pkg.fsm_edge_points(sim),
    "fsm_refine": lambda: pkg.fsm_refine(sim, 0.01),
    "fsm_serve_dry_run": lambda: pkg.fsm_serve_dry_run([(sim, 0.0, None)]),
    "Context": lambda: pkg.Context(0),
}
for name, f in calls.items():
    try:
        f()
    except ImportError as e:
        assert "libfsm.so" in str(e), (name, e)
        print("loud", name)
    else:
        print("SILENT", name)
"""


def test_missing_library_fails_loudly():
    r = subprocess.run([sys.executable, "-c", PROBE, ROOT], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr
    lines = r.stdout.split("\n")
    assert "SILENT" not in r.stdout, r.stdout
    assert sum(ln.startswith("loud ") for ln in lines) == 6, r.stdout
