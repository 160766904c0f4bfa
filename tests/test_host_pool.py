"""The planner's host thread pool, built from source with a small C++ check (tests/host):
every index runs exactly once, nested loops run inline, concurrent callers and exceptions are
handled, and a forked child does not wait for threads it does not own.  CPU only."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2603_28160_amd", "csrc")


def test_pool(tmp_path):
    exe = tmp_path / "pool_check"
    subprocess.run(["g++", "-O1", "-std=c++17", "-pthread", "-I", CSRC,
                    os.path.join(ROOT, "tests", "host", "pool_check.cpp"),
                    os.path.join(CSRC, "fsm_plan.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "OK" in r.stdout, r.stdout + r.stderr
