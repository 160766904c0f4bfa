"""The overlap check of caller-owned device maps (csrc/fsm_spans.h), built from source with
a small C++ check (tests/host/spans_check.cpp) against brute force.  CPU only."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2603_28160_amd", "csrc")


def test_spans(tmp_path):
    exe = tmp_path / "spans_check"
    subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-Werror", "-I", CSRC,
                    os.path.join(ROOT, "tests", "host", "spans_check.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "OK" in r.stdout, r.stdout + r.stderr
