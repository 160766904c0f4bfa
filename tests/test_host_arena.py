"""The serving loop's device-arena allocator (csrc/fsm_sched.cpp), built from source with a
small C++ check (tests/host/arena_check.cpp) against a granule map.  CPU only."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2603_28160_amd", "csrc")


def test_arena(tmp_path):
    exe = tmp_path / "arena_check"
    subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-Werror", "-I", CSRC,
                    os.path.join(ROOT, "tests", "host", "arena_check.cpp"),
                    os.path.join(CSRC, "fsm_sched.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "OK" in r.stdout, r.stdout + r.stderr
