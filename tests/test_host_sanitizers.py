"""The host-only C++ checks rebuilt with the compiler's sanitizers: the planner's thread pool
and the planner itself under ThreadSanitizer (no data race, no lock-order problem), and the
pool, the planner, map-overlap sweep and serving arena under AddressSanitizer with
UndefinedBehaviorSanitizer (no out-of-bounds access, leak or undefined operation).  g++ on the
CPU only; no device code is built here."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2603_28160_amd", "csrc")
HOST = os.path.join(ROOT, "tests", "host")

CHECKS = {
    "pool": ["pool_check.cpp", os.path.join(CSRC, "fsm_plan.cpp")],
    "spans": ["spans_check.cpp"],
    "arena": ["arena_check.cpp", os.path.join(CSRC, "fsm_sched.cpp")],
    "plan": ["plan_check.cpp", os.path.join(CSRC, "fsm_plan.cpp")],
}
SANITIZERS = {
    "thread": (["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1"}),
    "address": (["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                {"ASAN_OPTIONS": "detect_leaks=1", "UBSAN_OPTIONS": "halt_on_error=1"}),
}
CASES = [("pool", "thread"), ("pool", "address"), ("spans", "address"), ("arena", "address"),
         ("plan", "address"), ("plan", "thread")]


@pytest.mark.parametrize("check,san", CASES, ids=[f"{c}-{s}" for c, s in CASES])
def test_host_check_under_sanitizer(tmp_path, check, san):
    flags, env = SANITIZERS[san]
    srcs = [s if os.path.isabs(s) else os.path.join(HOST, s) for s in CHECKS[check]]
    exe = tmp_path / f"{check}_{san}"
    r = subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-pthread", *flags, "-I", CSRC, *srcs,
                        "-o", str(exe)], capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr:
        pytest.skip(f"{san} sanitizer unavailable: {r.stderr.strip()[:200]}")
    assert r.returncode == 0, r.stderr
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300,
                         env={**os.environ, **env})
    assert run.returncode == 0 and "OK" in run.stdout, run.stdout + run.stderr[-3000:]
