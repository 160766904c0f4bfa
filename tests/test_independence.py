"""The oracle and the library share no code: importing the package loads nothing from
oracle/, no library source names the oracle's modules or header, and no oracle source names
the package, its C sources or the public header.  Only the seeded input records
(paper_2603_28160_amd/workloads.py, no arithmetic of the method) are given to both, by the
tests.  CPU only."""
import os
import re
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2603_28160_amd")
ORACLE = os.path.join(ROOT, "oracle")


def sources(top, exts):
    for d, _, files in os.walk(top):
        if "__pycache__" in d:
            continue
        for f in files:
            if f.endswith(exts):
                yield os.path.join(d, f)


def test_package_import_loads_no_oracle():
    r = subprocess.run([sys.executable, "-c",
                        "import sys; sys.path.insert(0, sys.argv[1]); import paper_2603_28160_amd; "
                        "print(any(m == 'oracle' or m.startswith('oracle.') for m in sys.modules))",
                        ROOT], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip() == "False"


def test_library_sources_do_not_reach_the_oracle():
    bad = re.compile(r"^\s*(import oracle|from oracle)|fsm_oracle|liboracle", re.M)
    for path in sources(PKG, (".py", ".cpp", ".hip", ".h")):
        assert not bad.search(open(path).read()), path
    for path in (os.path.join(ROOT, "include", "fsm.h"),):
        assert not bad.search(open(path).read()), path


def test_oracle_sources_do_not_reach_the_library():
    # includes, imports and loaded libraries only (comments may say what the oracle is not)
    include = re.compile(r"^\s*#\s*include\s*[\"<]([^\">]+)[\">]", re.M)
    for path in sources(ORACLE, (".c", ".h")):
        for name in include.findall(open(path).read()):
            assert name == "fsm_oracle.h" or "/" not in name and not name.startswith("fsm"), (path, name)
    pyimport = re.compile(r"^\s*(?:import|from)\s+(\S+)", re.M)
    for path in sources(ORACLE, (".py",)):
        text = open(path).read()
        for mod in pyimport.findall(text):
            assert not mod.startswith(("paper_2603_28160_amd", "bench", "tests")), (path, mod)
        assert "libfsm" not in text, path
