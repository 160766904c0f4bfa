"""The C ABI from C and C++: a C11 program built against include/fsm.h and linked to
libfsm.so calls the host-only entry points (tests/host/abi_from_c.c), a C++ caller links with
C linkage, and the header is plain C99.  CPU only: nothing touches a device."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2603_28160_amd")


def test_host_calls_from_c(tmp_path):
    if not os.path.exists(os.path.join(PKG, "libfsm.so")):
        pytest.skip("libfsm.so not built")
    exe = tmp_path / "abi_from_c"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "host", "abi_from_c.c"), "-L", PKG, "-lfsm",
                    f"-Wl,-rpath,{PKG}", "-lm", "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0 and "OK" in r.stdout, r.stdout + r.stderr


def test_header_links_from_cpp_and_compiles_as_c99(tmp_path):
    # the declarations carry C linkage for C++ callers, and the header is plain C99 as well
    if not os.path.exists(os.path.join(PKG, "libfsm.so")):
        pytest.skip("libfsm.so not built")
    src = tmp_path / "use.cpp"
    src.write_text('#include "fsm.h"\n#include <cstdio>\n'
                   'int main() { std::printf("%d %s\\n", fsm_version(), fsm_strerror(FSM_EINVAL)); '
                   'return fsm_version() >= 1 ? 0 : 1; }\n')
    exe = tmp_path / "use"
    inc = os.path.join(ROOT, "include")
    subprocess.run(["g++", "-std=c++11", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", inc,
                    str(src), "-L", PKG, "-lfsm", f"-Wl,-rpath,{PKG}", "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-fsyntax-only",
                    "-x", "c", os.path.join(inc, "fsm.h")], check=True)
