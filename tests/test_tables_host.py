"""Injection/sampling tables and z-chunk policy of the host runtime (no GPU): builds
tests/tables_selftest.cpp, which compiles paper_1912_00695_amd/csrc/wave_api.cpp
with the host compiler and checks its tables against a brute-force reference, and
runs it. The launchers the file references resolve against the built libwave.so
(none is called) and the HIP runtime library."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1912_00695_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def test_tables_selftest(tmp_path):
    if not os.path.exists(os.path.join(PKG, "libwave.so")):
        pytest.fail("libwave.so is not built (run __graft_entry__.build())")
    exe = str(tmp_path / "tables_selftest")
    subprocess.run(["g++", "-O2", "-std=c++17", "-D__HIP_PLATFORM_AMD__",
                    "-I", os.path.join(ROCM, "include"), "-I", os.path.join(PKG, "csrc"),
                    os.path.join(ROOT, "tests", "tables_selftest.cpp"), "-o", exe,
                    "-L", PKG, "-lwave", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
                    "-Wl,-rpath," + PKG, "-Wl,-rpath," + os.path.join(ROCM, "lib")],
                   check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stderr
    assert "OK" in r.stdout
