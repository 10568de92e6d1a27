"""Serving-engine scheduling logic on the host (no GPU): builds tests/sched_selftest.cpp
against paper_1912_00695_amd/csrc/wave_sched.h -- the header the engine itself
uses -- with the host compiler and runs it."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_sched_selftest(tmp_path):
    exe = str(tmp_path / "sched_selftest")
    subprocess.run(["g++", "-O2", "-std=c++17", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "paper_1912_00695_amd", "csrc"),
                    os.path.join(ROOT, "tests", "sched_selftest.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    assert "OK" in r.stdout
