"""The warm-started min-cost flow of successive flow updates (host code, no GPU): compiled with
the host compiler from the library's own source and run on a sequence of problems."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2405_09400_amd", "csrc")


def test_warm_started_mcf_matches_cold_solves(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "mcf_warm_check"
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", CSRC,
                    os.path.join(ROOT, "tests", "mcf_warm_check.cpp"),
                    os.path.join(CSRC, "mcf.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout
