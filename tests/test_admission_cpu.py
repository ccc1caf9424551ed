"""Host tests of plain C++ parts of the library, compiled with g++ and run (no
GPU): the request server's device-pool allocator and admission rule
(paper_1509_04681_amd/csrc/admission.hpp) and the sweeps' wave schedules."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_admission_rule(tmp_path):
    exe = tmp_path / "admission_test"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "paper_1509_04681_amd", "csrc"),
                    os.path.join(ROOT, "tests", "cpp", "admission_test.cpp"), "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "checks passed" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_wave_schedules(tmp_path):
    """The tiled sweeps' wave schedules (paper_1509_04681_amd/csrc/schedule.hpp):
    every tile once, write-disjoint waves, exact ragged edges."""
    exe = tmp_path / "schedule_test"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "paper_1509_04681_amd", "csrc"),
                    os.path.join(ROOT, "tests", "cpp", "schedule_test.cpp"), "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "checks passed" in r.stdout
