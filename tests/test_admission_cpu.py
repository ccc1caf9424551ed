"""Host tests of plain C++ parts of the library, compiled with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer and run (no GPU): the request
server's device-pool allocator and admission rule
(paper_1509_04681_amd/csrc/admission.hpp), the sweeps' wave schedules and the
graph partitioner; and
the CPU oracle (oracle/cggm_oracle.c) under the same sanitizers."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
            "-fno-omit-frame-pointer", "-g"]


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_admission_rule(tmp_path):
    exe = tmp_path / "admission_test"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", *SANITIZE,
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
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", *SANITIZE,
                    "-I", os.path.join(ROOT, "paper_1509_04681_amd", "csrc"),
                    os.path.join(ROOT, "tests", "cpp", "schedule_test.cpp"), "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "checks passed" in r.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_graph_partitioner(tmp_path):
    """The block-wise method's graph partitioner
    (paper_1509_04681_amd/csrc/partition.hpp): valid parts within the size
    bound, the optimal cut on paths, grids and disjoint cliques, malformed
    patterns rejected, deterministic."""
    exe = tmp_path / "partition_test"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", *SANITIZE,
                    "-I", os.path.join(ROOT, "paper_1509_04681_amd", "csrc"),
                    os.path.join(ROOT, "tests", "cpp", "partition_test.cpp"), "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    """Every oracle entry point on small problems (incl. n < p and the
    huge-page allocation path) with ASan/UBSan: no invalid access, leak or
    undefined arithmetic.  OpenMP is left out of this sanitizer build (pragmas
    ignored)."""
    exe = tmp_path / "oracle_sanitize"
    subprocess.run(["gcc", "-std=c11", "-O1", "-Wall", "-Werror", "-Wno-unknown-pragmas",
                    *SANITIZE, "-I", os.path.join(ROOT, "oracle"),
                    os.path.join(ROOT, "tests", "cpp", "oracle_sanitize.c"),
                    os.path.join(ROOT, "oracle", "cggm_oracle.c"), "-lm", "-o", str(exe)],
                   check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle sanitize: ok" in r.stdout
