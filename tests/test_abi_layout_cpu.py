"""The ctypes mirrors of the C-ABI structs in the Python binding have the
offsets and sizes the C compiler gives include/cggm.h (compiled with gcc)."""
import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_struct_layouts_match(tmp_path):
    import paper_1509_04681_amd as m
    exe = tmp_path / "abi_layout"
    subprocess.run(["gcc", "-std=c11", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    os.path.join(ROOT, "tests", "cpp", "abi_layout.c"), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    c_lines = {ln for ln in out.splitlines() if ln}
    py_lines = set()
    for tag, st in (("req", m.Request), ("opt", m.Options), ("info", m.RequestInfo),
                    ("stats", m.ServerStats), ("trace", m.TraceEntry),
                    ("kstats", m.KernelStats)):
        for name, _ in st._fields_:
            if name != "_pad":
                py_lines.add(f"{tag} {name} {getattr(st, name).offset}")
        py_lines.add(f"{tag} size {ctypes.sizeof(st)}")
    assert c_lines == py_lines, (sorted(c_lines - py_lines), sorted(py_lines - c_lines))
