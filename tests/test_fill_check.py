"""Potential panels: every entry equals its factor's table value at that
configuration (zero where a lane has no factor), and non-finite table
values are rejected.
Host-only: a native program built against the in-tree liblbp.so."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2202_04110_amd")


def test_panels_hold_the_tables(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    lib = os.path.join(PKG, "liblbp.so")
    if not os.path.exists(lib):
        pytest.skip("liblbp.so is not built")
    exe = str(tmp_path / "fill_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           os.path.join(ROOT, "tests", "native", "fill_check.cpp"),
           "-L" + PKG, "-Wl,-rpath," + PKG, "-llbp", "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64",
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0 and "fill check ok" in r.stdout, (r.stdout, r.stderr[-2000:])
