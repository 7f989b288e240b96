"""The host layout check (check_layout) rejects corrupted layouts: the native
program tests/native/layout_check.cpp compiles two graphs that between them
use every tile kind and variable path, checks that the clean layouts pass,
then corrupts one address, offset or table entry at a time (an edge row past
the message array, a belief row past the panel, a hedge range, a fused slot
variable, a three-way table entry, ...) and expects each to be rejected with
the matching message.  Host only, no GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2202_04110_amd", "csrc")


def test_layout_check_rejects_corruptions(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    exe = str(tmp_path / "layout_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           os.path.join(CSRC, "compile.cpp"), os.path.join(CSRC, "hostmem.cpp"),
           os.path.join(ROOT, "tests", "native", "layout_check.cpp"),
           "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0 and "layout check ok" in r.stdout, (r.stdout, r.stderr[-2000:])
