"""Launch lists of several graphs: merging keeps every work item once, puts
all square pairwise tiles of 2..8 states into one mixed launch and the
variable tiles of buckets up to 8 into one launch, and leaves other classes
alone.  Host-only: a native program built against the in-tree liblbp.so."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2202_04110_amd")


def test_merged_launch_lists(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("needs g++")
    lib = os.path.join(PKG, "liblbp.so")
    if not os.path.exists(lib):
        pytest.skip("liblbp.so is not built")
    exe = str(tmp_path / "merge_lists")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           os.path.join(ROOT, "tests", "native", "merge_lists.cpp"),
           "-L" + PKG, "-Wl,-rpath," + PKG, "-llbp", "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64",
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0 and "merge lists ok" in r.stdout, (r.stdout, r.stderr[-2000:])
