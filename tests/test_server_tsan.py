"""ThreadSanitizer run of the serving scheduler on the host (no GPU): the
library's host sources are rebuilt with -fsanitize=thread (device code keeps
its normal build) and tests/native/server_threads.cpp drives the server from
several client threads while polling and cancelling; any data race reported
by ThreadSanitizer fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2202_04110_amd", "csrc")
KOBJ = os.path.join(ROOT, "paper_2202_04110_amd", "_build", "kernels.hip.o")
HOST = ["compile.cpp", "hostmem.cpp", "runtime.cpp", "api.cpp", "server.cpp"]


def test_scheduler_threads_under_tsan(tmp_path):
    if shutil.which("g++") is None or not os.path.exists(KOBJ):
        pytest.skip("needs g++ and the built kernel object (run the build first)")
    exe = str(tmp_path / "server_threads")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__",
           "-I/opt/rocm/include"] + [os.path.join(CSRC, f) for f in HOST] + \
          [os.path.join(ROOT, "tests", "native", "server_threads.cpp"), KOBJ,
           "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-lpthread", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "tsan" in (r.stderr or "").lower():
        pytest.skip("ThreadSanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 second_deadlock_stack=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, (r.stdout, r.stderr[-2000:])
