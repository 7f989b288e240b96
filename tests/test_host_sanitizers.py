"""Sanitizer runs of the library's host code (no GPU): the host sources are
rebuilt with ThreadSanitizer, or with AddressSanitizer and
UndefinedBehaviorSanitizer (device code keeps its normal build), and
tests/native/server_threads.cpp drives the serving scheduler from several
client threads while polling and cancelling, then runs concurrent graph
validation and layout checks; any sanitizer report fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2202_04110_amd", "csrc")
KOBJ = os.path.join(ROOT, "paper_2202_04110_amd", "_build", "kernels.hip.o")
HOST = ["compile.cpp", "hostmem.cpp", "runtime.cpp", "api.cpp", "server.cpp"]


@pytest.mark.parametrize("san", ["thread", "address,undefined"])
def test_scheduler_threads_under_sanitizers(tmp_path, san):
    if shutil.which("g++") is None or not os.path.exists(KOBJ):
        pytest.skip("needs g++ and the built kernel object (run the build first)")
    exe = str(tmp_path / "server_threads")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=" + san,
           "-ffp-contract=off", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"] + \
          [os.path.join(CSRC, f) for f in HOST] + \
          [os.path.join(ROOT, "tests", "native", "server_threads.cpp"), KOBJ,
           "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lamdhip64", "-lpthread", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and ("tsan" in r.stderr.lower() or "asan" in r.stderr.lower()):
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 second_deadlock_stack=1",
               ASAN_OPTIONS="detect_leaks=1 halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1 print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout)
    for word in ("ThreadSanitizer", "AddressSanitizer", "LeakSanitizer", "runtime error"):
        assert word not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, (r.stdout, r.stderr[-2000:])


def test_oracle_under_address_sanitizer(tmp_path):
    """The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
    runs its entry points (iterations with residuals, beliefs, single updates,
    scores, the reverse sweep) on trees, loopy and logical graphs cleanly."""
    if shutil.which("gcc") is None:
        pytest.skip("needs gcc")
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not asan or not os.path.isabs(asan):
        pytest.skip("libasan not found")
    lib = str(tmp_path / "liboracle_asan.so")
    r = subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fsanitize=address,undefined",
                        "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "lbp_oracle.c"), "-o", lib, "-lm"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    script = (
        "import numpy as np\n"
        "from oracle import OracleGraph\n"
        "from paper_2202_04110_amd import workloads as W\n"
        "gs = [W.random_factor_graph(3, num_vars=9, tree=True, max_arity=3, explicit_frac=0.4),\n"
        "      W.random_factor_graph(4, num_vars=14, tree=False, extra_factors=10, max_arity=4, logical_frac=0.3),\n"
        "      W.deconv(seed=4, K=2, tw=4, sd=8, img=10), W.potts_grid(6, 3, 2)]\n"
        "for i, g in enumerate(gs):\n"
        "    og = OracleGraph(g, lib_path=%r)\n"
        "    m, res = og.run(7, 0.5, 0.7, threads=2, residuals=True)\n"
        "    og.beliefs(m, 0.7); og.update(m, 0.0); og.score(np.zeros(og.V, np.int32))\n"
        "    if i in (0, 3):\n"
        "        og.backward(5, 0.5, 1.0, np.ones(og.VS))\n"
        "print('oracle ok')\n") % lib
    env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0 halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1 print_stacktrace=1",
               PYTHONPATH=ROOT + os.pathsep + os.environ.get("PYTHONPATH", ""))
    r = subprocess.run(["python3", "-c", script], capture_output=True, text=True, env=env, timeout=300, cwd=ROOT)
    for word in ("AddressSanitizer", "runtime error"):
        assert word not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0 and "oracle ok" in r.stdout, (r.stdout, r.stderr[-3000:])
