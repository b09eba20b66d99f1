"""Host AddressSanitizer + UndefinedBehaviorSanitizer build of the FP64 oracle (oracle.c) and
the native tile planner (csrc/plan.cpp), run on small inputs through tests/sanitize/driver.cpp:
no out-of-bounds access, leak-free use of the planner's containers aside (leak detection is
off: ptrace is not available everywhere), no undefined behaviour (signed overflow, bad
shifts, misaligned loads), and the planner's exact coverage of every pair."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


@pytest.mark.skipif(not (shutil.which("gcc") and shutil.which("g++")), reason="gcc/g++ not available")
def test_oracle_and_planner_under_asan_ubsan(tmp_path):
    rocm_inc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "include")
    if not os.path.isdir(os.path.join(rocm_inc, "hip")):
        pytest.skip("HIP headers not found (the planner uses its vector types)")
    o1, o2, o3 = (str(tmp_path / f) for f in ("oracle.o", "plan.o", "driver.o"))
    exe = str(tmp_path / "sanitized")
    cxx = ["g++", "-std=c++17", "-D__HIP_PLATFORM_AMD__", "-I" + rocm_inc, "-I" + os.path.join(ROOT, "include")]
    subprocess.check_call(["gcc", "-std=c11", "-fopenmp"] + SAN + ["-c", os.path.join(ROOT, "oracle", "oracle.c"), "-o", o1])
    subprocess.check_call(cxx + SAN + ["-c", os.path.join(ROOT, "paper_2009_04755_amd", "csrc", "plan.cpp"), "-o", o2])
    subprocess.check_call(cxx + SAN + ["-c", os.path.join(ROOT, "tests", "sanitize", "driver.cpp"), "-o", o3])
    subprocess.check_call(["g++", "-fopenmp"] + SAN + [o1, o2, o3, "-o", exe, "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.strip() == "ok"
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
