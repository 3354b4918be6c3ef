"""The CPU test lane under sanitizers: the FP64 oracle built with g++
AddressSanitizer + UndefinedBehaviorSanitizer runs all its pins, and the C-ABI
library with its host code (argument validation, tables, sequencing) built
with clang's ASan + UBSan runs the ABI tests; each in a subprocess with the
matching ASan runtime preloaded.  Any report fails the subprocess."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(env_extra, args, timeout):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *args], cwd=ROOT,
                       env=env, capture_output=True, text=True, timeout=timeout)
    assert r.returncode == 0, (r.stdout[-3000:], r.stderr[-3000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, r.stderr[-3000:]
    return r.stdout


def test_oracle_pins_under_asan_ubsan():
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan):
        pytest.skip("gcc's libasan is not installed")
    subprocess.run([sys.executable, "-c", "import oracle; oracle.build()"], cwd=ROOT, check=True,
                   env=dict(os.environ, ORACLE_SANITIZE="1"))
    out = _run({"ORACLE_SANITIZE": "1", "LD_PRELOAD": asan}, ["tests/test_oracle_pins.py"], 1200)
    assert "passed" in out


def test_library_abi_under_asan_ubsan():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not os.path.exists(hipcc) or not rt:
        pytest.skip("hipcc or clang's ASan runtime is not installed")
    subprocess.run([sys.executable, "-m", "paper_2012_03939_amd.build", "--sanitize"], cwd=ROOT, check=True,
                   capture_output=True)
    out = _run({"SHAPETRACE_SANITIZE": "1", "LD_PRELOAD": rt[-1]}, ["tests/test_library_abi.py"], 600)
    assert "passed" in out
