"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two builds, each exercised by its own tests in a child process (the gcc and
clang runtimes cannot share one process):

* the FP64 oracle built by gcc with -fsanitize=address,undefined, running the
  oracle's pins (trees, probability-domain BP, closed forms, exhaustive small
  codes, AEWA and serial schedule, wide codes);
* the library's host ABI layer (graph construction, argument checks, launch
  set-up) built by hipcc with -fsanitize=address,undefined for the host pass,
  running the ABI tests.

Any sanitizer report aborts the child (halt_on_error), which fails the test.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OPTS = {"ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1", "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _child(env_extra, tests):
    env = dict(os.environ, **OPTS, **env_extra)
    preload = env_extra["LD_PRELOAD"]
    if os.environ.get("LD_PRELOAD"):            # keep whatever the environment preloads
        preload += ":" + os.environ["LD_PRELOAD"]
    env["LD_PRELOAD"] = preload
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider"] + tests,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout


def test_oracle_under_asan_ubsan():
    if not shutil.which("gcc"):
        pytest.skip("gcc missing")
    libs = [subprocess.run(["gcc", "-print-file-name=" + n], capture_output=True, text=True).stdout.strip()
            for n in ("libasan.so", "libubsan.so")]
    if not all(os.path.isabs(x) and os.path.exists(x) for x in libs):
        pytest.skip("gcc sanitizer runtimes missing")
    env = {"BP4_ORACLE_SANITIZE": "1", "OMP_NUM_THREADS": "4", "LD_PRELOAD": ":".join(libs)}
    subprocess.run([sys.executable, "-c", "from oracle import oracle as O; O.build(force=True)"], cwd=ROOT,
                   env=dict(os.environ, BP4_ORACLE_SANITIZE="1"), check=True)
    _child(env, ["tests/test_oracle_pins.py", "tests/test_aewa_pins.py", "tests/test_serial_pins.py",
                 "tests/test_wide_codes.py"])


def test_abi_layer_under_asan_ubsan():
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt or not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc or clang's ASan runtime missing")
    from paper_2407_11523_amd import build as B
    B.build_sanitized()
    _child({"BP4_SANITIZE": "1", "LD_PRELOAD": rt[-1]}, ["tests/test_abi.py"])
