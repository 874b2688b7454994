"""The oracle and the library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

* The oracle (plain C) is compiled by gcc with both sanitizers and loaded in a
  Python process that preloads gcc's ASan runtime; its CPU pin tests of the
  pair forces, white noise, observables, pressure and barostat must pass with
  no report (every report is fatal).
* libqtb.so is compiled with the sanitizers on its host pass (the GPU code is
  unchanged) and loaded in a process that preloads clang's ASan runtime; the
  host-side tests (argument checks and workspace plan, exported symbols, the
  FIR design on the host) must pass with no report.
Leak detection is off: the Python interpreter itself does not free
everything at exit.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_TESTS = ["tests/test_oracle_forces.py", "tests/test_oracle_noise.py",
                "tests/test_oracle_observe.py", "tests/test_oracle_pressure.py",
                "tests/test_oracle_barostat.py", "tests/test_oracle_abi.py"]
HOST_TESTS = ["tests/test_host_layout.py", "tests/test_abi.py", "tests/test_host_filter.py"]
SAN_ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
           "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}


def _gcc_runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _pytest(files, env):
    e = dict(os.environ, **SAN_ENV, **env)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu", *files], cwd=ROOT, env=e, capture_output=True,
                       text=True, timeout=1200)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
    return tail


def test_oracle_under_asan_and_ubsan(tmp_path):
    from oracle import oracle
    asan, ubsan = _gcc_runtime("libasan.so"), _gcc_runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    so = oracle.build_sanitized(str(tmp_path))
    out = _pytest(ORACLE_TESTS, {"QTB_ORACLE_LIB": so, "LD_PRELOAD": f"{asan} {ubsan}"})
    assert " passed" in out


def test_library_host_code_under_asan_and_ubsan():
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt:
        pytest.skip("clang ASan runtime not installed")
    from paper_1905_02521_amd import build
    so = build.build(jobs=8, sanitize=True)
    out = _pytest(HOST_TESTS, {"QTB_LIB": so, "LD_PRELOAD": rt[-1]})
    assert " passed" in out
