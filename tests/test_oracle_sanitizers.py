"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (g++ instrumentation, on the
host): oracle/sanitize_run.py drives every oracle entry point on small meshes of every element
and face kind, and the run must end without a sanitizer report.  The HIP library's host code
is not covered here (its calls need a device)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    if shutil.which("g++") is None:
        return None
    path = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_is_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("no g++ AddressSanitizer runtime")
    so = str(tmp_path / "liboracle_san.so")
    build = subprocess.run(
        ["g++", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", "-fno-fast-math", "-fno-omit-frame-pointer",
         "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
         "-o", so, os.path.join(ROOT, "oracle", "fr_oracle.cpp")],
        capture_output=True, text=True)
    assert build.returncode == 0, build.stderr[-3000:]
    env = dict(os.environ)
    env.update(LMFR_ORACLE_LIB=so, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1:exitcode=66",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=67")
    run = subprocess.run([sys.executable, os.path.join(ROOT, "oracle", "sanitize_run.py")], env=env,
                         capture_output=True, text=True, timeout=600)
    report = run.stderr[-4000:]
    assert run.returncode == 0, report
    assert "ERROR: AddressSanitizer" not in run.stderr and "runtime error:" not in run.stderr, report
    assert run.stdout.strip().endswith("ok"), run.stdout[-2000:]
