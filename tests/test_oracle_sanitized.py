"""The oracle's pin tests with both oracle libraries built under
AddressSanitizer and UndefinedBehaviorSanitizer (gcc): any out-of-bounds
access, use after free or undefined behaviour in the oracle's C++ aborts the
run.  The tests run in a child process that preloads gcc's sanitizer
runtimes and points the oracle modules at the sanitized builds."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SUBSET = ["tests/test_oracle_pins.py", "tests/test_oracle_weno.py", "tests/test_oracle_rad.py",
          "tests/test_oracle_fld.py", "tests/test_oracle_opcount.py"]


def _runtime(name):
    r = subprocess.run(["g++", f"-print-file-name={name}"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_pins_under_asan_ubsan():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("gcc sanitizer runtimes not installed")
    sys.path.insert(0, ROOT)
    from oracle import build

    lib, fld_lib = build.build_sanitized()
    env = dict(os.environ, LD_PRELOAD=f"{asan} {ubsan}", ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1", HARD_ORACLE_LIB=lib,
               HARD_FLD_ORACLE_LIB=fld_lib)
    check = ("import oracle, oracle.fld as f; "
             "assert oracle.lib()._name.endswith('_asan.so'); "
             "assert f.lib()._name.endswith('_asan.so')")
    r = subprocess.run([sys.executable, "-c", check], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu"] + SUBSET, cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=1200)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
