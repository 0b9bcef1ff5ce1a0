"""The oracle's pins under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): the oracle's C source is built with both sanitizers
(oracle/build.py, host code, gcc) and every pin of the oracle and of the
network oracle runs against that build in a child process with the sanitizer
runtimes preloaded.  An out-of-bounds access, a use after free or undefined
behaviour in the oracle fails the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_pins_under_asan_and_ubsan():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc's sanitizer runtimes are not installed")
    from oracle import build
    lib = build.build(sanitize=True)
    # the sanitizer runtimes go first (ASan must lead the library list); anything the
    # environment already preloads stays preloaded after them
    pre = ":".join(x for x in (asan, ubsan, os.environ.get("LD_PRELOAD", "")) if x)
    env = dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=pre,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               OMP_NUM_THREADS="4")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
           os.path.join(ROOT, "tests", "test_oracle_pins.py"), os.path.join(ROOT, "tests", "test_cnn_oracle.py")]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    print(tail)
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
