"""The oracle's pin suite under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): oracle.c is built a second time with -fsanitize=address,undefined
(liboracle_asan.so) and every tests/test_oracle_*.py pin runs against it in a
child pytest with the ASan runtime preloaded; any invalid access, overflow or
undefined behaviour in the oracle ends that run with an error."""
import os
import shutil
import subprocess
import sys

import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def _runtime(name):
    if shutil.which("gcc") is None:
        return None
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.asan
def test_oracle_pins_under_asan():
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc with the AddressSanitizer runtime is not available")
    lib = oracle.build(force=True, sanitize=True)
    files = sorted(f for f in os.listdir(HERE) if f.startswith("test_oracle_") and f.endswith(".py")
                   and f != os.path.basename(__file__))
    env = dict(os.environ, LD_PRELOAD=asan, ORACLE_LIB=lib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    # the planted-mistake tests build their own unsanitized copies; the rest is the pin suite
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not asan", "-k", "not planted",
           "-n", "4", *files]
    r = subprocess.run(cmd, cwd=HERE, env=env, capture_output=True, text=True, timeout=1200)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
    # the child really loaded the sanitized build
    probe = subprocess.run([sys.executable, "-c", "import sys; sys.path.insert(0, sys.argv[1]); import oracle; "
                            "print(oracle._load()._name)", ROOT], env=env, capture_output=True, text=True,
                           timeout=120)
    assert probe.stdout.strip() == lib, probe.stdout + probe.stderr
