"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle is built a second time with -fsanitize=address,undefined (host
code; nothing here touches a GPU) and the oracle's own pin tests run against
that build in a child process with the sanitizer runtime preloaded: any
out-of-bounds access, use after free or undefined behaviour (signed
overflow, misaligned or null access, bad shift...) in the oracle aborts the
child and fails this test.  Leak checking is off: the child is a Python
interpreter, whose own allocations outlive it by design.
"""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PINS = ["tests/test_oracle_math.py", "tests/test_oracle_render.py", "tests/test_oracle_grad.py",
        "tests/test_oracle_recipe.py", "tests/test_oracle_models.py"]


def _runtime(name):
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True, check=True).stdout
    return out.strip()


@pytest.mark.slow
def test_oracle_pins_under_asan_and_ubsan():
    oracle.build(force=True, sanitize=True)
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    assert os.path.isabs(asan) and os.path.isabs(ubsan), "gcc has no sanitizer runtimes"
    env = dict(os.environ)
    env.update(LD_PRELOAD=f"{asan}:{ubsan}", FGS_ORACLE_LIB="sanitized", OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not slow",
                        *PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert " passed" in out
