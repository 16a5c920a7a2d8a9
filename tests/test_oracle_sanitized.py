"""The oracle's pins again, with the oracle built under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only): an out-of-bounds access, a use of freed
memory or undefined arithmetic in the C oracle aborts the run.

The instrumented library is built into a temporary directory and loaded by a
child pytest process (DG_ORACLE_LIB), with the ASan runtime preloaded because
the Python interpreter itself is not instrumented.  Leak detection is off: the
interpreter's own allocations outlive it by design."""
import os
import subprocess
import sys

import pytest

import oracle
from oracle import build as ob

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FILES = ["test_oracle_basis.py", "test_oracle_operator.py", "test_oracle_riemann_exact.py",
         "test_oracle_limiter.py", "test_oracle_isothermal.py", "test_oracle_forcing_closure.py",
         "test_oracle_diagnostics.py"]


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.slow
def test_oracle_pins_under_asan_ubsan(tmp_path):
    asan = _runtime("libasan.so")
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    lib = str(tmp_path / "liboracle_san.so")
    ob.build(out=lib, extra=("-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                             "-fno-sanitize-recover=undefined"))
    env = dict(os.environ)
    env.update(DG_ORACLE_LIB=lib, LD_PRELOAD=asan, OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-s", "-p", "no:cacheprovider", "-m", "not gpu and not slow"]
    cmd += [os.path.join(ROOT, "tests", f) for f in FILES]
    # -s: a sanitizer report goes to the child's stderr as it happens, not into pytest's capture
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout[-2000:] + "\n" + r.stderr[:3000])
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
    assert " passed" in r.stdout, tail
    # the child really loaded the instrumented build
    assert oracle is not None
