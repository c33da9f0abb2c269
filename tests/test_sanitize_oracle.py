"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle's C routines are built with -fsanitize=address,undefined (any
report aborts) and the CPU tests that call them -- the pins of the C oracle
against the Python oracle, bitmask matrices, Burnside dimensions, the
scatter form of S^-_q and the cached-structure variant -- run again in a child
process that loads that build.  The child preloads the ASan runtime because
the Python interpreter itself is not instrumented; leak checking is off (the
interpreter's own allocations at exit are not the oracle's).
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_TESTS = ["tests/test_oracle_native.py", "tests/test_oracle_basis.py",
                "tests/test_oracle_hamiltonian.py", "tests/test_oracle_solvers.py"]


def _asan_runtime():
    try:
        p = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True,
                           check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.slow
def test_c_oracle_under_asan_ubsan(tmp_path):
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("gcc's ASan runtime is not installed")
    sys.path.insert(0, ROOT)
    from oracle import native
    lib = native.build_sanitized(str(tmp_path / "libqs3_oracle_asan.so"))
    env = dict(os.environ)
    env.update({"QS3_ORACLE_LIB": lib, "LD_PRELOAD": rt, "OMP_NUM_THREADS": "2",
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:halt_on_error=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *ORACLE_TESTS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
