"""The library's host code under AddressSanitizer and UBSan on a GPU.

paper_2107_00872_amd/qs3_host_check (built by build(): every library source
with the host-code sanitizers, device code unchanged, linked with
tests/host_abi_check.cpp) drives the C-ABI's host paths -- argument
validation, structure builds, the solvers' restart control and Ritz
eigensolver, observables, S(q, omega), batches, point-group sectors and the
serving scheduler with refusal and cancellation.  Any sanitizer report aborts
it (leaks included, apart from the ROCm runtime's own); it exits 0 only when
all its consistency checks hold.
"""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "paper_2107_00872_amd", "qs3_host_check")


def test_host_code_under_asan_ubsan():
    assert os.path.exists(EXE), "qs3_host_check is not built (paper_2107_00872_amd.build.build_host_check)"
    env = dict(os.environ)
    # leaks are checked too, except those of the ROCm runtime's own allocations
    env.update({"ASAN_OPTIONS": "detect_leaks=1:halt_on_error=1",
                "LSAN_OPTIONS": "suppressions=" + os.path.join(ROOT, "tests", "lsan_rocm.supp"),
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    print("running qs3_host_check", flush=True)
    r = subprocess.run([EXE], env=env, capture_output=True, text=True, timeout=240)
    out = r.stdout + r.stderr
    assert "Sanitizer" not in out and "runtime error:" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    assert "host ABI check: ok" in out
