"""The C-ABI library loads without a GPU and exports every entry point that
include/qs3.h declares; the product path refuses to run without it."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    hdr = open(os.path.join(ROOT, "include", "qs3.h")).read()
    return set(re.findall(r"^\s*(?:const char \*|int |double )\s*\**(qs3_\w+)\(", hdr, re.M))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["qs3_ctx_create", "qs3_lattice_create", "qs3_sector_create", "qs3_matvec", "qs3_eigs",
                 "qs3_sz", "qs3_sisj", "qs3_sq", "qs3_smq", "qs3_dsf", "qs3_batch_eigs", "qs3_submit"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2107_00872_amd import qs3
    if not os.path.exists(qs3.LIB_PATH):
        pytest.skip("libqs3.so not built")
    L = ctypes.CDLL(qs3.LIB_PATH)
    for name in _declared():
        assert hasattr(L, name), name
    assert {s[0] for s in qs3.SIGNATURES} == _declared()
    assert b"gfx950" in qs3.lib().qs3_version()
    assert qs3.lib().qs3_strerror(-3) == b"not converged"


def test_missing_library_fails_loudly(monkeypatch):
    from paper_2107_00872_amd import qs3
    monkeypatch.setattr(qs3, "LIB_PATH", "/nonexistent/libqs3.so")
    monkeypatch.setattr(qs3, "_lib", None)
    with pytest.raises(ImportError):
        qs3.lib()
