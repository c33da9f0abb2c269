"""qs3_matvec_noalloc (the allocation-free product) against qs3_matvec through
the C ABI: bit-identical results on two calls in a row, the second on a
smaller sector (the device array keeps the first call's contents), in
complex128 and complex64 and on a fixed-N_down sector; no device memory is
taken by the calls; a sector beyond the array's size is refused before any
launch."""
import math

import numpy as np
import pytest

import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qs3():
    from paper_2107_00872_amd import qs3 as q
    assert torch.cuda.is_available()
    return q


@pytest.fixture(scope="module")
def ctx(qs3):
    return qs3.Context(0)


def _noalloc(qs3, sec, v, w):
    return qs3.lib().qs3_matvec_noalloc(sec.h, v.data_ptr(), w.data_ptr(), qs3._dtype_code(v),
                                        torch.cuda.current_stream().cuda_stream)


def _pair(qs3, sec, dtype, seed):
    """(w from qs3_matvec, w from qs3_matvec_noalloc) on one seeded input."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    if dtype.is_complex:
        re = torch.rand(sec.dim, generator=g, dtype=torch.float64) * 2 - 1
        im = torch.rand(sec.dim, generator=g, dtype=torch.float64) * 2 - 1
        v = torch.complex(re, im).to(dtype).cuda()
    else:
        v = (torch.rand(sec.dim, generator=g, dtype=torch.float64) * 2 - 1).to(dtype).cuda()
    w_ref = torch.full_like(v, float("nan"))
    sec.matvec(v, w_ref)
    w = torch.full_like(v, float("nan"))
    used0 = ctx_used(qs3, sec)
    assert _noalloc(qs3, sec, v, w) == qs3.QS3_OK
    torch.cuda.synchronize()
    assert ctx_used(qs3, sec) == used0          # nothing allocated through the library
    return w_ref.cpu(), w.cpu()


def ctx_used(qs3, sec):
    import ctypes
    used, budget = ctypes.c_uint64(), ctypes.c_uint64()
    qs3.lib().qs3_ctx_memory(sec.lattice.ctx.h, ctypes.byref(used), ctypes.byref(budget))
    return used.value


@pytest.mark.parametrize("dtype", ["complex128", "complex64"])
def test_noalloc_matches_matvec_two_calls(qs3, ctx, dtype):
    dt = getattr(torch, dtype)
    big = qs3.Sector(qs3.Lattice.of(ctx, wl.square(10)), 4, (1, 0, 0))
    small = qs3.Sector(qs3.Lattice.of(ctx, wl.square(6)), 2, (3, 0, 0))
    # the union of representatives (= the k = 0 basis) is larger than each
    # sector's basis, so the scratch path runs
    for sec in (big, small):
        k0 = qs3.Sector(sec.lattice, sec.n_down, (0, 0, 0))
        assert sec.dim < k0.dim
        k0.close()
    assert big.dim == 39200
    for sec, seed in ((big, 1), (small, 2), (big, 3)):
        ref, got = _pair(qs3, sec, dt, seed)
        assert torch.equal(ref, got), (sec.dim, dtype)
        assert not torch.isnan(got).any()
    big.close()
    small.close()


def test_noalloc_fixed_n_down_and_full_union(qs3, ctx):
    """No scratch needed: a fixed-N_down sector and a momentum sector whose
    basis is the whole union (10^3 cube, N_down = 2, all orbits full)."""
    u1 = qs3.Sector(qs3.Lattice.of(ctx, wl.chain(20)), 5)
    ref, got = _pair(qs3, u1, torch.float64, 4)
    assert torch.equal(ref, got)
    ref, got = _pair(qs3, u1, torch.float32, 5)
    assert torch.equal(ref, got)
    full = qs3.Sector(qs3.Lattice.of(ctx, wl.cube(10)), 2, (1, 2, 3))
    ref, got = _pair(qs3, full, torch.complex128, 6)
    assert torch.equal(ref, got)
    u1.close()
    full.close()


def test_noalloc_refuses_too_large_sector(qs3, ctx):
    """12 x 12 square, N_down = 5: 3,340,337 representatives (every orbit full).
    complex64 needs the array (the kernel's float64 row copies): refused
    with QS3_EINVAL and a message, the output untouched; complex128 needs no
    scratch and runs."""
    sec = qs3.Sector(qs3.Lattice.of(ctx, wl.square(12)), 5, (1, 0, 0))
    assert sec.dim == math.comb(144, 5) // 144 and sec.dim > 2_097_152
    v = torch.ones(sec.dim, dtype=torch.complex64, device="cuda")
    w = torch.full_like(v, 7.0)
    assert _noalloc(qs3, sec, v, w) == qs3.QS3_EINVAL
    assert "too large" in qs3.lib().qs3_last_error().decode()
    torch.cuda.synchronize()
    assert bool((w == 7.0).all())
    ref, got = _pair(qs3, sec, torch.complex128, 7)
    assert torch.equal(ref, got)
    sec.close()
