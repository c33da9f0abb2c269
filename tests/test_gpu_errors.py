"""Error paths of the C ABI, forced from the host through ctypes: every
declared status code that a caller can provoke with bad input or limits.
Nothing here launches a kernel on invalid data -- validation happens on the
host before any device work, and the numerical cases feed finite-size NaN or
zero vectors that the kernels process as ordinary numbers."""
import ctypes

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


def _lattice_rc(qs3, ctx, lx, ly, lz, bi, bj, jxy, jz, ns=1):
    bi = np.ascontiguousarray(bi, dtype=np.int32)
    bj = np.ascontiguousarray(bj, dtype=np.int32)
    jxy = np.ascontiguousarray(jxy, dtype=np.float64)
    jz = np.ascontiguousarray(jz, dtype=np.float64)
    h = ctypes.c_void_p()
    rc = qs3.lib().qs3_lattice_create_cells(ctx.h, ns, lx, ly, lz, len(bi), bi.ctypes.data, bj.ctypes.data,
                                            jxy.ctypes.data, jz.ctypes.data, ctypes.byref(h))
    return rc, h


def _msg(qs3):
    return qs3.lib().qs3_last_error().decode()


def test_lattice_create_rejects_bad_bonds(qs3, ctx):
    lat = wl.chain(8)
    cases = [
        (dict(bi=[0, 8], bj=[1, 2]), "out of range"),       # site 8 on an 8-site chain
        (dict(bi=[0, -1], bj=[1, 2]), "out of range"),
        (dict(bi=[0, 3], bj=[1, 3]), "i == j"),
        (dict(jxy=[1.0, np.nan]), "non-finite"),
        (dict(jz=[np.inf, 1.0]), "non-finite"),
    ]
    for over, text in cases:
        args = dict(bi=lat.bi[:2], bj=lat.bj[:2], jxy=lat.jxy[:2], jz=lat.jz[:2])
        args.update(over)
        rc, h = _lattice_rc(qs3, ctx, 8, 1, 1, **args)
        assert rc == qs3.QS3_EINVAL and h.value is None
        assert text in _msg(qs3)
    rc, h = _lattice_rc(qs3, ctx, 0, 1, 1, [], [], [], [])
    assert rc == qs3.QS3_EINVAL and "lengths" in _msg(qs3)
    rc, h = _lattice_rc(qs3, ctx, 4, 1, 1, [], [], [], [], ns=5)
    assert rc == qs3.QS3_EINVAL and "unit cell" in _msg(qs3)
    rc, h = _lattice_rc(qs3, ctx, 64, 64, 2, [], [], [], [])
    assert rc == qs3.QS3_EINVAL and "4096" in _msg(qs3)
    assert qs3.lib().qs3_strerror(qs3.QS3_EINVAL) == b"invalid argument"


def test_sector_and_batch_create_reject_bad_input(qs3, ctx):
    L = qs3.Lattice.of(ctx, wl.square(4))
    dis = qs3.Lattice.of(ctx, wl.with_disorder(wl.square(4), seed=3))   # per-bond disorder
    h = ctypes.c_void_p()
    lib = qs3.lib()
    # N_down out of range
    assert lib.qs3_sector_create(L.h, 17, None, ctypes.byref(h)) == qs3.QS3_EINVAL
    assert lib.qs3_sector_create(L.h, -1, None, ctypes.byref(h)) == qs3.QS3_EINVAL
    assert h.value is None
    # momentum index out of range along each axis
    for kv in [(4, 0, 0), (0, 4, 0), (0, 0, 1), (-1, 0, 0)]:
        k = np.array(kv, dtype=np.int32)
        assert lib.qs3_sector_create(L.h, 2, k.ctypes.data, ctypes.byref(h)) == qs3.QS3_EINVAL
        assert "momentum index" in _msg(qs3) and h.value is None
    # k on a bond set that is not translation invariant
    k = np.zeros(3, dtype=np.int32)
    assert lib.qs3_sector_create(dis.h, 2, k.ctypes.data, ctypes.byref(h)) == qs3.QS3_EINVAL
    assert "translation-invariant" in _msg(qs3)
    assert dis.info()[1] == 0
    # but its fixed-N_down sector is fine
    sec = qs3.Sector(dis, 2)
    assert sec.dim == 120
    sec.close()
    # batches: count and momenta
    kk = np.zeros(3 * 2049, dtype=np.int32)
    assert lib.qs3_batch_create(L.h, 2, 2049, kk.ctypes.data, ctypes.byref(h)) == qs3.QS3_EINVAL
    assert lib.qs3_batch_create(L.h, 2, 0, kk.ctypes.data, ctypes.byref(h)) == qs3.QS3_EINVAL
    kk = np.array([0, 0, 0, 1, 5, 0], dtype=np.int32)
    assert lib.qs3_batch_create(L.h, 2, 2, kk.ctypes.data, ctypes.byref(h)) == qs3.QS3_EINVAL
    assert h.value is None
    with pytest.raises(qs3.QS3Error) as e:
        qs3.Batch(dis, 2, [(0, 0, 0)])
    assert e.value.code == qs3.QS3_EINVAL


def test_matvec_rejects_dtype_and_aliasing(qs3, ctx):
    L = qs3.Lattice.of(ctx, wl.chain(10))
    u1 = qs3.Sector(L, 3)
    ks = qs3.Sector(L, 3, (1, 0, 0))
    v = torch.zeros(u1.dim, dtype=torch.float64, device="cuda")
    vc = torch.zeros(ks.dim, dtype=torch.complex128, device="cuda")
    lib = qs3.lib()
    w = torch.zeros_like(v)
    # a complex vector for a real sector and vice versa, and v == w
    assert lib.qs3_matvec(u1.h, v.data_ptr(), w.data_ptr(), qs3.C128, None) == qs3.QS3_EINVAL
    assert lib.qs3_matvec(ks.h, vc.data_ptr(), vc.data_ptr() + 16, qs3.F64, None) == qs3.QS3_EINVAL
    assert lib.qs3_matvec(u1.h, v.data_ptr(), v.data_ptr(), qs3.F64, None) == qs3.QS3_EINVAL
    assert "alias" in _msg(qs3)
    u1.close()
    ks.close()


def test_eigs_enoconv_keeps_partial_results(qs3, ctx):
    """One thick restart cannot converge a 10x10 N_down = 3 solve at tol 1e-14:
    QS3_ENOCONV, info.converged == 0, and the returned levels are the current
    Ritz estimates (finite, above the true lowest level, which the default
    solve reaches)."""
    L = qs3.Lattice.of(ctx, wl.square(10))
    sec = qs3.Sector(L, 3)
    r = sec.eigs(nev=2, max_restarts=1, tol=1e-14, seed=3)
    assert r.status == qs3.QS3_ENOCONV and r.info.converged == 0 and r.info.n_restarts == 1
    assert np.all(np.isfinite(r.evals)) and r.info.max_residual > 0
    full = sec.eigs(nev=2, seed=3)
    assert full.status == qs3.QS3_OK and full.info.converged == 1
    assert r.evals[0] >= full.evals[0] - 1e-9
    assert qs3.lib().qs3_strerror(qs3.QS3_ENOCONV) == b"not converged"
    # the same through the batch entry point: every column reports
    bat = qs3.Batch(L, 3, [(0, 0, 0), (1, 0, 0)])
    ev, infos, rc = bat.eigs(nev=1, max_restarts=1, tol=1e-14, seed=3)
    assert rc == qs3.QS3_ENOCONV and all(i.converged == 0 for i in infos)
    assert np.all(np.isfinite(ev))
    bat.close()
    sec.close()


def test_lanczos_enumeric_from_nan_or_zero_start(qs3, ctx):
    L = qs3.Lattice.of(ctx, wl.chain(12))
    sec = qs3.Sector(L, 3)
    lib = qs3.lib()
    steps = 10
    for bad in [float("nan"), 0.0]:
        v0 = torch.full((sec.dim,), bad, dtype=torch.float64, device="cuda")
        if bad != bad:
            v0[1:] = 1.0      # one NaN element
        a = np.full(steps, 7.0)
        b = np.full(steps, 7.0)
        n0 = ctypes.c_double(7.0)
        done = ctypes.c_int(-1)
        rc = lib.qs3_lanczos(sec.h, v0.data_ptr(), steps, qs3.PREC_F64, qs3.REORTH_FULL, 1, a.ctypes.data,
                             b.ctypes.data, ctypes.byref(n0), ctypes.byref(done), None)
        assert rc == qs3.QS3_ENUMERIC
        assert "start vector" in _msg(qs3)
        assert np.all(a == 7.0) and np.all(b == 7.0) and n0.value == 7.0 and done.value == -1
    # a finite start vector is fine
    a, b, n0, done = sec.lanczos(steps)
    assert np.all(np.isfinite(a)) and done == steps
    assert qs3.lib().qs3_strerror(qs3.QS3_ENUMERIC) == b"numerical failure"
    sec.close()


def test_eigs_rejects_bad_options(qs3, ctx):
    L = qs3.Lattice.of(ctx, wl.chain(10))
    sec = qs3.Sector(L, 2)
    for kw, text in [(dict(nev=17), "nev"), (dict(precision=7), "precision"), (dict(reorth=9), "reorth"),
                     (dict(alg=5), "algorithm"), (dict(reorth=qs3.REORTH_NONE), "thick restart")]:
        with pytest.raises(qs3.QS3Error) as e:
            sec.eigs(**kw)
        assert e.value.code == qs3.QS3_EINVAL and text in str(e.value), (kw, str(e.value))
    sec.close()
