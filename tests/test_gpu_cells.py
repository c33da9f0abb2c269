"""Momentum sectors on lattices with several sites per unit cell (kagome,
honeycomb, pyrochlore): translations act on the cells.  Representatives and stabilisers
bit-exact against the oracle's Alg. 5/6 over the cell translations, H.v and
the dense block against the oracle's Alg. 8 block, the batched launch over
all momenta, eigensolvers against dense diagonalisation, and the entry points
that need one site per cell refuse."""
import numpy as np
import pytest

import workloads as wl
from oracle.hamiltonian import bonds_1based
from oracle.lanczos import lowest_distinct
from oracle.translation import Geometry, gen_full_ham_sym_adapt, mk_list
from tolerances import hv_tol

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CELLS = [(wl.kagome(2, 2), 3), (wl.kagome(2, 2), 4), (wl.honeycomb(3, 2), 3), (wl.kagome(3, 3), 2),
         (wl.pyrochlore(2), 3), (wl.pyrochlore(2), 2),
         (wl.honeycomb(2, 2), 0), (wl.with_disorder(wl.kagome(2, 3), seed=6, per_bond=False), 3)]


@pytest.fixture(scope="module")
def qs3():
    from paper_2107_00872_amd import qs3 as q
    assert torch.cuda.is_available()
    return q


def _contexts(qs3):
    c_tab = qs3.Context(0)
    c_tab.set_structure_limits(1 << 34, 0)
    c_hops = qs3.Context(0)
    c_hops.set_structure_limits(0, 1 << 34)
    c_fly = qs3.Context(0)
    c_fly.set_structure_limits(0, 0)
    return {"table": c_tab, "hops": c_hops, "fly": c_fly}


_REF = {}


def _oracle(lat, K):
    key = (lat.name, K)
    if key not in _REF:
        geo = Geometry(lat.lx, lat.ly, lat.lz, lat.ns)
        bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
        out = {}
        for Kv in wl.all_momenta(lat):
            s, R = mk_list(geo, K, Kv)
            H = gen_full_ham_sym_adapt(geo, K, bonds, s, R, Kv) if s else None
            out[Kv] = (np.array(s, dtype=np.int64), np.array(R), H)
        _REF[key] = (geo, out)
    return _REF[key]


@pytest.mark.parametrize("mode", ["table", "hops", "fly"])
@pytest.mark.parametrize("lat,K", CELLS, ids=lambda x: getattr(x, "name", str(x)))
def test_cells_basis_matvec_dense(qs3, lat, K, mode):
    ctx = _contexts(qs3)[mode]
    L = qs3.Lattice.of(ctx, lat)
    assert L.info() == (lat.n_sites, True)
    geo, ref = _oracle(lat, K)
    scale = max(1.0, float(np.abs(lat.jxy).max()), float(np.abs(lat.jz).max()))
    for Kv, (sigma, R, Hk) in ref.items():
        if len(sigma) == 0:
            continue
        sec = qs3.Sector(L, K, Kv)
        assert sec.dim == len(sigma)
        ranks, stab = sec.basis()
        assert np.array_equal(ranks, sigma - 1)
        assert np.allclose(R * R, geo.NT * stab.astype(float), rtol=0, atol=1e-9)
        v = torch.empty(sec.dim, dtype=torch.complex128, device="cuda")
        sec.start_vector(3, v)
        w = torch.empty_like(v)
        sec.matvec(v, w)
        vh = v.cpu().numpy()
        assert np.abs(w.cpu().numpy() - Hk @ vh).max() <= hv_tol(lat, np.abs(vh).max() * 1.5)
        D = sec.dense().cpu().numpy().T  # column major
        assert np.abs(D - Hk).max() <= 1e-13 * scale * 8
        sec.close()
    L.close()


@pytest.mark.parametrize("lat,K", CELLS[:5], ids=lambda x: getattr(x, "name", str(x)))
def test_cells_batch_and_eigs(qs3, lat, K):
    """All momenta in one batched launch equal the single sectors; lowest two
    distinct levels per sector (batched thick restart) and the sector spectra
    (full diagonalisation) against the oracle's blocks."""
    ctx = qs3.Context(0)
    L = qs3.Lattice.of(ctx, lat)
    geo, ref = _oracle(lat, K)
    ks = wl.all_momenta(lat)
    bat = qs3.Batch(L, K, ks)
    rng = np.random.default_rng(4)
    vh = rng.normal(size=(bat.rows, bat.B)) + 1j * rng.normal(size=(bat.rows, bat.B))
    v = torch.from_numpy(vh).cuda()
    w = torch.empty_like(v)
    bat.matvec(v, w)
    wh = w.cpu().numpy()
    sec0 = qs3.Sector(L, K, (0, 0, 0))
    uni, _ = sec0.basis()
    sec0.close()
    for b, Kv in enumerate(ks):
        sigma, R, Hk = ref[Kv]
        assert bat.dims[b] == len(sigma)
        if len(sigma) == 0:
            continue
        pos = np.searchsorted(uni, sigma - 1)
        assert np.array_equal(uni[pos], sigma - 1)
        assert np.abs(wh[pos, b] - Hk @ vh[pos, b]).max() <= hv_tol(lat, np.abs(vh).max() * 1.5)
    ev, infos, rc = bat.eigs(nev=2, seed=5)
    assert rc == qs3.QS3_OK
    for b, Kv in enumerate(ks):
        sigma, R, Hk = ref[Kv]
        if len(sigma) == 0:
            continue
        full = np.linalg.eigvalsh(Hk)
        want = lowest_distinct(full, 2)
        got = ev[b, :len(want)]
        assert np.allclose(got, want, rtol=1e-10, atol=1e-10), (Kv, got, want)
        sec = qs3.Sector(L, K, Kv)
        assert np.abs(sec.full_diag() - full).max() < 1e-11 * max(1.0, np.abs(full).max())
        sec.close()
    bat.close()


@pytest.mark.parametrize("lat,K", [(wl.kagome(2, 2), 3), (wl.honeycomb(3, 2), 3), (wl.kagome(2, 2), 4),
                                   (wl.pyrochlore(2), 2)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_cells_observables_vs_oracle(qs3, lat, K):
    """<S^z_i>, <S^z_i S^z_j>, <S^+_i S^-_j> and S(q) (positions with the places'
    offsets) of momentum-sector states against the oracle's U(1) observables
    of the same states expanded by Eq. (akstate) (a momentum eigenstate's
    correlations are translation invariant, so the translation-averaged
    values are the plain ones); the fixed-N_down sector's S(q) against the
    oracle's with the same positions."""
    from oracle.observables import corr_pm, corr_zz, structure_factors, sz
    from oracle.translation import expand_to_u1
    ctx = qs3.Context(0)
    L = qs3.Lattice.of(ctx, lat)
    geo, ref = _oracle(lat, K)
    N = lat.n_sites
    R = np.zeros((N, 3))
    for i in range(N):
        s_, c = i % lat.ns, i // lat.ns
        R[i] = (c % lat.lx, (c // lat.lx) % lat.ly, c // (lat.lx * lat.ly))
        R[i] += lat.basis[s_]
    # momenta of the cell lattice (the translation-averaged form sums over
    # displacements within one period, so S(q) of a momentum sector is taken
    # on this grid), plus a point off the grid for the fixed-N_down sector
    qs = np.array([[2 * np.pi * kx / lat.lx, 2 * np.pi * ky / lat.ly, 2 * np.pi * kz / lat.lz]
                   for (kx, ky, kz) in wl.all_momenta(lat)])
    qs_off = np.vstack([qs, [[1.3, -0.7, 0.4]]])
    pi = [i for i in range(N) for j in range(N)]
    pj = [j for i in range(N) for j in range(N)]
    for Kv in list(ref)[:4]:
        sigma, Rk, Hk = ref[Kv]
        if len(sigma) == 0:
            continue
        sec = qs3.Sector(L, K, Kv)
        X = torch.empty(sec.dim, dtype=torch.complex128, device="cuda")
        sec.eigs(nev=1, evecs=X, seed=2)
        phi = X.cpu().numpy()
        u1 = expand_to_u1(geo, K, list(sigma), list(Rk), Kv, phi)
        rsz, rzz, rpm = sz(u1, N, K), corr_zz(u1, N, K), corr_pm(u1, N, K)
        assert np.abs(sec.sz(X) - rsz).max() < 1e-12
        zz, pm = sec.sisj(X, pi, pj)
        assert np.abs(zz - rzz.reshape(-1)).max() < 1e-12
        assert np.abs(pm - rpm.reshape(-1)).max() < 1e-12
        szz, spm, stot = sec.sq(X, qs)
        rs = structure_factors(rzz, rpm, rsz, R, qs)
        assert np.abs(szz - rs[:, 0]).max() < 1e-11
        assert np.abs(spm - rs[:, 1]).max() < 1e-11
        assert np.abs(stot - rs[:, 2]).max() < 1e-11
        sec.close()
    u1s = qs3.Sector(L, K)
    x = torch.empty(u1s.dim, dtype=torch.float64, device="cuda")
    u1s.eigs(nev=1, evecs=x, seed=1)
    ph = x.cpu().numpy()
    szz, spm, stot = u1s.sq(x, qs_off)
    rs = structure_factors(corr_zz(ph, N, K), corr_pm(ph, N, K), sz(ph, N, K), R, qs_off)
    assert np.abs(np.stack([szz, spm, stot], 1) - rs).max() < 1e-11


@pytest.mark.parametrize("op", ["-", "+", "z"])
@pytest.mark.parametrize("lat,K", [(wl.kagome(2, 2), 2), (wl.honeycomb(2, 2), 3), (wl.kagome(2, 3), 1),
                                   (wl.pyrochlore(2), 2)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_cells_sq_gather_vs_oracle(qs3, lat, K, op):
    """S^-_q, S^+_q and S^z_q between momentum sectors of a lattice with several
    sites per cell (positions with the places' offsets): the device's gather
    against the oracle's scatter for every q."""
    from oracle.dynamics import n_down_after, sq_to_vec
    code = {"-": qs3.OP_SMINUS, "+": qs3.OP_SPLUS, "z": qs3.OP_SZ}[op]
    ctx = qs3.Context(0)
    L = qs3.Lattice.of(ctx, lat)
    geo = Geometry(lat.lx, lat.ly, lat.lz, lat.ns, lat.basis)
    K1 = n_down_after(op, K)
    for Kv in wl.all_momenta(lat)[:3]:
        s_, R = mk_list(geo, K, Kv)
        if not s_:
            continue
        src = qs3.Sector(L, K, Kv)
        rng = np.random.default_rng(13)
        phi = rng.normal(size=len(s_)) + 1j * rng.normal(size=len(s_))
        X = torch.from_numpy(phi).cuda()
        for Qv in wl.all_momenta(lat):
            kq = tuple((Kv[a] + Qv[a]) % lat.dims[a] for a in range(3))
            s1, R1 = mk_list(geo, K1, kq)
            if not s1:
                continue
            dst = qs3.Sector(L, K1, kq)
            out = torch.empty(dst.dim, dtype=torch.complex128, device="cuda")
            src.sq_apply(X, dst, code, Qv, out)
            ref = sq_to_vec(geo, K, s_, R, Kv, phi, s1, R1, Qv, op)
            scale = np.abs(phi).max() * max(1, lat.n_sites if op != "-" else K + 1)
            assert np.abs(out.cpu().numpy() - ref).max() < 1e-13 * scale, (Kv, Qv)
            dst.close()
        src.close()


def test_cells_dsf_vs_oracle(qs3):
    """S^-(q, omega) on the 2x2 kagome cluster from its N_down = 1 ground state,
    all 4 q, 20 levels: weights, Lanczos coefficients and the continued
    fraction against the oracle (S^-_q by the scatter, Lanczos on the dense
    k + q blocks).  (The one-site sum rule sum_q S^{+-}(q) = N - K does not
    carry over: within a cell the places' offsets leave q-dependent phases.)"""
    from oracle.dynamics import continued_fraction, sq_to_vec
    from oracle.lanczos import lanczos as orc_lanczos
    ctx = qs3.Context(0)
    lat = wl.kagome(2, 2)
    L = qs3.Lattice.of(ctx, lat)
    geo = Geometry(lat.lx, lat.ly, lat.lz, lat.ns, lat.basis)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    ks = wl.all_momenta(lat)
    K = 1
    best = None
    for Kv in ks:
        s_, R = mk_list(geo, K, Kv)
        e = np.linalg.eigvalsh(gen_full_ham_sym_adapt(geo, K, bonds, s_, R, Kv))[0]
        if best is None or e < best[0] - 1e-10:
            best = (e, Kv)
    e0, k0 = best
    gs = qs3.Sector(L, K, k0)
    X = torch.empty(gs.dim, dtype=torch.complex128, device="cuda")
    res = gs.eigs(nev=1, evecs=X, seed=3)
    assert res.evals[0] == pytest.approx(e0, abs=1e-10)
    omega = np.linspace(-2, 8, 301)
    steps = 20
    S, a, b, w = gs.dsf(X, res.evals[0], ks, omega, steps=steps, eta=0.1, field=1.0)
    phi = X.cpu().numpy()
    sigma, R = mk_list(geo, K, k0)
    for qi, Qv in enumerate(ks):
        kq = tuple((k0[a_] + Qv[a_]) % lat.dims[a_] for a_ in range(3))
        s1, R1 = mk_list(geo, K + 1, kq)
        psi = sq_to_vec(geo, K, sigma, R, k0, phi, s1, R1, Qv, "-")
        wq = float(np.vdot(psi, psi).real) / float(np.vdot(phi, phi).real)
        assert w[qi] == pytest.approx(wq, abs=1e-12)
        Hk = gen_full_ham_sym_adapt(geo, K + 1, bonds, s1, R1, kq)
        m = min(steps, len(s1))
        oa, ob, _ = orc_lanczos(lambda x: Hk @ x, psi, m)
        eff = next((i + 1 for i in range(len(ob)) if ob[i] < 1e-8 * 8), len(ob))
        assert np.abs(a[qi, :eff] - oa[:eff]).max() < 1e-10
        Sref = continued_fraction(oa[:eff], ob[:eff], wq, omega, res.evals[0], 0.1, 1.0)
        assert np.abs(S[qi] - Sref).max() < 1e-8 * max(1.0, np.abs(Sref).max())
