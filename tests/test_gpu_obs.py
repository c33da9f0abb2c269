"""GPU observables (Sec. 3.6, 4.2), S^-_q, S^+_q and S^z_q (Sec. 3.8, Alg. 11)
and the continued-fraction S(q, omega) (Eq. (cfe)) against the oracle on the
same input vectors.

Tolerances: correlations and structure factors are sums of |phi|^2-weighted
terms of size <= 1 over at most C(N, K) states; 1e-12 absolute covers their
float64 rounding.  The continued fraction is compared through its Lanczos
coefficients (1e-10) and on the omega grid (1e-8 relative to max S).
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import native as orc
from oracle.dynamics import continued_fraction, smq_to_vec, sq_to_vec, n_down_after, trivial_sz
from oracle.lanczos import lanczos as orc_lanczos
from oracle.observables import corr_pm, corr_zz, positions, structure_factors, sz
from oracle.translation import Geometry, expand_to_u1, gen_full_ham_sym_adapt, mk_list
from oracle.hamiltonian import bonds_1based

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qs3():
    from paper_2107_00872_amd import qs3 as q
    orc.build(force=False)
    return q


@pytest.fixture(scope="module")
def ctx(qs3):
    return qs3.Context(0)


def all_pairs(N):
    return [i for i in range(N) for j in range(N)], [j for i in range(N) for j in range(N)]


def qgrid(lat):
    return np.array([[2 * np.pi * kx / lat.lx, 2 * np.pi * ky / lat.ly, 2 * np.pi * kz / lat.lz]
                     for (kx, ky, kz) in wl.all_momenta(lat)])


@pytest.mark.parametrize("lat,K", [(wl.with_disorder(wl.chain(10), 4), 3), (wl.square(4), 3),
                                   (wl.random_bonds(9, 16, 1), 4), (wl.chain(8), 1)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_u1_observables(qs3, ctx, lat, K):
    L = qs3.Lattice.of(ctx, lat)
    sec = qs3.Sector(L, K)
    N = lat.n_sites
    X = torch.empty(sec.dim, dtype=torch.float64, device="cuda")
    sec.eigs(nev=1, evecs=X, seed=4)
    phi = X.cpu().numpy()
    ref_sz = sz(phi, N, K)
    assert np.abs(sec.sz(X) - ref_sz).max() < 1e-12
    pi, pj = all_pairs(N)
    zz, pm = sec.sisj(X, pi, pj)
    rzz, rpm = corr_zz(phi, N, K), corr_pm(phi, N, K)
    assert np.abs(zz - rzz.reshape(-1)).max() < 1e-12
    assert np.abs(pm - rpm.reshape(-1)).max() < 1e-12
    qs = qgrid(lat)
    szz, spm, stot = sec.sq(X, qs)
    ref = structure_factors(rzz, rpm, ref_sz, positions(*lat.dims), qs)
    assert np.abs(szz - ref[:, 0]).max() < 1e-11
    assert np.abs(spm - ref[:, 1]).max() < 1e-11
    assert np.abs(stot - ref[:, 2]).max() < 1e-11
    # sum rules (pins independent of the oracle)
    M = N / 2 - K
    assert sec.sz(X).sum() == pytest.approx(M, abs=1e-12)
    if lat.translation_invariant:
        assert spm.sum() == pytest.approx(N - K, abs=1e-10)
        assert szz.sum() == pytest.approx(N / 4, abs=1e-10)


@pytest.mark.parametrize("lat,K", [(wl.chain(10), 3), (wl.with_disorder(wl.chain(12), 2), 4)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_u1_pair_subset_vs_oracle(qs3, ctx, lat, K):
    """Fewer than N pairs take the per-pair subset loops (all pairs take the
    Gram-matrix form): both against the oracle's pair sums."""
    L = qs3.Lattice.of(ctx, lat)
    sec = qs3.Sector(L, K)
    N = lat.n_sites
    X = torch.empty(sec.dim, dtype=torch.float64, device="cuda")
    sec.eigs(nev=1, evecs=X, seed=2)
    phi = X.cpu().numpy()
    rzz, rpm = corr_zz(phi, N, K), corr_pm(phi, N, K)
    pi = [0, 3, 5, N - 1, 2, 7]
    pj = [1, 0, 9, 4, 2, N - 2]
    zz, pm = sec.sisj(X, pi, pj)
    for t, (i, j) in enumerate(zip(pi, pj)):
        assert abs(zz[t] - rzz[i, j]) < 1e-12 and abs(pm[t] - rpm[i, j]) < 1e-12, (i, j)


@pytest.mark.parametrize("n_sites,K", [(100, 4), (200, 4)])
def test_u1_gram_pairs_vs_subset_loops(qs3, ctx, n_sites, K):
    """The Gram form at full size (10x10-square sites at N_down = 4: one factor
    chunk, two column tiles; a 200-site chain: eight chunks of the factor and
    a ragged fourth tile) against the per-pair subset loops on sampled pairs,
    for a seeded random state."""
    lat = wl.square(10) if n_sites == 100 else wl.chain(n_sites)
    L = qs3.Lattice.of(ctx, lat)
    sec = qs3.Sector(L, K)
    g = torch.Generator(device="cuda").manual_seed(11)
    X = torch.randn(int(sec.dim), dtype=torch.float64, device="cuda", generator=g)
    X /= X.norm()
    pi, pj = all_pairs(n_sites)
    zz, pm = sec.sisj(X, pi, pj)
    rng = np.random.default_rng(5)
    sample = rng.choice(n_sites * n_sites, size=3 * (n_sites - 1), replace=False)
    for c in range(3):
        idx = sample[c * (n_sites - 1):(c + 1) * (n_sites - 1)]
        zs, ps = sec.sisj(X, [pi[t] for t in idx], [pj[t] for t in idx])
        assert np.abs(ps - pm[idx]).max() < 1e-15 * max(1.0, np.abs(pm).max()) + 1e-17
        assert np.abs(zs - zz[idx]).max() < 1e-14
    # the matrix is symmetric and its diagonal <S+_i S-_i> = 1/2 + <S^z_i>
    # sums to N - N_down for any normalised state
    P = pm.real.reshape(n_sites, n_sites)
    assert np.allclose(P, P.T, atol=1e-15)
    assert np.trace(P) == pytest.approx(n_sites - K, abs=1e-10)


@pytest.mark.parametrize("lat,K", [(wl.square(4), 3), (wl.chain(8), 3), (wl.hypercubic(4, 2, 1), 2)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_k_observables_translation_averaged(qs3, ctx, lat, K):
    """Any vector of a momentum sector is an eigenvector of T, so its
    correlations are translation invariant: the translation-averaged values of
    the device equal the oracle's direct values on the expanded state."""
    L = qs3.Lattice.of(ctx, lat)
    geo = Geometry(*lat.dims)
    N = lat.n_sites
    pi, pj = all_pairs(N)
    for Kv in wl.all_momenta(lat)[:5]:
        s, R = mk_list(geo, K, Kv)
        if not s:
            continue
        sec = qs3.Sector(L, K, Kv)
        rng = np.random.default_rng(2)
        phi = rng.normal(size=len(s)) + 1j * rng.normal(size=len(s))
        X = torch.from_numpy(phi).cuda()
        u1 = expand_to_u1(geo, K, s, R, Kv, phi)
        rzz, rpm = corr_zz(u1, N, K), corr_pm(u1, N, K)
        zz, pm = sec.sisj(X, pi, pj)
        assert np.abs(zz - rzz.reshape(-1)).max() < 1e-12
        assert np.abs(pm - rpm.reshape(-1)).max() < 1e-12
        qs = qgrid(lat)
        szz, spm, stot = sec.sq(X, qs)
        ref = structure_factors(rzz, rpm, sz(u1, N, K), positions(*lat.dims), qs)
        assert np.abs(np.stack([szz, spm, stot], 1) - ref).max() < 1e-11
        assert np.abs(sec.sz(X) - sz(u1, N, K)).max() < 1e-12
        sec.close()


@pytest.mark.parametrize("lat,K", [(wl.chain(6), 2), (wl.square(4), 1), (wl.square(4), 2),
                                   (wl.hypercubic(4, 2, 1), 2), (wl.cube(3), 2)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_smq_gather_vs_alg11(qs3, ctx, lat, K):
    L = qs3.Lattice.of(ctx, lat)
    for Kv in wl.all_momenta(lat)[:3]:
        sigma, R = orc.mk_list(lat.dims, K, Kv)
        if len(sigma) == 0:
            continue
        src = qs3.Sector(L, K, Kv)
        rng = np.random.default_rng(7)
        phi = rng.normal(size=len(sigma)) + 1j * rng.normal(size=len(sigma))
        X = torch.from_numpy(phi).cuda()
        for Qv in wl.all_momenta(lat)[:6]:
            kq = tuple((Kv[a] + Qv[a]) % lat.dims[a] for a in range(3))
            s1, R1 = orc.mk_list(lat.dims, K + 1, kq)
            if len(s1) == 0:
                continue
            dst = qs3.Sector(L, K + 1, kq)
            out = torch.empty(dst.dim, dtype=torch.complex128, device="cuda")
            src.smq(X, dst, Qv, out)
            ref = orc.smq(lat.dims, K, Kv, sigma, R, phi, s1, R1, Qv)
            assert np.abs(out.cpu().numpy() - ref).max() < 1e-12 * max(1, np.abs(phi).max()) * (K + 1)
            dst.close()
        src.close()


def test_dsf_small_vs_oracle(qs3, ctx):
    """4x4 square, N_down = 2 ground state at its lowest k, S^-(q, omega) for all
    q at h = 2: Lanczos coefficients, weights and the continued fraction against
    the oracle (dense k+q blocks, oracle Lanczos from the oracle's S^-_q)."""
    lat = wl.square(4)
    L = qs3.Lattice.of(ctx, lat)
    geo = Geometry(*lat.dims)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    ks = wl.all_momenta(lat)
    K = 2
    best = None
    for Kv in ks:
        s, R = mk_list(geo, K, Kv)
        e = np.linalg.eigvalsh(gen_full_ham_sym_adapt(geo, K, bonds, s, R, Kv))[0]
        if best is None or e < best[0] - 1e-10:
            best = (e, Kv)
    e0, k0 = best
    gs = qs3.Sector(L, K, k0)
    X = torch.empty(gs.dim, dtype=torch.complex128, device="cuda")
    res = gs.eigs(nev=1, evecs=X, seed=9)
    assert res.evals[0] == pytest.approx(e0, abs=1e-10)
    omega = np.linspace(0, 8, 401)
    steps = 40
    S, a, b, w = gs.dsf(X, res.evals[0], ks, omega, steps=steps, eta=0.1, field=2.0)
    phi = X.cpu().numpy()
    sigma, R = orc.mk_list(lat.dims, K, k0)
    tot = 0.0
    for qi, Qv in enumerate(ks):
        kq = tuple((k0[a_] + Qv[a_]) % lat.dims[a_] for a_ in range(3))
        s1, R1 = orc.mk_list(lat.dims, K + 1, kq)
        psi = orc.smq(lat.dims, K, k0, sigma, R, phi, s1, R1, Qv)
        wq = float(np.vdot(psi, psi).real)
        assert w[qi] == pytest.approx(wq, abs=1e-12)
        tot += wq
        Hk = gen_full_ham_sym_adapt(geo, K + 1, bonds, list(map(int, s1)), list(R1), kq)
        m = min(steps, len(s1))
        oa, ob, _ = orc_lanczos(lambda x: Hk @ x, psi, m)
        # coefficients are defined up to the (numerical) end of the Krylov
        # space of psi': stop where beta falls below 1e-8 |H|
        eff = next((i + 1 for i in range(len(ob)) if ob[i] < 1e-8 * 8), len(ob))
        assert np.abs(a[qi, :eff] - oa[:eff]).max() < 1e-10
        if eff > 1:
            assert np.abs(b[qi, :eff - 1] - ob[:eff - 1]).max() < 1e-10
        Sref = continued_fraction(oa, ob, wq, omega, res.evals[0], 0.1, 2.0)
        assert np.abs(S[qi] - Sref).max() < 1e-8 * max(1.0, np.abs(Sref).max())
    assert tot == pytest.approx(lat.n_sites - K, abs=1e-10)   # sum_q S^{+-}(q) = N - K


def test_dsf_partial_reorthogonalisation(qs3, ctx):
    """S^-(q, omega) on the 10x10 square from the N_down = 2 ground state, 150
    levels for all 100 q: partial reorthogonalisation gives the same weights,
    the same Lanczos coefficients to 1e-10 over the first 40 levels (q != 0;
    at q = 0 the start vector is an eigenvector and the recurrence stops after
    one level), and a spectrum within 2e-4 of its maximum of the fully
    reorthogonalised one.  The late coefficients are fixed only to rounding:
    semi-orthogonality keeps the Ritz values, not the basis, at working
    accuracy, and even two fully reorthogonalised runs whose dot products sum
    in a different order agree to 1e-13 up to about level 85 and then drift
    apart exponentially, which moves S by 3e-5 of its maximum (partial against
    full: 4.6e-5 and 5.6e-5 with those two summation orders)."""
    lat = wl.square(10)
    L = qs3.Lattice.of(ctx, lat)
    ks = wl.all_momenta(lat)
    gs = qs3.Sector(L, 2, (0, 0, 0))
    X = torch.empty(gs.dim, dtype=torch.complex128, device="cuda")
    e0 = gs.eigs(nev=1, evecs=X, seed=3).evals[0]
    omega = np.linspace(0, 8, 801)
    Sf, af, bf, wf = gs.dsf(X, e0, ks, omega, steps=150, eta=0.05, field=4.0, reorth=qs3.REORTH_FULL)
    Sp, ap, bp, wp = gs.dsf(X, e0, ks, omega, steps=150, eta=0.05, field=4.0, reorth=qs3.REORTH_PARTIAL)
    assert np.abs(wp - wf).max() < 1e-13
    assert np.abs(ap[1:, :40] - af[1:, :40]).max() < 1e-10
    assert np.abs(bp[1:, :39] - bf[1:, :39]).max() < 1e-10
    assert np.abs(Sp - Sf).max() < 2e-4 * np.abs(Sf).max()


SQ_CASES = [(wl.square(4), 2), (wl.chain(8), 3), (wl.hypercubic(4, 2, 1), 3), (wl.cube(3), 2), (wl.chain(6), 1)]


def _sq_parity(qs3, ctx, lat, K, op):
    code = {"-": qs3.OP_SMINUS, "+": qs3.OP_SPLUS, "z": qs3.OP_SZ}[op]
    geo = Geometry(*lat.dims)
    L = qs3.Lattice.of(ctx, lat)
    K1 = n_down_after(op, K)
    for Kv in wl.all_momenta(lat)[:3]:
        s, R = mk_list(geo, K, Kv)
        if not s:
            continue
        src = qs3.Sector(L, K, Kv)
        rng = np.random.default_rng(11)
        phi = rng.normal(size=len(s)) + 1j * rng.normal(size=len(s))
        X = torch.from_numpy(phi).cuda()
        for Qv in wl.all_momenta(lat)[:6]:
            kq = tuple((Kv[a] + Qv[a]) % lat.dims[a] for a in range(3))
            s1, R1 = mk_list(geo, K1, kq)
            if not s1:
                continue
            dst = qs3.Sector(L, K1, kq)
            assert dst.dim == len(s1)
            out = torch.empty(dst.dim, dtype=torch.complex128, device="cuda")
            src.sq_apply(X, dst, code, Qv, out)
            ref = sq_to_vec(geo, K, s, R, Kv, phi, s1, R1, Qv, op)
            scale = np.abs(phi).max() * max(1, lat.n_sites if op != "-" else K + 1)
            assert np.abs(out.cpu().numpy() - ref).max() < 1e-13 * scale
            dst.close()
        src.close()


@pytest.mark.parametrize("op", ["+", "z"])
@pytest.mark.parametrize("lat,K", SQ_CASES, ids=lambda x: getattr(x, "name", str(x)))
def test_sp_sz_gather_vs_scatter(qs3, ctx, lat, K, op):
    """S^+_q and S^z_q as gathers over the target representatives equal the
    oracle's scatter (the procedure of Alg. 11 for S^+ and S^z)."""
    _sq_parity(qs3, ctx, lat, K, op)


def test_sp_gather_on_the_fly(qs3):
    """The S^+_q gather with every source canonicalised on the fly."""
    c = qs3.Context(0)
    c.set_structure_limits(0, 0)
    _sq_parity(qs3, c, wl.hypercubic(4, 2, 1), 3, "+")
    c.close()


@pytest.mark.parametrize("op", ["+", "z"])
def test_dsf_sp_sz_vs_oracle(qs3, ctx, op):
    """4x4 square, N_down = 3 ground state at its lowest k: S^+(q, omega) and
    S^z(q, omega) for all q at h = 1.5 against the oracle (its scatter, dense k+q
    blocks, its Lanczos and continued fraction); sum rules sum_q S^{-+}(q) = K and
    sum_q S^{zz}(q) = N/4; the trivial q = 0 longitudinal part subtracts to 0."""
    code = {"+": qs3.OP_SPLUS, "z": qs3.OP_SZ}[op]
    lat = wl.square(4)
    L = qs3.Lattice.of(ctx, lat)
    geo = Geometry(*lat.dims)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    ks = wl.all_momenta(lat)
    K = 3
    K1 = n_down_after(op, K)
    best = None
    for Kv in ks:
        s, R = mk_list(geo, K, Kv)
        e = np.linalg.eigvalsh(gen_full_ham_sym_adapt(geo, K, bonds, s, R, Kv))[0]
        if best is None or e < best[0] - 1e-10:
            best = (e, Kv)
    e0, k0 = best
    gs = qs3.Sector(L, K, k0)
    X = torch.empty(gs.dim, dtype=torch.complex128, device="cuda")
    res = gs.eigs(nev=1, evecs=X, seed=9)
    assert res.evals[0] == pytest.approx(e0, abs=1e-10)
    omega = np.linspace(-2, 8, 401)
    steps, eta, h = 30, 0.1, 1.5
    S, a, b, w = gs.dsf(X, res.evals[0], ks, omega, steps=steps, eta=eta, field=h, op=code)
    phi = X.cpu().numpy()
    phi = phi / np.linalg.norm(phi)
    sigma, R = mk_list(geo, K, k0)
    tot = 0.0
    for qi, Qv in enumerate(ks):
        kq = tuple((k0[a_] + Qv[a_]) % lat.dims[a_] for a_ in range(3))
        s1, R1 = mk_list(geo, K1, kq)
        if not s1:
            assert w[qi] == 0.0
            continue
        psi = sq_to_vec(geo, K, sigma, R, k0, phi, s1, R1, Qv, op)
        wq = float(np.vdot(psi, psi).real)
        assert w[qi] == pytest.approx(wq, abs=1e-12)
        tot += wq
        if wq < 1e-20:
            continue
        Hk = gen_full_ham_sym_adapt(geo, K1, bonds, s1, R1, kq)
        m = min(steps, len(s1))
        oa, ob, _ = orc_lanczos(lambda x: Hk @ x, psi, m)
        eff = next((i + 1 for i in range(len(ob)) if ob[i] < 1e-8 * 8), len(ob))
        assert np.abs(a[qi, :eff] - oa[:eff]).max() < 1e-10
        Sref = continued_fraction(oa[:eff], ob[:eff], wq, omega, res.evals[0], eta, h, op)
        assert np.abs(S[qi] - Sref).max() < 1e-8 * max(1.0, np.abs(Sref).max())
    assert tot == pytest.approx(K if op == "+" else lat.n_sites / 4, abs=1e-10)
    if op == "z":
        S2, _, _, w2 = gs.dsf(X, res.evals[0], [(0, 0, 0)], omega, steps=steps, eta=eta, field=h, op=code,
                              subtract_trivial=True)
        M = lat.n_sites / 2 - K
        assert w2[0] == pytest.approx(M * M / lat.n_sites, abs=1e-12)
        assert np.abs(S2[0]).max() < 1e-8 * trivial_sz(np.zeros(1), eta, M, lat.n_sites)[0]
