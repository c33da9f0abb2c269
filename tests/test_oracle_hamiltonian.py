"""Pins of the oracle's Hamiltonian code (Alg. 4, 8, 9) against an independent
bitmask construction of the spin operators, Hermiticity, spectra, the
translation eigenvalue, the one-magnon closed form and SU(2) descent."""
import itertools
import math

import numpy as np
import pytest

import workloads as wl
from oracle import native as nat
from oracle.cns import F
from oracle.hamiltonian import bonds_1based, gen_full_ham, ham_to_vec_u1
from oracle.translation import (Geometry, mk_list, gen_full_ham_sym_adapt, ham_to_vec_k,
                                expand_to_u1)


@pytest.fixture(scope="module", autouse=True)
def _build():
    nat.build(force=False)


def masks(N, K):
    """Every popcount-K mask below 2^N, ascending (sorted K-subsets, no rank code)."""
    return sorted(sum(1 << i for i in c) for c in itertools.combinations(range(N), K))


def bitmask_H(lat, K):
    """H of the model equation on popcount-K masks (bit i set = site i down),
    indexed by ascending mask value; built from s^z = +-1/2 and s^+s^- + s^-s^+
    flipping both bits -- no rank code."""
    N = lat.n_sites
    ms = masks(N, K)
    idx = {m: i for i, m in enumerate(ms)}
    H = np.zeros((len(ms), len(ms)))
    for c, m in enumerate(ms):
        for i, j, jxy, jz in zip(lat.bi, lat.bj, lat.jxy, lat.jz):
            si = 0.5 - (m >> int(i) & 1)
            sj = 0.5 - (m >> int(j) & 1)
            H[c, c] += jz * si * sj
            if si != sj:
                H[idx[m ^ (1 << int(i)) ^ (1 << int(j))], c] += jxy / 2.0
    return H


LATS = [(wl.chain(8), 3), (wl.chain(9), 4), (wl.square(4), 2), (wl.hypercubic(3, 2, 1), 3),
        (wl.random_bonds(9, 14, seed=3), 4), (wl.with_disorder(wl.square(3), seed=5), 3)]


@pytest.mark.parametrize("lat,K", LATS)
def test_dense_u1_equals_bitmask(lat, K):
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    H = gen_full_ham(lat.n_sites, K, bonds)
    Hb = bitmask_H(lat, K)
    assert np.array_equal(H != 0, Hb != 0)          # pattern bit-exact
    assert np.abs(H - Hb).max() <= 1e-15
    v = np.random.default_rng(0).normal(size=H.shape[0])
    assert np.abs(ham_to_vec_u1(lat.n_sites, K, bonds, v) - Hb @ v).max() < 1e-13
    B = nat.Bonds.of(lat)
    assert np.abs(nat.hv_u1(lat.n_sites, K, B, v) - Hb @ v).max() < 1e-13
    # sampled-rows API
    rows = np.array([1, 2, H.shape[0]], dtype=np.uint64)
    assert np.abs(nat.hv_u1(lat.n_sites, K, B, v, rows=rows) - (Hb @ v)[rows.astype(int) - 1]).max() < 1e-13


def test_row_nnz_formula_and_mean():
    """Off-diagonal entries per row = bonds with exactly one end down; the mean
    over the sector is N_b * 2K(N-K) / (N(N-1)) for any bond set."""
    for lat, K, expect in [(wl.chain(16), 3, 5.2), (wl.square(10), 4, 15.515151515)]:
        N = lat.n_sites
        B = nat.Bonds.of(lat)
        rng = np.random.default_rng(1)
        D = math.comb(N, K)
        rows = rng.integers(1, D + 1, size=400) if D > 5000 else np.arange(1, D + 1)
        tot = 0
        for a in rows:
            dg, cols, vals = nat.row_u1(N, K, B, int(a))
            n = set(int(x) - 1 for x in nat.f_bar(N, K, np.array([a], dtype=np.uint64))[0])
            one = sum(1 for i, j in zip(lat.bi, lat.bj) if (int(i) in n) != (int(j) in n))
            assert len(cols) == one
            tot += len(cols)
        assert lat.n_bonds * 2 * K * (N - K) / (N * (N - 1)) == pytest.approx(expect, rel=1e-8)
        if D <= 5000:
            assert tot / len(rows) == pytest.approx(expect, rel=1e-12)


def T_matrix(lat, K, t):
    """Translation of the unit cells by t on popcount-K masks (ascending mask
    order); a site keeps its place in the cell."""
    lx, ly, lz = lat.dims
    ns = lat.ns
    N = lat.n_sites
    ms = masks(N, K)
    idx = {m: i for i, m in enumerate(ms)}
    T = np.zeros((len(ms), len(ms)))
    for c, m in enumerate(ms):
        out = 0
        for i in range(N):
            if m >> i & 1:
                sub, cell = i % ns, i // ns
                x, y, z = cell % lx, (cell // lx) % ly, cell // (lx * ly)
                j = sub + ns * ((x + t[0]) % lx + lx * (((y + t[1]) % ly) + ly * ((z + t[2]) % lz)))
                out |= 1 << j
        T[idx[out], c] = 1.0
    return T


KLATS = [(wl.chain(8), 3), (wl.chain(6), 2), (wl.square(4), 2), (wl.hypercubic(4, 2, 1), 3),
         (wl.hypercubic(3, 3, 1), 3), (wl.with_disorder(wl.square(3), seed=9, per_bond=False), 2)]


@pytest.mark.parametrize("lat,K", KLATS)
def test_k_blocks_hermitian_and_spectrum(lat, K):
    geo = Geometry(*lat.dims)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    ev = np.linalg.eigvalsh(bitmask_H(lat, K))
    allev = []
    for Kv in wl.all_momenta(lat):
        s, R = mk_list(geo, K, Kv)
        if not s:
            continue
        Hk = gen_full_ham_sym_adapt(geo, K, bonds, s, R, Kv)
        assert np.abs(Hk - Hk.conj().T).max() < 1e-13
        allev.extend(np.linalg.eigvalsh(Hk))
    assert len(allev) == len(ev)
    assert np.abs(np.sort(allev) - ev).max() < 1e-12


@pytest.mark.parametrize("lat,K", KLATS[:4])
def test_k_block_projector_and_translation_eigenvalue(lat, K):
    """Independent projector check: eigenvalues of Q^+ H Q with Q an orthonormal
    basis of range((1/N) sum_t e^{-ik.t} T^t) in the bitmask basis equal those of
    the oracle's k block; and the oracle's k vectors, expanded to U(1)
    amplitudes, are eigenvectors of T^t with eigenvalue e^{ik.t} (pins the sign
    of the phase, which spectra alone cannot)."""
    geo = Geometry(*lat.dims)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    Hb = bitmask_H(lat, K)
    lx, ly, lz = lat.dims
    ts = [(tx, ty, tz) for tz in range(lz) for ty in range(ly) for tx in range(lx)]
    Ts = {t: T_matrix(lat, K, t) for t in ts}
    for Kv in wl.all_momenta(lat):
        kdot = lambda t: 2 * np.pi * (Kv[0] * t[0] / lx + Kv[1] * t[1] / ly + Kv[2] * t[2] / lz)
        P = sum(np.exp(-1j * kdot(t)) * Ts[t] for t in ts) / geo.N
        u, sv, _ = np.linalg.svd(P)
        Q = u[:, sv > 0.5]
        s, R = mk_list(geo, K, Kv)
        assert Q.shape[1] == len(s)
        if not s:
            continue
        Hk = gen_full_ham_sym_adapt(geo, K, bonds, s, R, Kv)
        e1 = np.linalg.eigvalsh(Q.conj().T @ Hb @ Q)
        e2 = np.linalg.eigvalsh(Hk)
        assert np.abs(e1 - e2).max() < 1e-12
        phi = np.random.default_rng(2).normal(size=len(s)) + 1j * np.random.default_rng(3).normal(size=len(s))
        u1 = expand_to_u1(geo, K, s, R, Kv, phi)
        for t in ts[:3]:
            assert np.abs(Ts[t] @ u1 - np.exp(1j * kdot(t)) * u1).max() < 1e-12
        # H commutes with the expansion: expand(Hk phi) == Hb expand(phi)
        assert np.abs(expand_to_u1(geo, K, s, R, Kv, Hk @ phi) - Hb @ u1).max() < 1e-12
        # and Alg. 9 reproduces the dense block
        assert np.abs(ham_to_vec_k(geo, K, bonds, s, R, Kv, phi) - Hk @ phi).max() < 1e-13
        B = nat.Bonds.of(lat)
        sc, Rc = nat.mk_list(lat.dims, K, Kv)
        assert np.abs(nat.hv_k(lat.dims, K, Kv, B, sc, Rc, phi) - Hk @ phi).max() < 1e-13


CELL_LATS = [(wl.kagome(2, 2), 3), (wl.kagome(2, 2), 4), (wl.honeycomb(3, 2), 3),
             (wl.honeycomb(2, 2), 2), (wl.with_disorder(wl.kagome(2, 2), seed=4, per_bond=False), 2),
             (wl.pyrochlore(2), 2)]


def _order(t, dims):
    return math.lcm(*(L // math.gcd(ti, L) for ti, L in zip(t, dims)))


@pytest.mark.parametrize("lat,K", CELL_LATS, ids=lambda x: getattr(x, "name", str(x)))
def test_multisite_cells_k_blocks(lat, K):
    """Several sites per unit cell (translations act on the cells): sector
    dimensions follow Burnside over the N_T cell translations, every k block
    is Hermitian, the union of the k spectra is the fixed-N_down spectrum, the
    projector check holds and expanded k vectors carry e^{ik.t} under T^t."""
    lx, ly, lz = lat.dims
    geo = Geometry(lx, ly, lz, lat.ns)
    assert geo.N == lat.n_sites and geo.NT == lx * ly * lz
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    Hb = bitmask_H(lat, K)
    ev = np.linalg.eigvalsh(Hb)
    ts = [(tx, ty, tz) for tz in range(lz) for ty in range(ly) for tx in range(lx)]
    Ts = {t: T_matrix(lat, K, t) for t in ts}
    N, NT = lat.n_sites, geo.NT
    allev = []
    total = 0
    for Kv in wl.all_momenta(lat):
        kdot = lambda t: 2 * np.pi * (Kv[0] * t[0] / lx + Kv[1] * t[1] / ly + Kv[2] * t[2] / lz)
        s, R = mk_list(geo, K, Kv)
        # Burnside with characters: a translation of order o splits the sites
        # into N/o cycles of length o
        d = sum(np.exp(1j * kdot(t)) * (math.comb(N // _order(t, lat.dims), K // _order(t, lat.dims))
                                        if K % _order(t, lat.dims) == 0 else 0) for t in ts) / NT
        assert abs(d.imag) < 1e-9 and round(d.real) == len(s)
        total += len(s)
        P = sum(np.exp(-1j * kdot(t)) * Ts[t] for t in ts) / NT
        u, sv, _ = np.linalg.svd(P)
        Q = u[:, sv > 0.5]
        assert Q.shape[1] == len(s)
        if not s:
            continue
        Hk = gen_full_ham_sym_adapt(geo, K, bonds, s, R, Kv)
        assert np.abs(Hk - Hk.conj().T).max() < 1e-13
        e2 = np.linalg.eigvalsh(Hk)
        assert np.abs(np.linalg.eigvalsh(Q.conj().T @ Hb @ Q) - e2).max() < 1e-12
        allev.extend(e2)
        phi = np.random.default_rng(2).normal(size=len(s)) + 1j * np.random.default_rng(3).normal(size=len(s))
        u1 = expand_to_u1(geo, K, s, R, Kv, phi)
        for t in ts[1:3]:
            assert np.abs(Ts[t] @ u1 - np.exp(1j * kdot(t)) * u1).max() < 1e-12
        assert np.abs(expand_to_u1(geo, K, s, R, Kv, Hk @ phi) - Hb @ u1).max() < 1e-12
    assert total == math.comb(N, K)
    assert np.abs(np.sort(allev) - ev).max() < 1e-12


@pytest.mark.parametrize("lat", [wl.chain(16), wl.square(6), wl.cube(4), wl.square(10, J=1.0, Delta=0.7)])
def test_one_magnon_closed_form(lat):
    """K = 1: E(k) - E_FM = -z J Delta / 2 + J sum_alpha cos k_alpha on a periodic
    hypercubic lattice with uniform J, Delta (E_FM = sum_b Jz_b / 4)."""
    geo = Geometry(*lat.dims)
    B = nat.Bonds.of(lat)
    J, Jz = lat.jxy[0], lat.jz[0]
    D = sum(1 for L in lat.dims if L > 1)
    efm = lat.jz.sum() / 4
    for Kv in wl.all_momenta(lat)[:: max(1, len(wl.all_momenta(lat)) // 12)]:
        s, R = nat.mk_list(lat.dims, 1, Kv)
        assert len(s) == 1
        e = nat.hv_k(lat.dims, 1, Kv, B, s, R, np.ones(1, dtype=np.complex128))[0]
        k = [2 * np.pi * Kv[a] / lat.dims[a] for a in range(3)]
        expect = efm - 2 * D * Jz / 2 + J * sum(math.cos(k[a]) for a in range(3) if lat.dims[a] > 1)
        assert abs(e.imag) < 1e-13 and e.real == pytest.approx(expect, abs=1e-12)


def test_su2_descent():
    """Delta = 1: every level of (K-1, k) appears in (K, k) for K <= N/2."""
    lat = wl.chain(10)
    geo = Geometry(*lat.dims)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    for Kv in [(0, 0, 0), (3, 0, 0), (5, 0, 0)]:
        lo = []
        for K in (2, 3):
            s, R = mk_list(geo, K, Kv)
            lo.append(np.linalg.eigvalsh(gen_full_ham_sym_adapt(geo, K, bonds, s, R, Kv)))
        for e in lo[0]:
            assert np.min(np.abs(lo[1] - e)) < 1e-10
    # E_FM in the k = 0 sector at every K
    efm = lat.jz.sum() / 4
    for K in (1, 2, 3):
        s, R = mk_list(geo, K, (0, 0, 0))
        ev = np.linalg.eigvalsh(gen_full_ham_sym_adapt(geo, K, bonds, s, R, (0, 0, 0)))
        assert np.min(np.abs(ev - efm)) < 1e-10
