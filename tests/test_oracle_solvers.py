"""Pins of the oracle's Lanczos/TRL (Alg. 10), observables (Sec. 3.6, 4.2),
S^-_q (Alg. 11) and continued fraction (Eq. (cfe)) against dense
diagonalisation, Kronecker-product spin operators on the full 2^N space, sum
rules, closed forms and the exact resolvent."""
import json
import math
import os

import numpy as np
import pytest

import workloads as wl
from oracle import native as nat
from oracle.cns import F
from oracle.hamiltonian import bonds_1based, gen_full_ham
from oracle.lanczos import lanczos, trl, diag_tri, lowest_distinct, ritz
from oracle.observables import sz, corr_zz, corr_pm, positions, structure_factors, all_tuples
from oracle.translation import Geometry, mk_list, gen_full_ham_sym_adapt, expand_to_u1
from oracle.dynamics import (smq_to_vec, smq_u1, continued_fraction, sq_to_vec, sq_u1, n_down_after,
                             trivial_sz)
from oracle.rng import splitmix64, start_vector
from oracle.thermal import thermal

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _build():
    nat.build(force=False)


def test_splitmix64_reference_outputs():
    g = json.load(open(os.path.join(GOLD, "splitmix64.json")))
    assert [str(splitmix64(1234567, i)) for i in range(3)] == g["seed_1234567"]
    assert hex(splitmix64(0, 0)) == g["seed_0_first_hex"]
    v = start_vector(1234567, np.arange(3), complex_=False)
    assert np.all((v >= -1) & (v < 1))
    assert v[0] == 2.0 * (6457827717110365317 >> 11) / 2.0 ** 53 - 1.0


# ---------------------------------------------------------------- full-space operators
def full_ops(N):
    """s^z_i, s^+_i as 2^N x 2^N matrices; bit i of the basis index set = site i down."""
    I = np.eye(2)
    sz1 = np.diag([0.5, -0.5])       # basis (up, down)
    sp1 = np.array([[0, 1], [0, 0]], dtype=float)   # |up><down|

    def site(op, i):
        out = np.array([[1.0]])
        for s in range(N - 1, -1, -1):          # site N-1 is the most significant bit
            out = np.kron(out, op if s == i else I)
        return out
    return [site(sz1, i) for i in range(N)], [site(sp1, i) for i in range(N)]


def test_observables_against_kronecker_operators():
    lat = wl.with_disorder(wl.chain(8), seed=11)
    N, K = 8, 3
    SZ, SP = full_ops(N)
    H = sum(j * 0.5 * (SP[i] @ SP[k].T + SP[i].T @ SP[k]) + jz * SZ[i] @ SZ[k]
            for i, k, j, jz in zip(lat.bi, lat.bj, lat.jxy, lat.jz))
    # sector states: popcount K, ascending index order == rank order
    idx = [m for m in range(1 << N) if bin(m).count("1") == K]
    Hs = H[np.ix_(idx, idx)]
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    assert np.abs(Hs - gen_full_ham(N, K, bonds)).max() < 1e-14
    e, U = np.linalg.eigh(Hs)
    phi = U[:, 0]
    full = np.zeros(1 << N)
    full[idx] = phi
    ref_sz = np.array([full @ SZ[i] @ full for i in range(N)])
    ref_zz = np.array([[full @ SZ[i] @ SZ[j] @ full for j in range(N)] for i in range(N)])
    ref_pm = np.array([[full @ SP[i] @ SP[j].T @ full for j in range(N)] for i in range(N)])
    assert np.abs(sz(phi, N, K) - ref_sz).max() < 1e-13
    assert np.abs(corr_zz(phi, N, K) - ref_zz).max() < 1e-13
    assert np.abs(corr_pm(phi, N, K) - ref_pm).max() < 1e-13
    # energy identity
    E = sum(j * 0.5 * (ref_pm[i, k] + ref_pm[k, i]) + jz * ref_zz[i, k]
            for i, k, j, jz in zip(lat.bi, lat.bj, lat.jxy, lat.jz))
    assert E == pytest.approx(e[0], abs=1e-12)
    # S^-_q by definition vs Kronecker
    pos = positions(N, 1, 1)
    q = np.array([2 * np.pi * 3 / N, 0, 0])
    Smq = sum(np.exp(-1j * q[0] * pos[r, 0]) * SP[r].T for r in range(N)) / math.sqrt(N)
    out_full = Smq @ full
    idx1 = [m for m in range(1 << N) if bin(m).count("1") == K + 1]
    assert np.abs(smq_u1(N, K, pos, q, phi.astype(complex)) - out_full[idx1]).max() < 1e-14


def test_sum_rules_u1_and_k():
    lat = wl.square(4)
    N, K = 16, 3
    M = N / 2 - K
    geo = Geometry(*lat.dims)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    pos = positions(*lat.dims)
    qs = [2 * np.pi * np.array([kx / 4, ky / 4, 0]) for (kx, ky, kz) in wl.all_momenta(lat)]
    for Kv in [(0, 0, 0), (1, 2, 0)]:
        s, R = mk_list(geo, K, Kv)
        e, U = np.linalg.eigh(gen_full_ham_sym_adapt(geo, K, bonds, s, R, Kv))
        u1 = expand_to_u1(geo, K, s, R, Kv, U[:, 0])
        szv = sz(u1, N, K)
        assert szv.sum() == pytest.approx(M, abs=1e-12)
        assert np.abs(szv - M / N).max() < 1e-12            # translation invariant
        zz = corr_zz(u1, N, K)
        pm = corr_pm(u1, N, K)
        assert np.abs(zz.sum(axis=1) - M * szv).max() < 1e-12
        sf = structure_factors(zz, pm, szv, pos, np.array(qs))
        assert sf[:, 0].sum() == pytest.approx(N / 4, abs=1e-10)
        assert sf[0, 0] == pytest.approx(M * M / N, abs=1e-10)   # q = 0 longitudinal part
        assert sf[:, 1].sum() == pytest.approx(N - K, abs=1e-10)
        E = sum(j * (zz[i, k] * 1.0 + 0.5 * (pm[i, k] + pm[k, i]).real)
                for i, k, j in zip(lat.bi, lat.bj, lat.jxy))
        assert E == pytest.approx(e[0], abs=1e-10)


def test_lanczos_c1_lowest_distinct_vs_dense():
    """C1: chain 16, N_down = 3, 100 steps with full reorthogonalisation give the
    4 lowest distinct levels of the dense matrix to 1e-10 relative."""
    lat = wl.chain(16)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    H = gen_full_ham(16, 3, bonds)
    ev = np.linalg.eigvalsh(H)
    ref = lowest_distinct(ev, 4)
    assert ref[0] == pytest.approx(-1.81500162, abs=1e-8)
    v0 = start_vector(1, np.arange(560), complex_=False)
    a, b, Psi = lanczos(lambda x: H @ x, v0, 100)
    e, res, _ = ritz(a, b)
    got = lowest_distinct(e, 4, residuals=res)
    assert len(lowest_distinct(e, 6)) == 6 and lowest_distinct(e, 6)[2] != got[2]
    assert np.allclose(got, ref, rtol=1e-10, atol=0)
    # orthonormal Lanczos basis
    G = Psi[:, :100].T @ Psi[:, :100]
    assert np.abs(G - np.eye(100)).max() < 1e-12


def test_trl_vs_dense_k_sector():
    lat = wl.square(4)
    geo = Geometry(*lat.dims)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    s, R = mk_list(geo, 4, (1, 0, 0))
    Hk = gen_full_ham_sym_adapt(geo, 4, bonds, s, R, (1, 0, 0))
    ev = np.linalg.eigvalsh(Hk)
    v0 = start_vector(5, np.array(s, dtype=np.uint64) - 1, complex_=True)
    e, X, nres, conv = trl(lambda x: Hk @ x, v0, NK=6, NM=14, IM=500, eps=1e-14)
    assert conv
    # distinct lowest levels present among Ritz values
    for lv in lowest_distinct(ev, 3):
        assert np.min(np.abs(e - lv)) < 1e-10 * max(1, abs(lv))
    r = Hk @ X[:, 0] - e[0] * X[:, 0]
    assert np.linalg.norm(r) < 1e-8


def test_smq_alg11_equals_definition_with_stabilisers():
    for lat, K in [(wl.chain(6), 2), (wl.square(4), 1), (wl.hypercubic(4, 2, 1), 2)]:
        geo = Geometry(*lat.dims)
        pos = positions(*lat.dims)
        for Kv in wl.all_momenta(lat)[:3]:
            s, R = mk_list(geo, K, Kv)
            if not s:
                continue
            phi = np.random.default_rng(4).normal(size=len(s)) + 0.3j
            u1 = expand_to_u1(geo, K, s, R, Kv, phi)
            for Qv in wl.all_momenta(lat)[:4]:
                kq = tuple((Kv[i] + Qv[i]) % lat.dims[i] for i in range(3))
                s1, R1 = mk_list(geo, K + 1, kq)
                q = 2 * np.pi * np.array(Qv) / np.array(lat.dims)
                ref = smq_u1(geo.N, K, pos, q, u1)
                got = expand_to_u1(geo, K + 1, s1, R1, kq, smq_to_vec(geo, K, s, R, Kv, phi, s1, R1, Qv)) \
                    if s1 else np.zeros_like(ref)
                assert np.abs(got - ref).max() < 1e-13


def test_continued_fraction_vs_resolvent_and_sum_rules():
    lat = wl.chain(10)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    N = 10
    H2 = gen_full_ham(N, 2, bonds)
    H3 = gen_full_ham(N, 3, bonds)
    e, U = np.linalg.eigh(H2)
    e0, phi = e[0], U[:, 0]
    pos = positions(N, 1, 1)
    q = np.array([2 * np.pi * 4 / N, 0, 0])
    psi = smq_u1(N, 2, pos, q, phi.astype(complex))
    w = np.vdot(psi, psi).real
    a, b, _ = lanczos(lambda x: H3 @ x, psi, 60)
    om = np.linspace(0, 8, 401)
    for h, eta in [(0.0, 0.05), (2.0, 0.1)]:
        S = continued_fraction(a, b, w, om, e0, eta, h)
        z = om - h + e0 + 1j * eta
        ref = np.array([-np.imag(np.vdot(psi, np.linalg.solve(zz * np.eye(H3.shape[0]) - H3, psi))) / np.pi
                        for zz in z])
        assert np.abs(S - ref).max() < 1e-10
    # pole weights from eig(T) sum to the numerator
    ee, C = diag_tri(a, b)
    assert (w * C[0, :] ** 2).sum() == pytest.approx(w, rel=1e-12)


def test_single_magnon_lorentzian():
    """From the fully polarised state (K = 0 -> 1): S^-_q|FM> is the one-magnon
    eigenstate, so S(q, w) is one Lorentzian of weight 1 at w = h + E_1(q) - E_FM."""
    lat = wl.square(4)
    N = 16
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    H1 = gen_full_ham(N, 1, bonds)
    efm = lat.jz.sum() / 4
    pos = positions(4, 4, 1)
    for Q in [(1, 0), (2, 2), (0, 3)]:
        q = 2 * np.pi * np.array([Q[0] / 4, Q[1] / 4, 0])
        psi = smq_u1(N, 0, pos, q, np.array([1.0 + 0j]))
        a, b, _ = lanczos(lambda x: H1 @ x, psi, 1)
        e1 = efm - 2 + math.cos(q[0]) + math.cos(q[1])
        assert a[0] == pytest.approx(e1, abs=1e-12)
        om = np.linspace(0, 8, 101)
        eta, h = 0.05, 4.0
        S = continued_fraction(a[:1], b[:1], 1.0, om, efm, eta, h)
        w0 = h + e1 - efm
        assert np.abs(S - eta / np.pi / ((om - w0) ** 2 + eta ** 2)).max() < 1e-12


def test_sq_u1_all_operators_against_kronecker():
    """S^-, S^+ and S^z at momentum q, by definition on U(1) amplitudes, equal the
    2^N Kronecker-product operators N^{-1/2} sum_r e^{-iq.R_r} s^a_r."""
    N, K = 8, 3
    SZ, SP = full_ops(N)
    pos = positions(N, 1, 1)
    idx = {k: [m for m in range(1 << N) if bin(m).count("1") == k] for k in (K - 1, K, K + 1)}
    rng = np.random.default_rng(8)
    phi = rng.normal(size=len(idx[K])) + 1j * rng.normal(size=len(idx[K]))
    full = np.zeros(1 << N, dtype=complex)
    full[idx[K]] = phi
    for Q in (0, 3, 5):
        q = np.array([2 * np.pi * Q / N, 0, 0])
        ph = [np.exp(-1j * q[0] * pos[r, 0]) / math.sqrt(N) for r in range(N)]
        for op, mats in (("-", [m.T for m in SP]), ("+", SP), ("z", SZ)):
            O = sum(ph[r] * mats[r] for r in range(N))
            ref = (O @ full)[idx[n_down_after(op, K)]]
            assert np.abs(sq_u1(N, K, pos, q, phi, op) - ref).max() < 1e-14


@pytest.mark.parametrize("op", ["-", "+", "z"])
def test_sq_scatter_equals_definition_with_stabilisers(op):
    """The momentum-basis scatter (Alg. 11 and its S^+ / S^z analogues) expanded
    to the U(1) basis equals the operator applied by definition."""
    for lat, K in [(wl.chain(6), 2), (wl.square(4), 2), (wl.hypercubic(4, 2, 1), 2), (wl.chain(6), 3)]:
        geo = Geometry(*lat.dims)
        pos = positions(*lat.dims)
        K1 = n_down_after(op, K)
        for Kv in wl.all_momenta(lat)[:3]:
            s, R = mk_list(geo, K, Kv)
            if not s:
                continue
            phi = np.random.default_rng(4).normal(size=len(s)) + 0.3j
            u1 = expand_to_u1(geo, K, s, R, Kv, phi)
            for Qv in wl.all_momenta(lat)[:4]:
                kq = tuple((Kv[i] + Qv[i]) % lat.dims[i] for i in range(3))
                s1, R1 = mk_list(geo, K1, kq)
                q = 2 * np.pi * np.array(Qv) / np.array(lat.dims)
                ref = sq_u1(geo.N, K, pos, q, u1, op)
                got = expand_to_u1(geo, K1, s1, R1, kq, sq_to_vec(geo, K, s, R, Kv, phi, s1, R1, Qv, op)) \
                    if s1 else np.zeros_like(ref)
                assert np.abs(got - ref).max() < 1e-13


@pytest.mark.parametrize("op", ["-", "+", "z"])
def test_sq_scatter_equals_definition_unit_cells(op):
    """Several sites per cell: the scatter expanded to the U(1) basis equals
    S^op_q applied by definition with positions = cell coordinates + the
    places' offsets (kagome, honeycomb, pyrochlore)."""
    for lat, K in [(wl.kagome(2, 2), 2), (wl.honeycomb(2, 2), 3), (wl.kagome(2, 2), 1), (wl.pyrochlore(2), 2)]:
        geo = Geometry(lat.lx, lat.ly, lat.lz, lat.ns, lat.basis)
        pos = np.array([geo.position(r) for r in range(1, geo.N + 1)])
        K1 = n_down_after(op, K)
        for Kv in wl.all_momenta(lat)[:3]:
            s, R = mk_list(geo, K, Kv)
            if not s:
                continue
            phi = np.random.default_rng(6).normal(size=len(s)) + 0.2j
            u1 = expand_to_u1(geo, K, s, R, Kv, phi)
            for Qv in wl.all_momenta(lat):
                kq = tuple((Kv[i] + Qv[i]) % lat.dims[i] for i in range(3))
                s1, R1 = mk_list(geo, K1, kq)
                q = 2 * np.pi * np.array(Qv) / np.array(lat.dims)
                ref = sq_u1(geo.N, K, pos, q, u1, op)
                got = expand_to_u1(geo, K1, s1, R1, kq, sq_to_vec(geo, K, s, R, Kv, phi, s1, R1, Qv, op)) \
                    if s1 else np.zeros_like(ref)
                assert np.abs(got - ref).max() < 1e-13


def test_sq_sum_rules():
    """sum_q |S^a_q phi|^2 = <sum_r s^a_r^+ s^a_r>: N - K (S^-), K (S^+), N/4 (S^z)
    for a normalised state with K down spins (Fourier completeness)."""
    lat = wl.hypercubic(3, 3, 1)
    N, K = 9, 4
    pos = positions(3, 3, 1)
    rng = np.random.default_rng(2)
    phi = rng.normal(size=math.comb(N, K)) + 1j * rng.normal(size=math.comb(N, K))
    phi /= np.linalg.norm(phi)
    qs = [2 * np.pi * np.array([kx / 3, ky / 3, 0]) for (kx, ky, kz) in wl.all_momenta(lat)]
    for op, want in (("-", N - K), ("+", K), ("z", N / 4)):
        tot = sum(np.vdot(v, v).real for v in (sq_u1(N, K, pos, q, phi, op) for q in qs))
        assert tot == pytest.approx(want, abs=1e-12)


def test_one_magnon_sp_sz_closed_forms():
    """One magnon |k> (N_down = 1, a single state per k): S^+_q |k> = |FM> exactly
    when k + q = 0 (and no target state otherwise); |S^z_q |k>|^2 = 1/N for q != 0
    and (N/2 - 1)^2 / N at q = 0."""
    lat = wl.square(4)
    geo = Geometry(4, 4, 1)
    N = 16
    for Kv in [(0, 0, 0), (1, 0, 0), (3, 2, 0)]:
        s, R = mk_list(geo, 1, Kv)
        assert len(s) == 1
        for Qv in wl.all_momenta(lat):
            kq = tuple((Kv[i] + Qv[i]) % 4 for i in range(3))
            s0, R0 = mk_list(geo, 0, kq)
            if kq == (0, 0, 0):
                v = sq_to_vec(geo, 1, s, R, Kv, np.array([1.0 + 0j]), s0, R0, Qv, "+")
                assert abs(v[0]) == pytest.approx(1.0, abs=1e-13)
            else:
                assert not s0
            s1, R1 = mk_list(geo, 1, kq)
            w = sq_to_vec(geo, 1, s, R, Kv, np.array([1.0 + 0j]), s1, R1, Qv, "z")
            want = (N / 2 - 1) ** 2 / N if Qv == (0, 0, 0) else 1.0 / N
            assert np.vdot(w, w).real == pytest.approx(want, abs=1e-13)


@pytest.mark.parametrize("op", ["+", "z"])
def test_continued_fraction_sp_sz_vs_resolvent_with_field(op):
    """S^+ / S^z continued fractions equal -(1/pi) Im <psi|(w + E0_h - H'_h + i eta)^-1|psi>
    with the Zeeman term -h S^z_tot included in both Hamiltonians (fixes the
    direction of the field shift)."""
    lat = wl.chain(10)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    N, K = 10, 3
    H = gen_full_ham(N, K, bonds)
    e, U = np.linalg.eigh(H)
    e0, phi = e[0], U[:, 0]
    K1 = n_down_after(op, K)
    H1 = gen_full_ham(N, K1, bonds)
    pos = positions(N, 1, 1)
    q = np.array([2 * np.pi * 3 / N, 0, 0])
    psi = sq_u1(N, K, pos, q, phi.astype(complex), op)
    w = np.vdot(psi, psi).real
    a, b, _ = lanczos(lambda x: H1 @ x, psi, 80)
    om = np.linspace(-2, 8, 301)
    for h, eta in [(0.0, 0.05), (1.5, 0.1)]:
        S = continued_fraction(a, b, w, om, e0, eta, h, op)
        e0h = e0 - h * (N / 2 - K)
        H1h = H1 - h * (N / 2 - K1) * np.eye(H1.shape[0])
        ref = np.array([-np.imag(np.vdot(psi, np.linalg.solve((o + e0h + 1j * eta) * np.eye(H1.shape[0]) - H1h, psi)))
                        / np.pi for o in om])
        assert np.abs(S - ref).max() < 1e-9


def test_trivial_sz_component_is_the_q0_response():
    """At q = 0, S^z_q |gs> = N^{-1/2} M |gs>: its continued fraction is a single
    Lorentzian at omega = 0 of weight M^2/N, the trivial part subtracted."""
    lat = wl.square(4)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    N, K = 16, 2
    H = gen_full_ham(N, K, bonds)
    e, U = np.linalg.eigh(H)
    pos = positions(4, 4, 1)
    psi = sq_u1(N, K, pos, np.zeros(3), U[:, 0].astype(complex), "z")
    a, b, _ = lanczos(lambda x: H @ x, psi, 5)
    M = N / 2 - K
    om = np.linspace(-1, 4, 201)
    S = continued_fraction(a[:1], b[:1], np.vdot(psi, psi).real, om, e[0], 0.05, 0.0, "z")
    assert np.vdot(psi, psi).real == pytest.approx(M * M / N, abs=1e-12)
    assert np.abs(S - trivial_sz(om, 0.05, M, N)).max() < 1e-10


def _all_levels(lat, Kmax=None, use_k=True):
    """Every level of every (N_down, k) sector from the oracle's dense blocks,
    with its S^z_tot."""
    geo = Geometry(*lat.dims)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    N = lat.n_sites
    E, Sz = [], []
    for K in range(0, (Kmax if Kmax is not None else N) + 1):
        if use_k:
            for Kv in wl.all_momenta(lat):
                s, R = mk_list(geo, K, Kv)
                if s:
                    ev = np.linalg.eigvalsh(gen_full_ham_sym_adapt(geo, K, bonds, s, R, Kv))
                    E += list(ev)
                    Sz += [N / 2 - K] * len(ev)
        else:
            ev = np.linalg.eigvalsh(gen_full_ham(N, K, bonds))
            E += list(ev)
            Sz += [N / 2 - K] * len(ev)
    return np.array(E), np.array(Sz)


def test_sector_spectra_make_the_full_spectrum():
    """The union of all (N_down, k) sector spectra is the spectrum of the 2^N
    Kronecker-product Hamiltonian (chain of 8 with disorder: U(1) sectors; the
    uniform chain of 8: momentum sectors)."""
    for lat, use_k in [(wl.with_disorder(wl.chain(8), seed=5), False), (wl.chain(8), True)]:
        N = lat.n_sites
        SZ, SP = full_ops(N)
        H = sum(j * 0.5 * (SP[i] @ SP[k].T + SP[i].T @ SP[k]) + jz * SZ[i] @ SZ[k]
                for i, k, j, jz in zip(lat.bi, lat.bj, lat.jxy, lat.jz))
        E, Sz = _all_levels(lat, use_k=use_k)
        assert len(E) == 1 << N
        assert np.abs(np.sort(E) - np.linalg.eigvalsh(H)).max() < 1e-12


def test_thermal_limits_and_closed_forms():
    """ln Z -> N ln 2, E -> 0, C ~ beta^2 Tr H^2 / 2^N at high temperature
    (Tr H^2 / 2^N = sum_b J_b^2 (2 + Delta_b^2) / 16 + h^2 N / 4); free spins in a
    field: Z = (2 cosh(beta h / 2))^N, M = (N/2) tanh(beta h / 2)."""
    lat = wl.with_disorder(wl.chain(8), seed=3)
    N = lat.n_sites
    E, Sz = _all_levels(lat, use_k=False)
    h = 0.7
    tr2 = sum(j * j * (2 + (jz / j) ** 2) / 16 for j, jz in zip(lat.jxy, lat.jz)) + h * h * N / 4
    b = 1e-4
    t = thermal(E, Sz, np.array([0.0, b]), h)
    assert t["lnZ"][0] == pytest.approx(N * math.log(2), abs=1e-12)
    assert abs(t["energy"][0]) < 1e-12 and abs(t["mag"][0]) < 1e-12
    assert t["heat"][1] == pytest.approx(b * b * tr2, rel=1e-3)
    free = wl.chain(8, J=0.0)
    E0, Sz0 = _all_levels(free, use_k=False)
    for beta in (0.3, 2.0):
        t = thermal(E0, Sz0, np.array([beta]), h)
        assert t["lnZ"][0] == pytest.approx(N * math.log(2 * math.cosh(beta * h / 2)), abs=1e-11)
        assert t["mag"][0] == pytest.approx(N / 2 * math.tanh(beta * h / 2), abs=1e-11)
