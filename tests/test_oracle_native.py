"""Pins of the plain C oracle's routines that the GPU parity tests use as
references: a fixed-N_down row (values and pattern) against the bitmask
construction of the spin operators, a momentum-block row against the dense
block whose spectrum and projector are pinned in test_oracle_hamiltonian,
the S^-_q scatter against the operator applied by definition in the U(1)
basis, and the cached-structure variant against the row-by-row Alg. 9."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import native as nat
from oracle.dynamics import smq_u1
from oracle.observables import positions
from oracle.translation import Geometry, expand_to_u1, gen_full_ham_sym_adapt, mk_list
from oracle.hamiltonian import bonds_1based
from test_oracle_hamiltonian import bitmask_H


@pytest.fixture(scope="module", autouse=True)
def _build():
    nat.build(force=False)


@pytest.mark.parametrize("lat,K", [(wl.chain(10), 3), (wl.square(4), 3),
                                   (wl.with_disorder(wl.square(3), seed=5), 4),
                                   (wl.random_bonds(9, 14, seed=3), 4)])
def test_row_u1_values_against_bitmask(lat, K):
    """Every row of the C oracle's fixed-N_down matrix, diagonal and
    off-diagonal values, equals the bitmask matrix row (rank order equals
    ascending mask order, pinned in test_oracle_basis)."""
    Hb = bitmask_H(lat, K)
    B = nat.Bonds.of(lat)
    for a in range(1, Hb.shape[0] + 1):
        dg, cols, vals = nat.row_u1(lat.n_sites, K, B, a)
        row = np.zeros(Hb.shape[0])
        row[a - 1] += dg
        np.add.at(row, cols.astype(np.int64), vals)
        assert np.abs(row - Hb[a - 1]).max() <= 1e-15
        # one entry per bond with exactly one end down
        down = set(int(x) - 1 for x in nat.f_bar(lat.n_sites, K, np.array([a], dtype=np.uint64))[0])
        assert len(cols) == sum(1 for i, j in zip(lat.bi, lat.bj) if (int(i) in down) != (int(j) in down))


@pytest.mark.parametrize("lat,K", [(wl.chain(8), 3), (wl.square(4), 2), (wl.hypercubic(4, 2, 1), 3),
                                   (wl.hypercubic(3, 3, 1), 3)])
def test_row_k_against_dense_block(lat, K):
    """Every row of the C oracle's momentum block equals the row of the
    Python oracle's dense block (pinned by its projector and spectrum)."""
    geo = Geometry(*lat.dims)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    B = nat.Bonds.of(lat)
    for Kv in wl.all_momenta(lat)[:4]:
        s, R = mk_list(geo, K, Kv)
        if not s:
            continue
        Hk = gen_full_ham_sym_adapt(geo, K, bonds, s, R, Kv)
        sc, Rc = nat.mk_list(lat.dims, K, Kv)
        assert np.array_equal(sc, np.array(s, dtype=np.uint64))
        assert np.abs(Rc - np.array(R)).max() < 1e-13
        for al in range(1, len(s) + 1):
            dg, cols, vals = nat.row_k(lat.dims, K, Kv, B, sc, Rc, al)
            row = np.zeros(len(s), dtype=np.complex128)
            row[al - 1] += dg
            np.add.at(row, cols, vals)
            assert np.abs(row - Hk[al - 1]).max() < 1e-14


@pytest.mark.parametrize("lat,K", [(wl.chain(6), 2), (wl.square(4), 1), (wl.hypercubic(4, 2, 1), 2),
                                   (wl.square(4), 2)])
def test_smq_c_oracle_equals_definition(lat, K):
    """The C oracle's S^-_q scatter, expanded to U(1) amplitudes, equals
    S^-_q = N^-1/2 sum_r e^{-iq.R_r} s^-_r applied to the expanded input by
    definition (no translation code), including stabilised representatives."""
    geo = Geometry(*lat.dims)
    pos = positions(*lat.dims)
    rng = np.random.default_rng(11)
    for Kv in wl.all_momenta(lat)[:3]:
        sc, Rc = nat.mk_list(lat.dims, K, Kv)
        if len(sc) == 0:
            continue
        phi = rng.normal(size=len(sc)) + 1j * rng.normal(size=len(sc))
        u1 = expand_to_u1(geo, K, [int(x) for x in sc], Rc, Kv, phi)
        for Qv in wl.all_momenta(lat)[:4]:
            kq = tuple((Kv[i] + Qv[i]) % lat.dims[i] for i in range(3))
            s1, R1 = nat.mk_list(lat.dims, K + 1, kq)
            q = 2 * np.pi * np.array(Qv) / np.array(lat.dims)
            ref = smq_u1(geo.N, K, pos, q, u1)
            if len(s1) == 0:
                assert np.abs(ref).max() < 1e-13
                continue
            got = nat.smq(lat.dims, K, Kv, sc, Rc, phi, s1, R1, Qv)
            assert np.abs(expand_to_u1(geo, K + 1, [int(x) for x in s1], R1, kq, got) - ref).max() < 1e-13


@pytest.mark.parametrize("lat,K", [(wl.chain(12), 3), (wl.square(4), 3), (wl.square(6), 2),
                                   (wl.hypercubic(4, 3, 1), 3), (wl.cube(3), 2),
                                   (wl.with_disorder(wl.square(4), seed=9, per_bond=False), 3)])
def test_kstruct_equals_row_by_row(lat, K):
    """The cached-structure variant: its sectors are the mk_list sectors
    (same ranks, same R), their sizes add up to C(N, K), and its H.v is the
    row-by-row Alg. 9 bit for bit (same terms in the same order)."""
    B = nat.Bonds.of(lat)
    ks = nat.KStruct(lat.dims, K, B)
    rng = np.random.default_rng(5)
    total = 0
    for Kv in wl.all_momenta(lat):
        mem, sig, R = ks.sector(Kv)
        sc, Rc = nat.mk_list(lat.dims, K, Kv)
        assert np.array_equal(sig, sc) and np.array_equal(R, Rc)
        assert np.array_equal(ks.sector(Kv)[0], mem)
        total += len(sig)
        if len(sig) == 0:
            continue
        phi = rng.normal(size=len(sig)) + 1j * rng.normal(size=len(sig))
        assert np.array_equal(ks.hv(Kv, mem, R, phi), nat.hv_k(lat.dims, K, Kv, B, sc, Rc, phi))
    assert total == math.comb(lat.n_sites, K)
    # every orbit representative once; hops = off-diagonal entries of the rows
    assert ks.nrep == len(nat.mk_list(lat.dims, K, (0, 0, 0))[0])


def test_kstruct_one_magnon_closed_form_cube():
    """K = 1 on the 6^3 cube through the cached structure: E(k) - E_FM =
    -z J Delta / 2 + J sum_a cos k_a for every momentum."""
    lat = wl.cube(6)
    ks = nat.KStruct(lat.dims, 1, nat.Bonds.of(lat))
    EFM = lat.jz.sum() / 4
    for Kv in wl.all_momenta(lat):
        mem, sig, R = ks.sector(Kv)
        assert len(sig) == 1
        e = ks.hv(Kv, mem, R, np.ones(1, dtype=np.complex128))[0]
        ref = EFM - 6 / 2 + sum(math.cos(2 * math.pi * k / 6) for k in Kv)
        assert abs(e.imag) < 1e-13 and abs(e.real - ref) < 1e-12
