"""Pins of the oracle's point-group sectors: the dimension of every (k, chi)
sector from the character formula over fixed states (no representative code),
symmetric blocks, the spectra against projectors built in the bitmask basis,
the expanded vectors transforming with the character, and the 1D blocks'
levels inside the momentum block's."""
import itertools
import math

import numpy as np
import pytest

import workloads as wl
from oracle.hamiltonian import bonds_1based
from oracle.pointgroup import expand_pg, gen_full_ham_pg, mk_list_pg
from oracle.translation import Geometry, gen_full_ham_sym_adapt, mk_list
from test_oracle_hamiltonian import bitmask_H, masks


def _perm_of(lat, perms, p, t):
    """Site permutation of T^t P_p (0-based)."""
    lx, ly, lz = lat.dims
    out = []
    for i in range(lat.n_sites):
        j = int(perms[p][i])
        x, y, z = j % lx, (j // lx) % ly, j // (lx * ly)
        out.append((x + t[0]) % lx + lx * (((y + t[1]) % ly) + ly * ((z + t[2]) % lz)))
    return out


def _fixed_states(perm, K):
    """Number of K-subsets mapped onto themselves: unions of whole cycles."""
    seen, lens = set(), []
    for i in range(len(perm)):
        if i in seen:
            continue
        n, j = 0, i
        while j not in seen:
            seen.add(j)
            j = perm[j]
            n += 1
        lens.append(n)
    poly = [1] + [0] * K
    for ln in lens:
        new = poly[:]
        for k in range(K + 1 - ln):
            new[k + ln] += poly[k]
        poly = new
    return poly[K]


def _U(lat, K, perm):
    ms = masks(lat.n_sites, K)
    idx = {m: i for i, m in enumerate(ms)}
    U = np.zeros((len(ms), len(ms)))
    for c, m in enumerate(ms):
        out = 0
        for i in range(lat.n_sites):
            if m >> i & 1:
                out |= 1 << perm[i]
        U[idx[out], c] = 1.0
    return U


CASES = [(wl.square(4), 2, (0, 0, 0)), (wl.square(4), 3, (2, 2, 0)),
         (wl.with_disorder(wl.square(4), seed=3, per_bond=False), 3, (0, 0, 0)),
         (wl.square_j1j2(4, 0.45), 2, (2, 2, 0))]


@pytest.mark.parametrize("lat,K,Kv", CASES, ids=lambda x: getattr(x, "name", str(x)))
def test_c4v_sectors(lat, K, Kv):
    L = lat.lx
    perms = wl.c4v_ops(L)
    geo = Geometry(*lat.dims)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    ts = [(tx, ty, 0) for ty in range(L) for tx in range(L)]
    kph = lambda t: 1.0 if math.cos(geo.kdot(Kv, t)) > 0 else -1.0
    fixed = {(p, t): _fixed_states(_perm_of(lat, perms, p, t), K) for p in range(8) for t in ts}
    G = 8 * len(ts)
    s_k, R_k = mk_list(geo, K, Kv)
    ek = np.linalg.eigvalsh(gen_full_ham_sym_adapt(geo, K, bonds, s_k, R_k, Kv))
    Hb = bitmask_H(lat, K)
    Us = {(p, t): _U(lat, K, _perm_of(lat, perms, p, t)) for p in range(8) for t in ts}
    total = 0
    for name, chars in wl.C4V_CHARS.items():
        d = round(sum(chars[p] * kph(t) * fixed[(p, t)] for p in range(8) for t in ts))
        assert d % G == 0
        d //= G
        s, R = mk_list_pg(geo, perms, chars, K, Kv)
        assert len(s) == d, name
        total += d
        if not s:
            continue
        H = gen_full_ham_pg(geo, perms, chars, K, bonds, s, R, Kv)
        assert np.abs(H - H.T).max() < 1e-13
        e = np.linalg.eigvalsh(H)
        for x in e:
            assert np.min(np.abs(ek - x)) < 1e-10
        # projector onto the (k, chi) subspace in the bitmask basis
        P = sum(chars[p] * kph(t) * Us[(p, t)] for p in range(8) for t in ts) / G
        u, sv, _ = np.linalg.svd(P)
        Q = u[:, sv > 0.5]
        assert Q.shape[1] == d
        assert np.abs(np.linalg.eigvalsh(Q.T @ Hb @ Q) - e).max() < 1e-12
        phi = np.random.default_rng(5).normal(size=d)
        u1 = expand_pg(geo, perms, chars, K, s, R, Kv, phi)
        # the bitmask order of the masks is the rank order: same basis
        for (p, t) in [(1, (0, 0, 0)), (4, (1, 0, 0)), (6, (2, 1, 0))]:
            assert np.abs(Us[(p, t)] @ u1 - chars[p] * kph(t) * u1).max() < 1e-12
        assert np.abs(expand_pg(geo, perms, chars, K, s, R, Kv, H @ phi) - Hb @ u1).max() < 1e-12
    dE = round(sum(wl.C4V_E[p] * kph(t) * fixed[(p, t)] for p in range(8) for t in ts)) // G
    assert total + 2 * dE == len(s_k)


def test_oh_sectors_cube3():
    """O_h (48 signed axis permutations) on the periodic 3x3x3 cube at
    N_down = 2, k = 0: every one-dimensional sector's dimension from the
    character formula over fixed states, and the non-empty blocks' spectra
    against the projector onto the (k, chi) subspace in the bitmask basis."""
    lat = wl.cube(3)
    K, Kv = 2, (0, 0, 0)
    perms = wl.oh_ops(3)
    geo = Geometry(*lat.dims)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    ts = [(tx, ty, tz) for tz in range(3) for ty in range(3) for tx in range(3)]
    G = len(perms) * len(ts)
    Hb = bitmask_H(lat, K)
    ms = masks(lat.n_sites, K)
    idx = {m: i for i, m in enumerate(ms)}
    for name, chars in wl.oh_chars().items():
        d = 0
        P = np.zeros((len(ms), len(ms)))
        for p in range(len(perms)):
            for t in ts:
                perm = _perm_of(lat, perms, p, t)
                d += chars[p] * _fixed_states(perm, K)
                for c, m in enumerate(ms):
                    out = 0
                    for i in range(lat.n_sites):
                        if m >> i & 1:
                            out |= 1 << perm[i]
                    P[idx[out], c] += chars[p] / G
        assert d % G == 0
        s, R = mk_list_pg(geo, perms, chars, K, Kv)
        assert len(s) == d // G, name
        if not s:
            continue
        e = np.linalg.eigvalsh(gen_full_ham_pg(geo, perms, chars, K, bonds, s, R, Kv))
        u, sv, _ = np.linalg.svd(P)
        Q = u[:, sv > 0.5]
        assert Q.shape[1] == len(s)
        assert np.abs(np.linalg.eigvalsh(Q.T @ Hb @ Q) - e).max() < 1e-12


def _cell_perm_of(lat, perms, p, t):
    """Site permutation of T^t P_p on a lattice of lat.ns places per cell."""
    lx, ly, lz = lat.dims
    ns = lat.ns
    out = []
    for i in range(lat.n_sites):
        j = int(perms[p][i])
        s, c = j % ns, j // ns
        x, y, z = c % lx, (c // lx) % ly, c // (lx * ly)
        out.append(s + ns * ((x + t[0]) % lx + lx * (((y + t[1]) % ly) + ly * ((z + t[2]) % lz))))
    return out


@pytest.mark.parametrize("L,K,Kv", [(3, 3, (0, 0, 0)), (4, 2, (2, 2, 0)), (4, 2, (0, 2, 0))])
def test_honeycomb_inversion_sectors(L, K, Kv):
    """Inversion through a bond centre exchanges the two places of the
    honeycomb cell: the sector dimensions from the character formula over
    fixed states, and the blocks' spectra against the projector onto the
    (k, chi) subspace in the bitmask basis."""
    lat = wl.honeycomb(L, L)
    perms = wl.honeycomb_inversion_ops(L, L)
    geo = Geometry(L, L, 1, 2)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    ts = [(tx, ty, 0) for ty in range(L) for tx in range(L)]
    G = 2 * len(ts)
    kph = lambda t: 1.0 if math.cos(geo.kdot(Kv, t)) > 0 else -1.0
    Hb = bitmask_H(lat, K)
    ms = masks(lat.n_sites, K)
    idx = {m: i for i, m in enumerate(ms)}
    total = 0
    for chars in ((1, 1), (1, -1)):
        d = 0
        P = np.zeros((len(ms), len(ms)))
        for p in range(2):
            for t in ts:
                perm = _cell_perm_of(lat, perms, p, t)
                ch = chars[p] * kph(t)
                d += ch * _fixed_states(perm, K)
                for c, m in enumerate(ms):
                    out = 0
                    for i in range(lat.n_sites):
                        if m >> i & 1:
                            out |= 1 << perm[i]
                    P[idx[out], c] += ch / G
        assert round(d) % G == 0
        s, R = mk_list_pg(geo, perms, chars, K, Kv)
        assert len(s) == round(d) // G
        total += len(s)
        if not s:
            continue
        e = np.linalg.eigvalsh(gen_full_ham_pg(geo, perms, chars, K, bonds, s, R, Kv))
        u, sv, _ = np.linalg.svd(P)
        Q = u[:, sv > 0.5]
        assert Q.shape[1] == len(s)
        assert np.abs(np.linalg.eigvalsh(Q.T @ Hb @ Q) - e).max() < 1e-12
    # the two one-dimensional sectors exhaust the momentum sector
    assert total == len(mk_list(geo, K, Kv)[0])


def _cell_group_sectors(lat, perms, charsets, K, Kv):
    """Dimensions from the character formula and projector spectra for a
    group of cell translations x point operations on lat (any places per cell)."""
    lx, ly, lz = lat.dims
    geo = Geometry(lx, ly, lz, lat.ns)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    ts = [(tx, ty, tz) for tz in range(lz) for ty in range(ly) for tx in range(lx)]
    G = len(perms) * len(ts)
    kph = lambda t: 1.0 if math.cos(geo.kdot(Kv, t)) > 0 else -1.0
    Hb = bitmask_H(lat, K)
    ms = masks(lat.n_sites, K)
    idx = {m: i for i, m in enumerate(ms)}
    dims = []
    for chars in charsets:
        d = 0
        P = np.zeros((len(ms), len(ms)))
        for p in range(len(perms)):
            for t in ts:
                perm = _cell_perm_of(lat, perms, p, t)
                ch = chars[p] * kph(t)
                d += ch * _fixed_states(perm, K)
                for c, m in enumerate(ms):
                    out = 0
                    for i in range(lat.n_sites):
                        if m >> i & 1:
                            out |= 1 << perm[i]
                    P[idx[out], c] += ch / G
        assert round(d) % G == 0
        s, R = mk_list_pg(geo, perms, chars, K, Kv)
        assert len(s) == round(d) // G
        dims.append(len(s))
        if not s:
            continue
        e = np.linalg.eigvalsh(gen_full_ham_pg(geo, perms, chars, K, bonds, s, R, Kv))
        u, sv, _ = np.linalg.svd(P)
        Q = u[:, sv > 0.5]
        assert Q.shape[1] == len(s)
        assert np.abs(np.linalg.eigvalsh(Q.T @ Hb @ Q) - e).max() < 1e-12
    return dims


@pytest.mark.parametrize("L,K", [(2, 3), (3, 2)])
def test_kagome_c6v_sectors(L, K):
    """C6v of the kagome lattice about a hexagon centre (rotations and
    mirrors exchange the three places of a cell): the one-dimensional sectors
    at k = 0 by the character formula and the projector."""
    lat = wl.kagome(L, L)
    dims = _cell_group_sectors(lat, wl.kagome_c6v_ops(L), list(wl.C6V_CHARS.values()), K, (0, 0, 0))
    assert sum(dims) > 0


@pytest.mark.parametrize("K", [2, 3])
def test_honeycomb_c6v_sectors(K):
    """C6v of the 3x3 honeycomb about a hexagon centre (exchanging its two
    places): the one-dimensional sectors at k = 0 by the character formula
    and the projector."""
    lat = wl.honeycomb(3, 3)
    dims = _cell_group_sectors(lat, wl.honeycomb_c6v_ops(3), list(wl.C6V_CHARS.values()), K, (0, 0, 0))
    assert sum(dims) > 0
