"""Pins of the oracle's basis code (Sec. 3.1, Alg. 1-3, Sec. 3.3 Alg. 5-7)
against the paper's worked example, bitmask enumeration, closed forms and
Burnside counting -- none of which uses the oracle's rank/unrank code."""
import itertools
import json
import math
import os

import numpy as np
import pytest

import workloads as wl
from oracle import native as nat
from oracle.cns import C, F, f_bar, hop
from oracle.translation import Geometry, mk_list, representative, check_state

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.fixture(scope="module", autouse=True)
def _build():
    nat.build(force=False)


def test_worked_example():
    ex = GOLD["worked_example"]
    assert F(tuple(ex["n"])) == ex["a"]
    assert 1 + sum(math.comb(k, m) for k, m, _ in ex["terms"]) == ex["a"]
    for k, m, v in ex["terms"]:
        assert C(k, m) == v
    assert f_bar(ex["a"], ex["K"], ex["N"]) == tuple(ex["n"])
    # the intermediate s of Alg. 1: s -> s - C(n_m - 1, m)
    s = ex["a"]
    seq = [s]
    n = ex["n"]
    for m in range(ex["K"], 1, -1):
        s -= C(n[m - 1] - 1, m)
        seq.append(s)
    assert seq == ex["s_sequence"]
    # C oracle agrees
    assert list(nat.f_bar(8, 4, np.array([50], dtype=np.uint64))[0]) == ex["n"]
    assert int(nat.F(8, 4, np.array([ex["n"]]))[0]) == 50


def _gosper_masks(N, K):
    """All N-bit masks with K ones in ascending numeric order (Gosper's hack)."""
    if K == 0:
        yield 0
        return
    v = (1 << K) - 1
    while v < (1 << N):
        yield v
        c = v & -v
        r = v + c
        v = (((r ^ v) >> 2) // c) | r


@pytest.mark.parametrize("N,K", [(8, 3), (10, 1), (10, 5), (12, 6), (13, 4)])
def test_rank_is_ascending_bitmask_order(N, K):
    for pos, mask in enumerate(_gosper_masks(N, K), start=1):
        n = tuple(i + 1 for i in range(N) if mask >> i & 1)
        assert F(n) == pos
        assert f_bar(pos, K, N) == n


@pytest.mark.parametrize("N,K", [(24, 5), (20, 10), (24, 1), (17, 16)])
def test_bijection_all_ranks_c_oracle(N, K):
    D = math.comb(N, K)
    a = np.arange(1, D + 1, dtype=np.uint64)
    n = nat.f_bar(N, K, a)
    assert np.all(np.diff(n, axis=1) > 0) and n.min() >= 1 and n.max() <= N
    assert np.array_equal(nat.F(N, K, n), a)
    # all tuples distinct and exactly the K-subsets
    assert len({tuple(r) for r in n}) == D


def test_boundary_and_64bit_ranks():
    for N, K in [(16, 3), (100, 4), (1000, 3), (1000, 4)]:
        assert f_bar(1, K, N) == tuple(range(1, K + 1))
        assert f_bar(math.comb(N, K), K, N) == tuple(range(N - K + 1, N + 1))
    D = math.comb(1000, 4)
    assert D == 41417124750 and D > 2 ** 32
    rng = np.random.default_rng(7)
    a = np.concatenate([rng.integers(1, D + 1, size=2000, dtype=np.uint64),
                        np.array([1, 2, 2 ** 32 - 1, 2 ** 32, 2 ** 32 + 1, D - 1, D], dtype=np.uint64)])
    n = nat.f_bar(1000, 4, a)
    assert np.array_equal(nat.F(1000, 4, n), a)
    for i in range(20):
        assert f_bar(int(a[i]), 4, 1000) == tuple(int(x) for x in n[i])


def test_hop_matches_bit_operations():
    """The exchanged state of a bond with one end down is the bitmask with both
    bond bits flipped (mask ^ (1 << i) ^ (1 << j)): no tuple code involved."""
    N, K = 9, 4
    for mask in _gosper_masks(N, K):
        n = tuple(i + 1 for i in range(N) if mask >> i & 1)
        for r in range(1, N + 1):
            for rp in range(r + 1, N + 1):
                if ((mask >> (r - 1)) & 1) == ((mask >> (rp - 1)) & 1):
                    continue
                m2 = mask ^ (1 << (r - 1)) ^ (1 << (rp - 1))
                assert hop(n, r, rp) == tuple(i + 1 for i in range(N) if m2 >> i & 1)


def _burnside_dim(dims, K, Kvec):
    """d_k = (1/N) sum_t e^{ik.t} Fix(t), Fix(t) = C(N/o, K/o) if the order o of t
    divides K (every cycle of T^t has length o), else 0."""
    lx, ly, lz = dims
    N = lx * ly * lz
    tot = 0.0
    for tz in range(lz):
        for ty in range(ly):
            for tx in range(lx):
                o = math.lcm(lx // math.gcd(tx, lx), ly // math.gcd(ty, ly), lz // math.gcd(tz, lz))
                fix = math.comb(N // o, K // o) if K % o == 0 else 0
                ph = 2 * math.pi * (Kvec[0] * tx / lx + Kvec[1] * ty / ly + Kvec[2] * tz / lz)
                tot += math.cos(ph) * fix
    return round(tot / N)


def test_paper_dimensions_burnside():
    d = GOLD["dimensions"]
    assert math.comb(216, 5) == d["cubic6_K5_u1"]
    assert _burnside_dim((6, 6, 6), 5, (0, 0, 0)) == d["cubic6_K5_k0"]
    assert math.comb(1000, 3) == d["cubic10_K3_u1"]
    assert _burnside_dim((10, 10, 10), 3, (0, 0, 0)) == d["cubic10_K3_u1"] // 1000


@pytest.mark.parametrize("dims,K", [((8, 1, 1), 4), ((6, 1, 1), 3), ((4, 4, 1), 4), ((4, 2, 1), 2),
                                    ((3, 3, 1), 3), ((2, 2, 2), 4), ((6, 2, 1), 2)])
def test_mk_list_dims_burnside_python(dims, K):
    geo = Geometry(*dims)
    tot = 0
    for kz in range(dims[2]):
        for ky in range(dims[1]):
            for kx in range(dims[0]):
                sigma, R = mk_list(geo, K, (kx, ky, kz))
                assert len(sigma) == _burnside_dim(dims, K, (kx, ky, kz))
                # R^2 = N * |stabiliser|, an integer multiple of N
                for r in R:
                    s = r * r / geo.N
                    assert abs(s - round(s)) < 1e-9 and round(s) >= 1
                tot += len(sigma)
    assert tot == math.comb(geo.N, K)


@pytest.mark.parametrize("Kvec", [(0, 0, 0), (1, 0, 0), (5, 5, 0), (2, 4, 0), (5, 0, 0)])
def test_mk_list_dims_c2_c_oracle(Kvec):
    sigma, R = nat.mk_list((10, 10, 1), 4, Kvec)
    assert len(sigma) == _burnside_dim((10, 10, 1), 4, Kvec)
    assert len(sigma) == (39249 if (Kvec[0] % 2 == 0 and Kvec[1] % 2 == 0) else 39200)
    assert np.all(np.diff(sigma.astype(np.int64)) > 0)


def test_representative_is_orbit_minimum_bitmask():
    """The representative search returns the orbit minimum, computed
    independently on bitmasks, and a translation reaching it."""
    dims = (4, 3, 1)
    geo = Geometry(*dims)
    N, K = geo.N, 3

    def translate_mask(mask, t):
        out = 0
        for i in range(N):
            if mask >> i & 1:
                x, y, z = i % dims[0], (i // dims[0]) % dims[1], 0
                j = (x + t[0]) % dims[0] + dims[0] * ((y + t[1]) % dims[1])
                out |= 1 << j
        return out

    masks = list(_gosper_masks(N, K))
    pos = {m: i + 1 for i, m in enumerate(masks)}
    for m in masks:
        orbit = [translate_mask(m, (tx, ty, 0)) for tx in range(4) for ty in range(3)]
        rep, ell = representative(geo, pos[m], K)
        assert rep == pos[min(orbit)]
        assert translate_mask(m, geo.t(ell)) == min(orbit)
    # C oracle agrees on a batch
    a = np.arange(1, len(masks) + 1, dtype=np.uint64)
    rep_c, ell_c = nat.representative(dims, K, a)
    for i in range(len(masks)):
        assert (int(rep_c[i]), int(ell_c[i])) == representative(geo, i + 1, K)


def test_check_state_compatibility():
    """N_{a,k} = N * |stab| when e^{ik.t} = 1 on the stabiliser, else 0 (the
    norm of Eq. (akstate); Alg. 5 computes the same)."""
    geo = Geometry(6, 1, 1)
    a = F((1, 4))                  # {1, 4} on a 6-ring: stabiliser {0, 3}
    assert check_state(geo, a, 2, (0, 0, 0)) == pytest.approx(12.0)
    assert check_state(geo, a, 2, (2, 0, 0)) == pytest.approx(12.0)
    assert check_state(geo, a, 2, (1, 0, 0)) == 0.0
    assert check_state(geo, F((1, 2)), 2, (1, 0, 0)) == pytest.approx(6.0)


@pytest.mark.parametrize("make,ns,deg", [(lambda: wl.kagome(3, 4), 3, 4), (lambda: wl.honeycomb(4, 3), 2, 3),
                                         (lambda: wl.kagome(2, 2), 3, 4), (lambda: wl.pyrochlore(2), 4, 6),
                                         (lambda: wl.pyrochlore(3), 4, 6)])
def test_cell_lattices(make, ns, deg):
    """The unit-cell workloads: sites = ns * cells, every site has the
    lattice's coordination, each bond appears once, and the bond set is mapped
    onto itself by a translation of the cells (sublattice kept)."""
    lat = make()
    assert lat.ns == ns and lat.n_sites == ns * lat.lx * lat.ly * lat.lz
    d = np.zeros(lat.n_sites, int)
    seen = set()
    for i, j in zip(lat.bi, lat.bj):
        key = (min(i, j), max(i, j))
        assert key not in seen and i != j
        seen.add(key)
        d[i] += 1
        d[j] += 1
    assert np.all(d == deg)
    assert lat.n_bonds == lat.n_sites * deg // 2

    def tr(i, ax):
        s, c = i % ns, i // ns
        x, y, z = c % lat.lx, (c // lat.lx) % lat.ly, c // (lat.lx * lat.ly)
        x, y, z = [(v + 1) % L if a == ax else v for a, (v, L) in enumerate(zip((x, y, z), lat.dims))]
        return s + ns * (x + lat.lx * (y + lat.ly * z))
    for ax in range(3 if lat.lz > 1 else 2):
        moved = {(min(tr(i, ax), tr(j, ax)), max(tr(i, ax), tr(j, ax))) for i, j in seen}
        assert moved == seen


def test_pyrochlore_geometry():
    """Pyrochlore from its geometry alone: with the fcc cell vectors a1 =
    (0, 1/2, 1/2), a2 = (1/2, 0, 1/2), a3 = (1/2, 1/2, 0) and the places at
    0 and a_s / 2, the bonds are exactly the pairs at the nearest-neighbour
    distance sqrt(2)/4 (minimum image over the periodic 3 x 3 x 3 cells)."""
    lat = wl.pyrochlore(3)
    A = np.array([[0, .5, .5], [.5, 0, .5], [.5, .5, 0]])
    N, L = lat.n_sites, 3
    frac = np.zeros((N, 3))
    for i in range(N):
        s, c = i % 4, i // 4
        frac[i] = (c % L, (c // L) % L, c // (L * L))
        frac[i] += np.array(lat.basis[s])
    pairs = set()
    for i in range(N):
        for j in range(i + 1, N):
            df = frac[j] - frac[i]
            df -= L * np.round(df / L)
            if abs(np.linalg.norm(df @ A) - np.sqrt(2) / 4) < 1e-12:
                pairs.add((i, j))
    assert pairs == {(min(i, j), max(i, j)) for i, j in zip(lat.bi, lat.bj)}

