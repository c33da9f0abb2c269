"""GPU parity of the basis, H.v and row structure against the CPU oracle.

Integer work (representatives, stabilisers, row sparsity patterns, start
vectors) must match bit for bit.  H.v values use the tolerances of
tests/tolerances.py, derived from the oracle's bond-by-bond accumulation.
"""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import native as orc
from oracle.rng import start_vector as orc_start
from tolerances import hv_tol, hv_tol32

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qs3():
    from paper_2107_00872_amd import qs3 as q
    assert torch.cuda.is_available()
    orc.build(force=False)
    return q


@pytest.fixture(scope="module")
def ctx(qs3):
    c = qs3.Context(0)
    yield c


def _scale(lat):
    return max(1.0, float(np.abs(lat.jxy).max()), float(np.abs(lat.jz).max()))


U1_CASES = [(wl.chain(16), 3), (wl.chain(16), 0), (wl.chain(8), 8), (wl.chain(12), 1),
            (wl.square(6), 3), (wl.random_bonds(20, 45, seed=2), 5),
            (wl.with_disorder(wl.square(5), seed=3), 4), (wl.cube(4), 2), (wl.chain(40), 7)]


@pytest.mark.parametrize("lat,K", U1_CASES, ids=lambda x: getattr(x, "name", str(x)))
def test_u1_matvec_full(qs3, ctx, lat, K):
    L = qs3.Lattice.of(ctx, lat)
    sec = qs3.Sector(L, K)
    assert sec.dim == math.comb(lat.n_sites, K)
    v = torch.empty(sec.dim, dtype=torch.float64, device="cuda")
    sec.start_vector(7, v)
    vh = v.cpu().numpy()
    assert np.array_equal(vh, orc_start(7, np.arange(sec.dim), complex_=False))
    w = torch.empty_like(v)
    sec.matvec(v, w)
    ref = orc.hv_u1(lat.n_sites, K, orc.Bonds.of(lat), vh)
    assert np.abs(w.cpu().numpy() - ref).max() <= hv_tol(lat, np.abs(vh).max())
    # float32 rows
    v32 = v.float()
    w32 = torch.empty_like(v32)
    sec.matvec(v32, w32)
    assert np.abs(w32.cpu().numpy() - ref).max() <= hv_tol32(lat, np.abs(vh).max(), K)
    # determinism: same bits twice
    w2 = torch.empty_like(v)
    sec.matvec(v, w2)
    assert torch.equal(w, w2)


@pytest.mark.parametrize("lat,K", [(wl.chain(16), 3), (wl.square(10), 4), (wl.random_bonds(20, 45, 2), 5),
                                   (wl.cube(10), 3), (wl.cube(10), 4)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_u1_row_pattern_bit_exact(qs3, ctx, lat, K):
    """The sparsity pattern and values of sampled rows, as formed on the device,
    equal the oracle's (Alg. 4 order differs; compare sorted)."""
    L = qs3.Lattice.of(ctx, lat)
    sec = qs3.Sector(L, K)
    B = orc.Bonds.of(lat)
    rng = np.random.default_rng(3)
    rows = list(rng.integers(0, sec.dim, size=60)) + [0, sec.dim - 1]
    for r in rows:
        dg, cols, vals = sec.row(int(r))
        odg, ocols, ovals = orc.row_u1(lat.n_sites, K, B, int(r) + 1)
        assert sorted(zip(cols.tolist(), vals.tolist())) == sorted(zip(ocols.astype(np.int64).tolist(), ovals.tolist()))
        assert abs(dg - odg) <= 1e-13 * _scale(lat) * lat.n_bonds


@pytest.mark.parametrize("lat,K", [(wl.square(10), 4), (wl.cube(10), 3)], ids=["C2-full-sector", "cube10-K3"])
def test_u1_matvec_full_size_sampled(qs3, ctx, lat, K):
    """Full-size sectors in the benchmark's launch configuration, checked on
    sampled rows computed one by one by the oracle."""
    L = qs3.Lattice.of(ctx, lat)
    sec = qs3.Sector(L, K)
    v = torch.empty(sec.dim, dtype=torch.float64, device="cuda")
    sec.start_vector(11, v)
    w = torch.empty_like(v)
    sec.matvec(v, w)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    rows = np.unique(np.concatenate([rng.integers(0, sec.dim, size=3000), [0, 1, sec.dim - 1]]))
    vh = v.cpu().numpy()
    ref = orc.hv_u1(lat.n_sites, K, orc.Bonds.of(lat), vh, rows=rows + 1)
    got = w.cpu().numpy()[rows]
    assert np.abs(got - ref).max() <= hv_tol(lat, np.abs(vh).max())


K_CASES = [((8, 1, 1), wl.chain(8), 3), ((6, 1, 1), wl.chain(6), 2), ((4, 4, 1), wl.square(4), 2),
           ((4, 4, 1), wl.square(4), 4), ((4, 2, 1), wl.hypercubic(4, 2, 1), 3),
           ((3, 3, 3), wl.cube(3), 2), ((4, 4, 1), wl.with_disorder(wl.square(4), 9, per_bond=False), 3),
           ((12, 1, 1), wl.chain(12), 6), ((4, 4, 1), wl.square(4), 0), ((5, 5, 1), wl.square(5), 1)]


@pytest.mark.parametrize("dims,lat,K", K_CASES, ids=lambda x: getattr(x, "name", str(x)))
def test_k_basis_and_matvec(qs3, ctx, dims, lat, K):
    L = qs3.Lattice.of(ctx, lat)
    assert L.info()[1]
    B = orc.Bonds.of(lat)
    for Kv in wl.all_momenta(lat):
        sigma, R = orc.mk_list(dims, K, Kv)
        if len(sigma) == 0:
            continue
        sec = qs3.Sector(L, K, Kv)
        ranks, stab = sec.basis()
        # representatives bit-exact; N_{a,k} = N * stab
        assert np.array_equal(ranks, sigma - 1)
        assert np.allclose(R * R, lat.n_sites * stab.astype(float), rtol=0, atol=1e-9)
        v = torch.empty(sec.dim, dtype=torch.complex128, device="cuda")
        sec.start_vector(3, v)
        vh = v.cpu().numpy()
        assert np.array_equal(vh, orc_start(3, sigma - 1, complex_=True))
        w = torch.empty_like(v)
        sec.matvec(v, w)
        ref = orc.hv_k(dims, K, Kv, B, sigma, R, vh)
        assert np.abs(w.cpu().numpy() - ref).max() <= hv_tol(lat, np.abs(vh).max() * 1.5)
        # row structure: columns bit-exact, values within rounding
        for r in list(range(min(sec.dim, 6))) + [sec.dim - 1]:
            dg, cols, vals = sec.row(r)
            odg, ocols, ovals = orc.row_k(dims, K, Kv, B, sigma, R, r + 1)
            # merge duplicate targets (several hops can land in one orbit)
            def merged(c, x):
                d = {}
                for a, b in zip(c.tolist(), x.tolist()):
                    d[a] = d.get(a, 0) + b
                return d
            m1, m2 = merged(cols, vals), merged(ocols, ovals)
            assert set(m1) == set(m2)
            for key in m1:
                assert abs(m1[key] - m2[key]) <= 1e-13 * _scale(lat) * 8
            assert abs(dg - odg) <= 1e-13 * _scale(lat) * lat.n_bonds
        # float32 rows
        w32 = torch.empty(sec.dim, dtype=torch.complex64, device="cuda")
        sec.matvec(v.to(torch.complex64), w32)
        assert np.abs(w32.cpu().numpy() - ref).max() <= hv_tol32(lat, np.abs(vh).max() * 1.5, K)
        sec.close()


def test_k_sector_64bit_ranks_cube10_k4(qs3, ctx):
    """The periodic 10^3 cube at N_down = 4, k = 0: C(1000, 4) = 4.1e10 ranks
    (64-bit ranks, hop lists).  Sampled representatives are orbit minima with
    the oracle's stabiliser sizes (Alg. 5/7 at N = 1000); the uniform
    superposition sqrt(N / s_a) per representative -- (S^-_tot)^4 of the
    ferromagnet -- is an eigenvector with E_FM = 3000 / 4; H is Hermitian on
    seeded random vectors."""
    from oracle.translation import Geometry, check_state
    lat = wl.cube(10)
    L = qs3.Lattice.of(ctx, lat)
    sec = qs3.Sector(L, 4, (0, 0, 0))
    ranks, stab = sec.basis()
    N = lat.n_sites
    assert ranks.dtype == np.uint64 and int(ranks[-1]) >= 2 ** 32
    # Burnside: the number of orbits is the mean number of states a
    # translation fixes, C(N/o, K/o) for a translation of order o dividing K
    fixed = 0
    for tx in range(10):
        for ty in range(10):
            for tz in range(10):
                o = math.lcm(10 // math.gcd(tx, 10), 10 // math.gcd(ty, 10), 10 // math.gcd(tz, 10))
                fixed += math.comb(N // o, 4 // o) if 4 % o == 0 else 0
    assert fixed % N == 0 and sec.dim == fixed // N
    rng = np.random.default_rng(7)
    idx = np.unique(np.concatenate([rng.integers(0, sec.dim, size=60), [0, sec.dim - 1]]))
    geo = Geometry(10, 10, 10)
    reps1 = ranks[idx].astype(np.uint64) + np.uint64(1)
    mins, _ = orc.representative((10, 10, 10), 4, reps1)
    assert np.array_equal(mins, reps1)
    for i in idx[:20]:
        assert check_state(geo, int(ranks[i]) + 1, 4, (0, 0, 0)) == pytest.approx(N * int(stab[i]), abs=1e-6)
    phi = torch.from_numpy(np.sqrt(N / stab.astype(np.float64))).to(torch.complex128).cuda()
    w = torch.empty_like(phi)
    sec.matvec(phi, w)
    assert (w - 750.0 * phi).abs().max().item() <= 1e-10 * 750.0 * phi.abs().max().item()
    u = torch.empty_like(phi)
    v = torch.empty_like(phi)
    sec.start_vector(1, u)
    sec.start_vector(2, v)
    hu, hv = torch.empty_like(u), torch.empty_like(v)
    sec.matvec(u, hu)
    sec.matvec(v, hv)
    lhs, rhs = torch.vdot(u, hv).item(), torch.vdot(hu, v).item()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    sec.close()


def test_k_sector_large_hop_lists_vs_on_the_fly(qs3, ctx, ctx_fly):
    """A momentum sector of 41,417,000 representatives (10^3 cube, N_down = 4,
    k = (5, 0, 0)) takes the single-sector hop-list product with one lane per
    row; k = (5, 0, 0) excludes the orbits whose stabiliser holds a translation
    with odd x component, so rows and targets of class 0 occur.  Its H.v
    (float64 and float32 rows) must equal the product that canonicalises
    every hop on the fly -- the kernel checked element by element against
    Alg. 9 on every lattice of K_CASES -- within rounding, and be Hermitian."""
    lat = wl.cube(10)
    Kv = (5, 0, 0)
    sec = qs3.Sector(qs3.Lattice.of(ctx, lat), 4, Kv)
    fly = qs3.Sector(qs3.Lattice.of(ctx_fly, lat), 4, Kv)
    assert sec.dim == fly.dim and sec.dim > (2 << 20)
    r1, s1 = sec.basis()
    r2, s2 = fly.basis()
    assert np.array_equal(r1, r2) and np.array_equal(s1, s2)
    assert (s1 > 1).any()
    v = torch.empty(sec.dim, dtype=torch.complex128, device="cuda")
    sec.start_vector(9, v)
    w, wf = torch.empty_like(v), torch.empty_like(v)
    sec.matvec(v, w)
    fly.matvec(v, wf)
    vmax = v.abs().max().item()
    assert (w - wf).abs().max().item() <= hv_tol(lat, vmax * 1.5)
    w32 = torch.empty(sec.dim, dtype=torch.complex64, device="cuda")
    sec.matvec(v.to(torch.complex64), w32)
    assert (w32.to(torch.complex128) - wf).abs().max().item() <= hv_tol32(lat, vmax * 1.5, 4)
    u = torch.empty_like(v)
    sec.start_vector(10, u)
    hu = torch.empty_like(u)
    sec.matvec(u, hu)
    lhs, rhs = torch.vdot(u, w).item(), torch.vdot(hu, v).item()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    sec.close()
    fly.close()


@pytest.mark.parametrize("nsec,split", [(1000, (4, 250)), (601, (3, 201))], ids=["1000-sectors", "601-ragged"])
def test_wide_batch_in_sector_groups(qs3, ctx, nsec, split):
    """The momentum sectors of the 10^3 cube at N_down = 3 (2.66 GB vectors
    for all 1000 of them) run their batched H.v as launches over groups of at
    most 256 sectors with the whole batch's row stride: 4 x 250 for 1000
    sectors, 201 + 201 + 199 for 601.  Every float64 column must equal, bit
    for bit, the same sector's column from a 64-sector batch that runs in one
    launch: every schedule sums a sector's hops in hop order.  Float32 rows
    agree within their rounding bound (instances of other widths may contract
    the complex multiply-adds differently)."""
    lat = wl.cube(10)
    L = qs3.Lattice.of(ctx, lat)
    ks = wl.all_momenta(lat)[:nsec]
    pick = sorted(np.random.default_rng(11).choice(len(ks), 64, replace=False).tolist())
    big = qs3.Batch(L, 3, ks)
    small = qs3.Batch(L, 3, [ks[i] for i in pick])
    assert big.rows == small.rows
    gen = torch.Generator(device="cuda").manual_seed(5)
    v = torch.complex(torch.rand(big.rows, big.B, dtype=torch.float64, device="cuda", generator=gen) - 0.5,
                      torch.rand(big.rows, big.B, dtype=torch.float64, device="cuda", generator=gen) - 0.5)
    idx = torch.tensor(pick, device="cuda")
    vs = v.index_select(1, idx).contiguous()
    for dt in (torch.complex128, torch.complex64):
        w = torch.empty(big.rows, big.B, dtype=dt, device="cuda")
        ws = torch.empty(small.rows, small.B, dtype=dt, device="cuda")
        big.matvec(v.to(dt), w)
        assert big.groups() == split
        small.matvec(vs.to(dt), ws)
        assert small.groups() == (1, 64)
        if dt == torch.complex128:
            assert torch.equal(w.index_select(1, idx), ws)
        else:
            d = (w.index_select(1, idx) - ws).abs().max().item()
            assert math.isfinite(d)
            assert d <= hv_tol32(lat, 0.75, 3), d
        del w, ws
    big.close()
    small.close()


@pytest.fixture(scope="module")
def ctx_fly(qs3):
    """A context that never builds rank tables: every hop is resolved by
    on-the-fly canonicalisation and a directory search."""
    c = qs3.Context(0)
    c.set_structure_limits(0, 0)
    yield c


@pytest.fixture(scope="module")
def ctx_hops(qs3):
    """A context that resolves hops through per-representative hop lists."""
    c = qs3.Context(0)
    c.set_structure_limits(0, 1 << 34)
    yield c


@pytest.fixture(scope="module")
def ctx_table(qs3):
    """A context that resolves hops through the rank table only."""
    c = qs3.Context(0)
    c.set_structure_limits(1 << 34, 0)
    yield c


@pytest.mark.parametrize("dims,lat,K", K_CASES, ids=lambda x: getattr(x, "name", str(x)))
def test_k_basis_and_matvec_rank_table(qs3, ctx_table, dims, lat, K):
    test_k_basis_and_matvec(qs3, ctx_table, dims, lat, K)


@pytest.mark.parametrize("dims,lat,K", K_CASES, ids=lambda x: getattr(x, "name", str(x)))
def test_k_basis_and_matvec_on_the_fly(qs3, ctx_fly, dims, lat, K):
    test_k_basis_and_matvec(qs3, ctx_fly, dims, lat, K)


@pytest.mark.parametrize("dims,lat,K", K_CASES, ids=lambda x: getattr(x, "name", str(x)))
def test_k_basis_and_matvec_hop_lists(qs3, ctx_hops, dims, lat, K):
    test_k_basis_and_matvec(qs3, ctx_hops, dims, lat, K)


def test_k_c2_sampled_sectors(qs3, ctx):
    """C2 10x10 N_down=4 momentum sectors: sector dimensions (Burnside values
    39249 / 39200) and full H.v against the oracle's Alg. 9 for a sample of k."""
    lat = wl.square(10)
    L = qs3.Lattice.of(ctx, lat)
    B = orc.Bonds.of(lat)
    for Kv in [(0, 0, 0), (1, 0, 0), (5, 5, 0), (3, 7, 0)]:
        sec = qs3.Sector(L, 4, Kv)
        assert sec.dim == (39249 if Kv[0] % 2 == 0 and Kv[1] % 2 == 0 else 39200)
        sigma, R = orc.mk_list(lat.dims, 4, Kv)
        ranks, stab = sec.basis()
        assert np.array_equal(ranks, sigma - 1)
        v = torch.empty(sec.dim, dtype=torch.complex128, device="cuda")
        sec.start_vector(5, v)
        w = torch.empty_like(v)
        sec.matvec(v, w)
        rows = np.arange(1, sec.dim + 1, 7)
        ref = orc.hv_k(lat.dims, 4, Kv, B, sigma, R, v.cpu().numpy(), rows=rows)
        assert np.abs(w.cpu().numpy()[rows - 1] - ref).max() <= hv_tol(lat, 1.5)
        sec.close()


@pytest.mark.parametrize("lat,K", [(wl.square(4), 2), (wl.square(6), 3), (wl.chain(12), 4), (wl.cube(3), 3)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_batch_all_k_equals_single_sectors(qs3, ctx, lat, K):
    """One batched launch over every momentum equals the oracle per sector."""
    L = qs3.Lattice.of(ctx, lat)
    ks = wl.all_momenta(lat)
    bat = qs3.Batch(L, K, ks)
    B = orc.Bonds.of(lat)
    v = torch.zeros(bat.rows, bat.B, dtype=torch.complex128, device="cuda")
    rng = np.random.default_rng(1)
    vh = (rng.normal(size=(bat.rows, bat.B)) + 1j * rng.normal(size=(bat.rows, bat.B)))
    v.copy_(torch.from_numpy(vh))
    w = torch.empty_like(v)
    bat.matvec(v, w)
    wh = w.cpu().numpy()
    # union of representatives = all orbit minima
    sig0, _ = orc.mk_list(lat.dims, K, (0, 0, 0))
    for b, Kv in enumerate(ks):
        sigma, R = orc.mk_list(lat.dims, K, Kv)
        assert bat.dims[b] == len(sigma)
        if len(sigma) == 0:
            continue
        # positions of this sector's representatives in the union
        sec = qs3.Sector(L, K, Kv)
        ranks, _ = sec.basis()
        sec.close()
        uni_all = _union_ranks(qs3, ctx, L, K, lat)
        pos = np.searchsorted(uni_all, sigma - 1)
        assert np.array_equal(uni_all[pos], sigma - 1)
        ref = orc.hv_k(lat.dims, K, Kv, B, sigma, R, vh[pos, b])
        assert np.abs(wh[pos, b] - ref).max() <= hv_tol(lat, np.abs(vh).max())
        # rows of incompatible representatives are zero
        mask = np.ones(bat.rows, bool)
        mask[pos] = False
        assert np.all(wh[mask, b] == 0)
    bat.close()


_UNI = {}


@pytest.mark.parametrize("lat,K", [(wl.square(6), 3), (wl.cube(3), 3), (wl.hypercubic(4, 2, 2), 4)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_batch_all_k_on_the_fly(qs3, ctx_fly, lat, K):
    test_batch_all_k_equals_single_sectors(qs3, ctx_fly, lat, K)


@pytest.mark.parametrize("lat,K", [(wl.square(6), 3), (wl.cube(3), 3), (wl.hypercubic(4, 2, 2), 4),
                                   (wl.with_disorder(wl.square(4), 9, per_bond=False), 3)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_batch_all_k_hop_lists(qs3, ctx_hops, lat, K):
    test_batch_all_k_equals_single_sectors(qs3, ctx_hops, lat, K)


def _union_ranks(qs3, ctx, L, K, lat):
    key = (lat.name, K)
    if key not in _UNI:
        # every orbit has a representative compatible with k = 0 except orbits
        # whose stabiliser meets k = 0 trivially -- k = 0 is compatible with all
        sec = qs3.Sector(L, K, (0, 0, 0))
        r, _ = sec.basis()
        sec.close()
        _UNI[key] = r
    return _UNI[key]


# Wide batches: more sectors than one wavefront of lanes, so each lane owns
# several sectors (ceil(B / 64) per lane, rounded up to 2, 4, 8, 16 or 32),
# the instances the full momentum sweeps launch (10x10: 100 sectors, 2 per
# lane; 10^3: 1000 sectors, 16 per lane).
WIDE = [(wl.square(10), 3, None), (wl.square(12), 2, None), (wl.square(20), 2, 24),
        (wl.cube(10), 2, 20), (wl.cube(12), 2, 10)]


def _wide_batch(qs3, c, lat, K, n_sample):
    L = qs3.Lattice.of(c, lat)
    ks = wl.all_momenta(lat)
    bat = qs3.Batch(L, K, ks)
    per = -(-bat.B // 64)
    assert bat.B > 64 and per >= 2
    B = orc.Bonds.of(lat)
    rng = np.random.default_rng(3)
    vh = rng.uniform(-1, 1, size=(bat.rows, bat.B)) + 1j * rng.uniform(-1, 1, size=(bat.rows, bat.B))
    v = torch.from_numpy(vh).cuda()
    w = torch.empty_like(v)
    bat.matvec(v, w)
    wh = w.cpu().numpy()
    # the union of representatives: every orbit minimum, i.e. the k = 0 sector
    sig0, _ = orc.mk_list(lat.dims, K, (0, 0, 0))
    assert bat.rows == len(sig0)
    pick = range(bat.B) if n_sample is None else sorted(
        set(rng.choice(bat.B, n_sample, replace=False).tolist()) | {0, bat.B - 1})
    for b in pick:
        Kv = ks[b]
        sigma, R = orc.mk_list(lat.dims, K, Kv)
        assert bat.dims[b] == len(sigma)
        pos = np.searchsorted(sig0, sigma)
        assert np.array_equal(sig0[pos], sigma)
        ref = orc.hv_k(lat.dims, K, Kv, B, sigma, R, vh[pos, b])
        assert np.abs(wh[pos, b] - ref).max() <= hv_tol(lat, 1.5), (Kv, per)
        mask = np.ones(bat.rows, bool)
        mask[pos] = False
        assert np.all(wh[mask, b] == 0)
    bat.close()
    L.close()


@pytest.mark.parametrize("lat,K,n_sample", WIDE, ids=lambda x: getattr(x, "name", str(x)))
def test_batch_wide_hop_lists(qs3, ctx_hops, lat, K, n_sample):
    """Every sector (or a seeded sample of them) of a wide batch against the
    oracle's Alg. 9, element by element, hops through hop lists."""
    _wide_batch(qs3, ctx_hops, lat, K, n_sample)


@pytest.mark.parametrize("lat,K,n_sample", WIDE, ids=lambda x: getattr(x, "name", str(x)))
def test_batch_wide_rank_table(qs3, ctx_table, lat, K, n_sample):
    _wide_batch(qs3, ctx_table, lat, K, n_sample)


@pytest.mark.parametrize("lat,K,n_sample", WIDE[:2] + WIDE[3:4], ids=lambda x: getattr(x, "name", str(x)))
def test_batch_wide_on_the_fly(qs3, ctx_fly, lat, K, n_sample):
    _wide_batch(qs3, ctx_fly, lat, K, n_sample)
