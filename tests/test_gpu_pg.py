"""Point-group sectors (translations x point operations, one-dimensional real
characters) through the C-ABI against the oracle's construction: the
representatives and their norms bit-exact / to rounding, H.v against the
oracle's dense block, the lowest levels and eigenvectors against dense
diagonalisation; at the 10 x 10 size, sampled rows against rows the oracle
builds one at a time, the identity-only group against the momentum sector,
and the variational bound below every one-dimensional block; and the host
checks that refuse a group or character that is not one."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle.cns import C, F, f_bar
from oracle.hamiltonian import bonds_1based, row_terms
from oracle.lanczos import lowest_distinct
from oracle.pointgroup import _char, check_state_pg, gen_full_ham_pg, mk_list_pg, representative_pg
from oracle.translation import Geometry
from tolerances import EPS64

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qs3():
    from paper_2107_00872_amd import qs3 as q
    assert torch.cuda.is_available()
    return q


@pytest.fixture(scope="module")
def ctx(qs3):
    c = qs3.Context(0)
    yield c
    c.close()


def _ops(lat):
    if lat.ns == 3:
        return wl.kagome_c6v_ops(lat.lx)
    if lat.ns == 2:
        return wl.honeycomb_inversion_ops(lat.lx, lat.ly)
    if lat.lz > 1:
        return wl.oh_ops(lat.lx)
    return wl.c4v_ops(lat.lx) if lat.ly > 1 else wl.inversion_ops(lat.lx)


def _chars(lat):
    if lat.ns == 3:
        return list(wl.C6V_CHARS.items())
    if lat.ns == 2:
        return [("even", (1, 1)), ("odd", (1, -1))]
    if lat.lz > 1:
        return list(wl.oh_chars().items())
    if lat.ly > 1:
        return list(wl.C4V_CHARS.items())
    return [("even", (1, 1)), ("odd", (1, -1))]


CASES = [(wl.square(4), 2, (0, 0, 0)), (wl.square(4), 3, (2, 2, 0)), (wl.square(4), 4, (0, 0, 0)),
         (wl.square(6), 2, (3, 3, 0)), (wl.chain(14), 5, (7, 0, 0)), (wl.chain(12), 6, (0, 0, 0)),
         (wl.with_disorder(wl.square(4), seed=3, per_bond=False), 3, (2, 2, 0)),
         (wl.square_j1j2(4, 0.45), 3, (2, 2, 0)), (wl.square_j1j2(4, 0.45), 4, (0, 0, 0)),
         (wl.cube(3), 2, (0, 0, 0)), (wl.honeycomb(3, 3), 3, (0, 0, 0)), (wl.honeycomb(4, 4), 3, (2, 2, 0)),
         (wl.kagome(2, 2), 3, (0, 0, 0)), (wl.kagome(3, 3), 3, (0, 0, 0))]


def _tol(H, vmax, width):
    # each output sums <= width + 1 products on both sides
    return 2.0 * (width + 2) * EPS64 * np.abs(H).sum(axis=1).max() * max(vmax, 1e-300)


@pytest.mark.parametrize("lat,K,Kv", CASES, ids=lambda x: getattr(x, "name", str(x)))
def test_pg_sector_against_oracle(qs3, ctx, lat, K, Kv):
    perms = _ops(lat)
    geo = Geometry(lat.lx, lat.ly, lat.lz, lat.ns)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    L = qs3.Lattice.of(ctx, lat)
    width = K * int(np.bincount(np.concatenate([lat.bi, lat.bj])).max())  # ELL slots per row
    for name, chars in _chars(lat):
        print(f"pg {lat.name} K={K} k={Kv} {name}", flush=True)
        sigma, R = mk_list_pg(geo, perms, chars, K, Kv)
        sec = qs3.PGSector(L, K, Kv, perms, chars)
        assert sec.dim == len(sigma)
        ranks, norms = sec.basis()
        assert np.array_equal(ranks.astype(np.int64), np.array(sigma, dtype=np.int64) - 1)
        if not sigma:
            sec.close()
            continue
        assert np.allclose(norms, np.array(R) ** 2, rtol=1e-13, atol=0)
        H = gen_full_ham_pg(geo, perms, chars, K, bonds, sigma, R, Kv)
        rng = np.random.default_rng(11)
        vh = rng.normal(size=sec.dim)
        v = torch.from_numpy(vh).cuda()
        w = torch.empty_like(v)
        sec.matvec(v, w)
        torch.cuda.synchronize()
        assert np.abs(w.cpu().numpy() - H @ vh).max() <= _tol(H, np.abs(vh).max(), width)
        ref = np.linalg.eigvalsh(H)
        nev = min(3, len(set(np.round(ref, 8))))
        X = torch.zeros(nev * sec.dim, dtype=torch.float64, device="cuda")
        res = sec.eigs(nev=nev, evecs=X, seed=3)
        assert res.status == qs3.QS3_OK
        want = lowest_distinct(ref, nev)
        assert np.allclose(res.evals, want, rtol=0, atol=1e-9 * max(1.0, np.abs(want).max()))
        Xh = X.cpu().numpy().reshape(nev, sec.dim)
        for y in range(nev):
            x = Xh[y]
            assert abs(np.linalg.norm(x) - 1.0) < 1e-9
            assert np.linalg.norm(H @ x - res.evals[y] * x) < 1e-7 * max(1.0, abs(res.evals[y]))
        sec.close()
    L.close()


def _oracle_row(geo, perms, chars, K, bonds, Kv, a):
    """Row of the (k, chi) block at the 0-based representative rank a, one
    hop at a time (representative_pg and check_state_pg give each target's
    rank and norm): (diag, {target rank: element})."""
    Na = check_state_pg(geo, perms, chars, a + 1, K, Kv)
    diag, offs = row_terms(f_bar(a + 1, K, geo.N), bonds)
    out = {}
    for (np_, jhalf) in offs:
        rep, p, t = representative_pg(geo, perms, F(np_), K)
        Nb = check_state_pg(geo, perms, chars, rep, K, Kv)
        if Nb > 0:
            out[rep - 1] = out.get(rep - 1, 0.0) + jhalf * _char(geo, chars, Kv, p, t) * math.sqrt(Nb / Na)
    return diag, out


SAMPLED = [("square10", 4, (0, 0, 0)), ("square10", 4, (5, 5, 0)), ("kagome12", 3, (0, 0, 0))]


@pytest.mark.parametrize("which,K,Kv", SAMPLED)
def test_pg_full_size_sampled_rows(qs3, ctx, which, K, Kv):
    """Full size (the 10 x 10 square with C4v, the 12 x 12 kagome with C6v):
    rows sampled from orbits the oracle picks (random ranks mapped to their
    representatives) against the oracle's row, as columns of H (the block is
    symmetric)."""
    if which == "square10":
        lat, perms, charsets = wl.square(10), wl.c4v_ops(10), list(wl.C4V_CHARS.items())[::3]
    else:
        lat, perms, charsets = wl.kagome(12, 12), wl.kagome_c6v_ops(12), list(wl.C6V_CHARS.items())[::3]
    geo = Geometry(lat.lx, lat.ly, lat.lz, lat.ns)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    L = qs3.Lattice.of(ctx, lat)
    rng = np.random.default_rng(2)
    for name, chars in charsets:
        print(f"pg {lat.name} K={K} k={Kv} {name}", flush=True)
        sec = qs3.PGSector(L, K, Kv, perms, chars)
        ranks, norms = sec.basis()
        assert sec.dim > 0 and np.all(np.diff(ranks.astype(np.int64)) > 0)
        pos = {int(r): i for i, r in enumerate(ranks)}
        picked = 0
        while picked < 3:
            a = representative_pg(geo, perms, int(rng.integers(1, C(geo.N, K) + 1)), K)[0] - 1
            Na = check_state_pg(geo, perms, chars, a + 1, K, Kv)
            if Na == 0:
                assert a not in pos
                continue
            picked += 1
            assert a in pos and abs(norms[pos[a]] - Na) <= 1e-12 * Na
            diag, row = _oracle_row(geo, perms, chars, K, bonds, Kv, a)
            e = torch.zeros(sec.dim, dtype=torch.float64, device="cuda")
            e[pos[a]] = 1.0
            w = torch.empty_like(e)
            sec.matvec(e, w)
            col = w.cpu().numpy()
            want = np.zeros(sec.dim)
            want[pos[a]] += diag
            for bb, x in row.items():
                want[pos[bb]] += x
            assert np.abs(col - want).max() <= 1e-12 * max(1.0, np.abs(want).max())
        sec.close()
    L.close()


@pytest.mark.parametrize("Kv", [(0, 0, 0), (5, 5, 0), (5, 0, 0)])
def test_pg_identity_group_is_momentum_sector(qs3, ctx, Kv):
    """With the identity alone the sector is the momentum sector (k.t = 0 or
    pi makes it real): same representatives, same lowest levels."""
    lat = wl.square(10)
    L = qs3.Lattice.of(ctx, lat)
    ident = np.arange(lat.n_sites, dtype=np.int32)[None, :]
    sec = qs3.PGSector(L, 3, Kv, ident, [1])
    mom = qs3.Sector(L, 3, Kv)
    assert sec.dim == mom.dim
    r_pg, n_pg = sec.basis()
    r_k, _ = mom.basis()
    assert np.array_equal(r_pg, r_k)
    a = sec.eigs(nev=3, seed=1)
    b = mom.eigs(nev=3, seed=1)
    assert a.status == qs3.QS3_OK and b.status == qs3.QS3_OK
    assert np.allclose(a.evals, b.evals, rtol=0, atol=1e-9 * np.abs(b.evals).max())
    sec.close()
    mom.close()
    L.close()


def test_pg_blocks_above_momentum_ground_state(qs3, ctx):
    """Each one-dimensional block is a subspace of the momentum block, so its
    lowest level is at or above the momentum sector's (10 x 10 square,
    N_down = 4, k = 0)."""
    lat = wl.square(10)
    L = qs3.Lattice.of(ctx, lat)
    mom = qs3.Sector(L, 4, (0, 0, 0))
    e0 = mom.eigs(nev=1, seed=1).evals[0]
    for name, chars in wl.C4V_CHARS.items():
        sec = qs3.PGSector(L, 4, (0, 0, 0), wl.c4v_ops(10), chars)
        r = sec.eigs(nev=1, seed=2)
        assert r.status == qs3.QS3_OK
        print(f"pg square10x10 K=4 k=0 {name}: dim {sec.dim} E0 {r.evals[0]:.12f} (momentum {e0:.12f})", flush=True)
        assert r.evals[0] >= e0 - 1e-9 * abs(e0)
        sec.close()
    mom.close()
    L.close()


def test_pg_refuses_non_groups(qs3, ctx):
    lat = wl.square(4)
    L = qs3.Lattice.of(ctx, lat)
    ops = wl.c4v_ops(4)
    A1 = wl.C4V_CHARS["A1"]

    def refused(**kw):
        args = dict(n_down=2, k=(0, 0, 0), perms=ops, chars=A1)
        args.update(kw)
        with pytest.raises(qs3.QS3Error) as ei:
            qs3.PGSector(L, args["n_down"], args["k"], args["perms"], args["chars"])
        assert ei.value.code == qs3.QS3_EINVAL

    refused(k=(2, 0, 0))                       # r90 maps (pi, 0) to (0, pi)
    refused(k=(1, 0, 0))                       # not 0 or pi
    refused(chars=(1, -1, 1, -1, 1, -1, 1, -1))  # not a representation
    refused(perms=ops[:5], chars=A1[:5])       # not closed
    refused(perms=ops[[1, 0, 2, 3, 4, 5, 6, 7]])  # row 0 not the identity
    refused(n_down=7)
    bad = ops.copy()
    bad[1, [0, 1]] = bad[1, [1, 0]]
    refused(perms=bad)                         # breaks the couplings
    L.close()
    D = qs3.Lattice.of(ctx, wl.with_disorder(wl.square(4), seed=3, per_bond=True))
    with pytest.raises(qs3.QS3Error):
        qs3.PGSector(D, 2, (0, 0, 0), ops, A1)
    D.close()
    # several places per cell: a map that does not keep the couplings is
    # refused, the identity alone gives the momentum sector
    kag = qs3.Lattice.of(ctx, wl.kagome(2, 2))
    swap = np.arange(12, dtype=np.int32)
    swap[[0, 1]] = swap[[1, 0]]
    with pytest.raises(qs3.QS3Error):
        qs3.PGSector(kag, 2, (0, 0, 0), np.stack([np.arange(12, dtype=np.int32), swap]), [1, 1])
    ident = qs3.PGSector(kag, 2, (0, 0, 0), np.arange(12, dtype=np.int32)[None, :], [1])
    mom = qs3.Sector(kag, 2, (0, 0, 0))
    assert ident.dim == mom.dim
    ident.close()
    mom.close()
    kag.close()


@pytest.mark.parametrize("lat,K,Kv", [(wl.square(4), 3, (2, 2, 0)), (wl.square(4), 4, (0, 0, 0)),
                                      (wl.chain(12), 4, (6, 0, 0)), (wl.square_j1j2(4, 0.45), 3, (0, 0, 0)),
                                      (wl.honeycomb(4, 4), 2, (2, 2, 0))],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_pg_to_momentum_against_oracle(qs3, ctx, lat, K, Kv):
    """A seeded point-group vector carried into the momentum sector: the
    oracle's expansion by the definition (sum over the space group) projected
    on the oracle's momentum basis states."""
    from oracle.pointgroup import expand_pg
    from oracle.translation import expand_to_u1, mk_list
    perms = _ops(lat)
    geo = Geometry(lat.lx, lat.ly, lat.lz, lat.ns)
    L = qs3.Lattice.of(ctx, lat)
    s_k, R_k = mk_list(geo, K, Kv)
    Bk = np.stack([expand_to_u1(geo, K, s_k, R_k, Kv, np.eye(len(s_k))[i]) for i in range(len(s_k))], axis=1)
    msec = qs3.Sector(L, K, Kv)
    assert msec.dim == len(s_k)
    for name, chars in _chars(lat):
        sigma, R = mk_list_pg(geo, perms, chars, K, Kv)
        if not sigma:
            continue
        sec = qs3.PGSector(L, K, Kv, perms, chars)
        phi = np.random.default_rng(17).normal(size=len(sigma))
        psi = sec.to_momentum(torch.from_numpy(phi).cuda(), msec).cpu().numpy()
        want = Bk.conj().T @ expand_pg(geo, perms, chars, K, sigma, R, Kv, phi)
        assert np.abs(psi - want).max() < 1e-12 * max(1.0, np.abs(phi).max()), name
        sec.close()
    msec.close()
    L.close()


def test_pg_ground_state_in_momentum_sector(qs3, ctx):
    """10 x 10 square, N_down = 4, k = 0: the A1 ground state carried into the
    momentum sector is a unit eigenvector of the momentum block with the same
    level, and its magnetisation is uniform."""
    lat = wl.square(10)
    L = qs3.Lattice.of(ctx, lat)
    sec = qs3.PGSector(L, 4, (0, 0, 0), wl.c4v_ops(10), wl.C4V_CHARS["A1"])
    X = torch.zeros(sec.dim, dtype=torch.float64, device="cuda")
    r = sec.eigs(nev=1, evecs=X, seed=4)
    msec = qs3.Sector(L, 4, (0, 0, 0))
    psi = sec.to_momentum(X, msec)
    w = torch.empty_like(psi)
    msec.matvec(psi, w)
    e = r.evals[0]
    assert abs(torch.linalg.vector_norm(psi).item() - 1.0) < 1e-12
    assert torch.linalg.vector_norm(w - e * psi).item() < 1e-7 * abs(e)
    sz = msec.sz(psi)
    assert np.abs(sz - (0.5 - 4 / 100)).max() < 1e-10
    other = qs3.Sector(L, 4, (5, 5, 0))
    with pytest.raises(qs3.QS3Error):
        sec.to_momentum(X, other)
    other.close()
    sec.close()
    msec.close()
    L.close()


def test_pg_oh_cube3_n3_a1g_against_oracle(qs3, ctx):
    """O_h on the 3x3x3 cube at N_down = 3, k = 0, A1g: representatives, norms
    and the lowest levels against the oracle's block."""
    lat = wl.cube(3)
    perms, chars = wl.oh_ops(3), wl.oh_chars()["A1g"]
    geo = Geometry(*lat.dims)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    sigma, R = mk_list_pg(geo, perms, chars, 3, (0, 0, 0))
    L = qs3.Lattice.of(ctx, lat)
    sec = qs3.PGSector(L, 3, (0, 0, 0), perms, chars)
    ranks, norms = sec.basis()
    assert np.array_equal(ranks.astype(np.int64), np.array(sigma, dtype=np.int64) - 1)
    assert np.allclose(norms, np.array(R) ** 2, rtol=1e-13, atol=0)
    ref = np.linalg.eigvalsh(gen_full_ham_pg(geo, perms, chars, 3, bonds, sigma, R, (0, 0, 0)))
    res = sec.eigs(nev=3, seed=5)
    assert np.allclose(res.evals, lowest_distinct(ref, 3), rtol=0, atol=1e-9 * np.abs(ref).max())
    sec.close()
    L.close()


@pytest.mark.parametrize("Kv", [(0, 0, 0), (5, 5, 5)])
def test_pg_oh_cube10(qs3, ctx, Kv):
    """10 x 10 x 10 cube, N_down = 3 (C(1000, 3) = 166,167,000 states): every
    one-dimensional O_h block lies above the momentum block's ground level,
    and the lowest A1g state carried into the momentum sector is an eigenvector
    there with the same level."""
    lat = wl.cube(10)
    L = qs3.Lattice.of(ctx, lat)
    mom = qs3.Sector(L, 3, Kv)
    e0 = mom.eigs(nev=1, seed=1).evals[0]
    for name, chars in wl.oh_chars().items():
        sec = qs3.PGSector(L, 3, Kv, wl.oh_ops(10), chars)
        print(f"pg cube10 K=3 k={Kv} {name}: dim {sec.dim}", flush=True)
        if sec.dim == 0:
            sec.close()
            continue
        X = torch.zeros(sec.dim, dtype=torch.float64, device="cuda")
        r = sec.eigs(nev=1, evecs=X, seed=2)
        assert r.status == qs3.QS3_OK
        assert r.evals[0] >= e0 - 1e-9 * abs(e0)
        if name == "A1g":
            psi = sec.to_momentum(X, mom)
            w = torch.empty_like(psi)
            mom.matvec(psi, w)
            assert abs(torch.linalg.vector_norm(psi).item() - 1.0) < 1e-12
            assert torch.linalg.vector_norm(w - r.evals[0] * psi).item() < 1e-7 * abs(r.evals[0])
        sec.close()
    mom.close()
    L.close()



def test_pg_float32_products(qs3, ctx):
    """Float32 products (float32 row sums, float64 recurrences) against the
    float64 solve, to the 1e-5 relative bound stated for float32 products:
    one exchange constant (packed slots, 10 x 10 square, N_down = 4) and two
    (J1-J2 4 x 4, against the oracle's block)."""
    lat = wl.square(10)
    L = qs3.Lattice.of(ctx, lat)
    for name in ("A1", "B1"):
        sec = qs3.PGSector(L, 4, (0, 0, 0), wl.c4v_ops(10), wl.C4V_CHARS[name])
        e64 = sec.eigs(nev=2, seed=1).evals
        r32 = sec.eigs(nev=2, seed=1, precision=qs3.PREC_F32MV, tol=1e-5)
        assert r32.status == qs3.QS3_OK
        assert np.abs(r32.evals - e64).max() <= 1e-5 * np.abs(e64).max(), (name, r32.evals, e64)
        sec.close()
    L.close()
    lat = wl.square_j1j2(4, 0.45)
    perms, chars = wl.c4v_ops(4), wl.C4V_CHARS["A1"]
    geo = Geometry(*lat.dims)
    sigma, R = mk_list_pg(geo, perms, chars, 4, (0, 0, 0))
    H = gen_full_ham_pg(geo, perms, chars, 4, bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz), sigma, R, (0, 0, 0))
    ref = lowest_distinct(np.linalg.eigvalsh(H), 2)
    L = qs3.Lattice.of(ctx, lat)
    sec = qs3.PGSector(L, 4, (0, 0, 0), perms, chars)
    r32 = sec.eigs(nev=2, seed=1, precision=qs3.PREC_F32MV, tol=1e-5)
    assert r32.status == qs3.QS3_OK
    assert np.abs(r32.evals - ref).max() <= 1e-5 * max(1.0, np.abs(ref).max())
    sec.close()
    L.close()


def test_pg_kagome12_c6v(qs3, ctx):
    """12 x 12 kagome (432 sites), N_down = 3, k = 0: every one-dimensional
    C6v block lies above the momentum block's ground level, and the lowest
    A1 state carried into the momentum sector is an eigenvector there."""
    lat = wl.kagome(12, 12)
    L = qs3.Lattice.of(ctx, lat)
    mom = qs3.Sector(L, 3, (0, 0, 0))
    e0 = mom.eigs(nev=1, seed=1).evals[0]
    for name, chars in wl.C6V_CHARS.items():
        sec = qs3.PGSector(L, 3, (0, 0, 0), wl.kagome_c6v_ops(12), chars)
        print(f"pg kagome12 K=3 {name}: dim {sec.dim}", flush=True)
        if sec.dim == 0:
            sec.close()
            continue
        X = torch.zeros(sec.dim, dtype=torch.float64, device="cuda")
        r = sec.eigs(nev=1, evecs=X, seed=2)
        assert r.status == qs3.QS3_OK
        assert r.evals[0] >= e0 - 1e-9 * abs(e0)
        if name == "A1":
            psi = sec.to_momentum(X, mom)
            w = torch.empty_like(psi)
            mom.matvec(psi, w)
            assert torch.linalg.vector_norm(w - r.evals[0] * psi).item() < 1e-7 * abs(r.evals[0])
        sec.close()
    mom.close()
    L.close()



def test_pg_honeycomb_c6v_against_oracle(qs3, ctx):
    """C6v of the 3x3 honeycomb at N_down = 3, k = 0: every one-dimensional
    sector's representatives, norms, H.v and lowest level against the
    oracle's block."""
    lat = wl.honeycomb(3, 3)
    perms = wl.honeycomb_c6v_ops(3)
    geo = Geometry(3, 3, 1, 2)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    L = qs3.Lattice.of(ctx, lat)
    for name, chars in wl.C6V_CHARS.items():
        sigma, R = mk_list_pg(geo, perms, chars, 3, (0, 0, 0))
        sec = qs3.PGSector(L, 3, (0, 0, 0), perms, chars)
        ranks, norms = sec.basis()
        assert np.array_equal(ranks.astype(np.int64), np.array(sigma, dtype=np.int64) - 1), name
        if not sigma:
            sec.close()
            continue
        assert np.allclose(norms, np.array(R) ** 2, rtol=1e-13, atol=0)
        H = gen_full_ham_pg(geo, perms, chars, 3, bonds, sigma, R, (0, 0, 0))
        vh = np.random.default_rng(3).normal(size=sec.dim)
        w = torch.empty(sec.dim, dtype=torch.float64, device="cuda")
        sec.matvec(torch.from_numpy(vh).cuda(), w)
        assert np.abs(w.cpu().numpy() - H @ vh).max() <= _tol(H, np.abs(vh).max(), 9)
        ref = np.linalg.eigvalsh(H)
        r = sec.eigs(nev=1, seed=2)
        assert abs(r.evals[0] - ref[0]) <= 1e-9 * max(1.0, abs(ref[0])), name
        sec.close()
    L.close()


def test_pg_ground_state_dsf(qs3, ctx):
    """S^-(q, omega) of a point-group ground state carried into the momentum
    sector equals that of the momentum sector's own ground state, on a
    cluster where exactly one one-dimensional block holds the ground level
    and every other block (and the next level) lies clearly above it, so the
    two states differ by a phase only (6 x 6 square, N_down = 2, k = 0)."""
    lat = wl.square(6)
    L = qs3.Lattice.of(ctx, lat)
    mom = qs3.Sector(L, 2, (0, 0, 0))
    Xk = torch.empty(2 * mom.dim, dtype=torch.complex128, device="cuda")
    rk = mom.eigs(nev=2, evecs=Xk, seed=1)
    e0, e1 = rk.evals[0], rk.evals[1]
    gap = e1 - e0
    assert gap > 1e-3 * abs(e0)
    holders = []
    for name, chars in wl.C4V_CHARS.items():
        sec = qs3.PGSector(L, 2, (0, 0, 0), wl.c4v_ops(6), chars)
        if sec.dim == 0:
            sec.close()
            continue
        X = torch.zeros(sec.dim, dtype=torch.float64, device="cuda")
        r = sec.eigs(nev=1, evecs=X, seed=2)
        if abs(r.evals[0] - e0) <= 1e-9 * abs(e0):
            holders.append((name, sec.to_momentum(X, mom)))
        else:
            assert r.evals[0] >= e0 + 0.5 * gap
        sec.close()
    assert len(holders) == 1
    qv = [(1, 0, 0), (2, 3, 0), (3, 3, 0)]
    omega = np.linspace(0.0, 8.0, 200)
    S_pg, _, _, w_pg = mom.dsf(holders[0][1], e0, qv, omega, steps=40, eta=0.1, field=4.0)
    S_k, _, _, w_k = mom.dsf(Xk[:mom.dim].contiguous(), e0, qv, omega, steps=40, eta=0.1, field=4.0)
    assert np.allclose(w_pg, w_k, rtol=1e-8, atol=1e-12)
    assert np.abs(S_pg - S_k).max() <= 1e-6 * np.abs(S_k).max()
    mom.close()
    L.close()
