"""Full diagonalisation (Sec. 3.4) and thermal averages (Eq. (ens)) on the GPU
against the oracle: dense blocks element by element, all eigenvalues,
eigenvector residuals, and thermal averages from every sector's spectrum.

Tolerances: dense elements are single products of couplings and phases
(1e-14 absolute for J ~ 1); eigenvalues 1e-10 relative (float64 divide and
conquer); thermal averages 1e-10 relative."""
import numpy as np
import pytest

import workloads as wl
from oracle import native as orc
from oracle.hamiltonian import bonds_1based, gen_full_ham
from oracle.thermal import thermal as orc_thermal
from oracle.translation import Geometry, gen_full_ham_sym_adapt, mk_list

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


@pytest.mark.parametrize("lat,K", [(wl.chain(10), 3), (wl.with_disorder(wl.square(4), 7), 3),
                                   (wl.random_bonds(12, 30, seed=4), 5), (wl.cube(3), 2), (wl.chain(9), 0)],
                         ids=lambda x: getattr(x, "name", str(x)))
def test_dense_and_full_diag_u1(qs3, ctx, lat, K):
    L = qs3.Lattice.of(ctx, lat)
    sec = qs3.Sector(L, K)
    ref = gen_full_ham(lat.n_sites, K, bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz))
    H = sec.dense().cpu().numpy().T          # column major on the device
    assert np.abs(H - ref).max() < 1e-14 * max(1.0, np.abs(ref).max())
    V = torch.empty(sec.dim, sec.dim, dtype=torch.float64, device="cuda")
    ev = sec.full_diag(evecs=V)
    er = np.linalg.eigvalsh(ref)
    assert np.abs(ev - er).max() < 1e-10 * max(1.0, np.abs(er).max())
    Vh = V.cpu().numpy().T                   # columns = eigenvectors
    assert np.abs(ref @ Vh - Vh * ev).max() < 1e-9 * max(1.0, np.abs(er).max())
    sec.close()


def _k_cases():
    return [(wl.square(4), 3), (wl.hypercubic(4, 2, 1), 3), (wl.chain(12), 6), (wl.cube(3), 2)]


@pytest.mark.parametrize("mode", ["table", "fly"])
@pytest.mark.parametrize("lat,K", _k_cases(), ids=lambda x: getattr(x, "name", str(x)))
def test_dense_and_full_diag_k(qs3, lat, K, mode):
    c = qs3.Context(0)
    if mode == "fly":
        c.set_structure_limits(0, 0)
    L = qs3.Lattice.of(c, lat)
    geo = Geometry(*lat.dims)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    for Kv in wl.all_momenta(lat)[:5]:
        s, R = mk_list(geo, K, Kv)
        if not s:
            continue
        sec = qs3.Sector(L, K, Kv)
        ref = gen_full_ham_sym_adapt(geo, K, bonds, s, R, Kv)
        H = sec.dense().cpu().numpy().T
        assert np.abs(H - ref).max() < 1e-13
        V = torch.empty(sec.dim, sec.dim, dtype=torch.complex128, device="cuda")
        ev = sec.full_diag(evecs=V)
        er = np.linalg.eigvalsh(ref)
        assert np.abs(ev - er).max() < 1e-10 * max(1.0, np.abs(er).max())
        Vh = V.cpu().numpy().T
        assert np.abs(ref @ Vh - Vh * ev).max() < 1e-9 * max(1.0, np.abs(er).max())
        sec.close()
    L.close()
    c.close()


def test_thermal_from_all_sectors(qs3, ctx):
    """Periodic chain of 10: every (N_down, k) sector with N_down <= 5 fully
    diagonalised on the GPU, and N_down > 5 from N - N_down (the XXZ model is
    invariant under flipping every spin), give 2^10 levels; thermal averages at
    several temperatures and fields equal the oracle's from its own dense
    momentum blocks of every N_down."""
    lat = wl.chain(10)
    N = lat.n_sites
    L = qs3.Lattice.of(ctx, lat)
    geo = Geometry(*lat.dims)
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    E, Sz, Eo, Szo = [], [], [], []
    for K in range(N + 1):
        for Kv in wl.all_momenta(lat):
            Kg = min(K, N - K)
            if mk_list(geo, Kg, Kv)[0]:
                sec = qs3.Sector(L, Kg, Kv)
                ev = sec.full_diag()
                sec.close()
                E += list(ev)
                Sz += [N / 2 - K] * len(ev)
            s, R = mk_list(geo, K, Kv)
            if not s:
                continue
            er = np.linalg.eigvalsh(gen_full_ham_sym_adapt(geo, K, bonds, s, R, Kv))
            Eo += list(er)
            Szo += [N / 2 - K] * len(er)
    assert len(E) == 1 << N
    beta = np.array([0.0, 0.1, 1.0, 5.0, 20.0])
    for h in (0.0, 1.3):
        got = qs3.thermal(E, Sz, beta, h)
        ref = orc_thermal(np.array(Eo), np.array(Szo), beta, h)
        for key in ("lnZ", "energy", "heat", "mag", "chi"):
            assert np.allclose(got[key], ref[key], rtol=1e-10, atol=1e-10), key
