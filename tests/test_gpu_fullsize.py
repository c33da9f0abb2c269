"""Full-size parity against values the oracle stored in
tests/golden/full_size_levels.json (written by tests/golden/make_goldens.py,
which calls only oracle/: the plain C Alg. 9 or its cached-structure variant,
solved by the oracle's fully reorthogonalised Lanczos and by scipy's eigsh,
which agree to 1e-11; dense diagonalisation and Sec. 3.8-3.9 for S(q, omega)).

The GPU side runs each workload with the library's default solver settings,
in the launch configurations the benchmark times:
  * 10x10 square, N_down = 4, fixed-N_down sector (3,921,225 rows): ground level
  * the same lattice, all 100 momentum sectors in one batch (2 sectors per
    lane), lowest 5 distinct levels; three sectors are stored, among them
    k = (5, 5) whose lowest three levels lie within 2.6e-6 of each other
  * 10^3 cube, N_down = 3, all 1000 momentum sectors in one batch (16 sectors
    per lane): the lowest level of nine stored sectors, among them sectors
    whose lowest two levels are split by ~2e-6 at E ~ 734 (3e-9 relative)
  * 10x10 square S^-(q, omega): ground state over the 100 N_down = 3 momenta,
    S^-_q into N_down = 4 for all 100 q in one batch (2 targets per lane),
    300 levels, eta = 0.05, h = 4: three stored q.
Eigenvalues must agree to 1e-10 relative.  S(q, omega) depends on the
ground-state vector to first order, so the workload converges it to a
residual of 1e-13 x the Ritz spread (about 2e-12; with the gap 0.44 above
the ground level its admixture of other states is ~1e-11).  The Lanczos
coefficients of S^-_q |gs> then agree with the oracle's at the head of the
sequence only: two float64 runs from start vectors 1e-13 apart agree to
~4e-10 in the first 20 coefficients and not at all by level 300 (measured on
the oracle alone), while their continued fractions agree to 9e-7 of the
maximum of S and their integrals over the grid to 1e-11; any two float64
implementations diverge the same way from rounding alone (GPU against the
oracle: 2.7e-6 of the maximum).  The tolerances: weights 1e-9 relative, the
first 3 (2) alpha (beta) 1e-10, S 1e-5 of its maximum, the integral of S
over the grid 1e-7 relative (measured 9.5e-9; |dS| <= 1e-5 max S bounds it
by 5.6e-4).
"""
import json
import os

import numpy as np
import pytest

import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "full_size_levels.json")))
REL = 1e-10


@pytest.fixture(scope="module")
def qs3():
    from paper_2107_00872_amd import qs3 as q
    assert torch.cuda.is_available()
    return q


@pytest.fixture(scope="module")
def ctx(qs3):
    return qs3.Context(0)


def _rel(a, b):
    return abs(a - b) / max(1.0, abs(b))


def test_c2_full_sector_ground_level(qs3, ctx):
    g = GOLD["c2_full"]
    L = qs3.Lattice.of(ctx, wl.square(10))
    sec = qs3.Sector(L, 4)
    assert sec.dim == g["dim"]
    r = sec.eigs(nev=1, seed=1)
    assert r.status == qs3.QS3_OK
    assert _rel(r.evals[0], g["levels"][0]) <= REL, (r.evals[0], g["levels"][0])
    sec.close()


def test_c2_momentum_sectors_lowest_five(qs3, ctx):
    g = GOLD["c2_k"]
    lat = wl.square(10)
    L = qs3.Lattice.of(ctx, lat)
    ks = wl.all_momenta(lat)
    bat = qs3.Batch(L, 4, ks)
    ev, infos, rc = bat.eigs(nev=5, seed=1)
    assert rc == qs3.QS3_OK
    for s in g["sectors"]:
        b = ks.index(tuple(s["k"]))
        assert int(bat.dims[b]) == s["dim"]
        for got, ref in zip(ev[b], s["levels"]):
            assert _rel(got, ref) <= REL, (s["k"], ev[b], s["levels"])
    # the full-sector ground level is the lowest over the momenta
    assert _rel(ev[:, 0].min(), GOLD["c2_full"]["levels"][0]) <= REL
    bat.close()


def test_c3_all_sectors_default_solver(qs3, ctx):
    g = GOLD["c3"]
    lat = wl.cube(10)
    L = qs3.Lattice.of(ctx, lat)
    ks = wl.all_momenta(lat)
    bat = qs3.Batch(L, 3, ks)
    ev, infos, rc = bat.eigs(nev=1, seed=1)
    assert rc == qs3.QS3_OK and all(i.converged for i in infos)
    errs = {}
    for s in g["sectors"]:
        b = ks.index(tuple(s["k"]))
        assert int(bat.dims[b]) == s["dim"]
        errs[tuple(s["k"])] = _rel(ev[b, 0], s["levels"][0])
    assert max(errs.values()) <= REL, errs
    # a second seed settles on the same levels
    ev2, infos2, rc2 = bat.eigs(nev=1, seed=77)
    for s in g["sectors"]:
        b = ks.index(tuple(s["k"]))
        assert _rel(ev2[b, 0], s["levels"][0]) <= REL, (s["k"], ev2[b, 0], s["levels"][0])
    bat.close()


def test_c3_all_sectors_float32_products(qs3, ctx):
    """The 1000-sector solve with float32 products (float64 recurrences; the
    batched H.v in four float32 launches over 250 sectors): rounding v to
    float32 perturbs H.v by at most about eps32 * ||H|| ||v||, so by Weyl's
    inequality every level moves by at most about 6e-8 of the spectrum's
    scale (|E| ~ 730 here, ||H|| <= 750); the stored oracle levels are met
    within 2e-7 relative."""
    g = GOLD["c3"]
    lat = wl.cube(10)
    L = qs3.Lattice.of(ctx, lat)
    ks = wl.all_momenta(lat)
    bat = qs3.Batch(L, 3, ks)
    ev, infos, rc = bat.eigs(nev=1, seed=1, precision=qs3.PREC_F32MV)
    assert rc == qs3.QS3_OK and all(i.converged for i in infos)
    errs = {tuple(s["k"]): _rel(ev[ks.index(tuple(s["k"])), 0], s["levels"][0]) for s in g["sectors"]}
    assert max(errs.values()) <= 2e-7, errs
    bat.close()


def test_c3_single_sectors_default_solver(qs3, ctx):
    """The plain one-sector path (one lane per row) on the stored sectors."""
    g = GOLD["c3"]
    L = qs3.Lattice.of(ctx, wl.cube(10))
    for s in g["sectors"]:
        sec = qs3.Sector(L, 3, tuple(s["k"]))
        r = sec.eigs(nev=1, seed=5)
        assert r.status == qs3.QS3_OK
        assert _rel(r.evals[0], s["levels"][0]) <= REL, (s["k"], r.evals[0], s["levels"][0])
        sec.close()


def test_c4_dsf_against_oracle(qs3, ctx):
    g = GOLD["c4"]
    lat = wl.square(10)
    L = qs3.Lattice.of(ctx, lat)
    ks = wl.all_momenta(lat)
    bat = qs3.Batch(L, 3, ks)
    ev, infos, rc = bat.eigs(nev=1, seed=1)
    assert rc == qs3.QS3_OK
    order = sorted(range(len(ks)), key=lambda b: (round(ev[b, 0], 9), ks[b][0], ks[b][1]))
    k0 = ks[order[0]]
    assert list(k0) == g["k0"]
    bat.close()
    gs = qs3.Sector(L, 3, k0)
    X = torch.empty(gs.dim, dtype=torch.complex128, device="cuda")
    r = gs.eigs(nev=1, evecs=X, seed=1, tol=1e-13)
    assert r.status == qs3.QS3_OK and _rel(r.evals[0], g["E0"]) <= REL
    omega = np.linspace(*g["omega"][:2], int(g["omega"][2]))
    # all 100 q in one call (the launch configuration of the workload)
    S, a, b, w = gs.dsf(X, r.evals[0], ks, omega, steps=g["steps"], eta=g["eta"], field=g["field"])
    assert abs(w.sum() - (lat.n_sites - 3)) <= 1e-9          # sum_q S^{+-}(q) = N - K
    for q in g["q"]:
        qi = ks.index(tuple(q["q"]))
        assert abs(w[qi] - q["weight"]) <= 1e-9 * q["weight"], (q["q"], w[qi], q["weight"])
        # the coefficient sequence amplifies a start-vector difference level
        # by level, so only its head is compared; S(omega), a smooth function
        # of the spectral measure, is compared in full
        assert np.abs(a[qi, :3] - np.array(q["alpha"][:3])).max() <= 1e-10
        assert np.abs(b[qi, :2] - np.array(q["beta"][:2])).max() <= 1e-10
        Sref = np.array(q["S"])
        assert np.abs(S[qi] - Sref).max() <= 1e-5 * Sref.max(), (q["q"], np.abs(S[qi] - Sref).max())
        I, Iref = np.trapezoid(S[qi], omega), np.trapezoid(Sref, omega)
        assert abs(I - Iref) <= 1e-7 * abs(Iref), (q["q"], I, Iref)
    gs.close()
