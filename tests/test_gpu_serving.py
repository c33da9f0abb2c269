"""Serving (continuous batching of solve requests): results against the oracle,
the same result alone and in a mix (bit for bit: a request's kernels and their
order do not depend on the other requests), admission by device footprint,
and cancellation."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle.hamiltonian import bonds_1based, gen_full_ham
from oracle.lanczos import lowest_distinct
from oracle.translation import Geometry, gen_full_ham_sym_adapt, mk_list

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qs3():
    from paper_2107_00872_amd import qs3 as q
    return q


@pytest.fixture(scope="module")
def ctx(qs3):
    return qs3.Context(0)


def dense_levels(lat, K, k, n):
    bonds = bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz)
    if k is None:
        return lowest_distinct(np.linalg.eigvalsh(gen_full_ham(lat.n_sites, K, bonds)), n)
    geo = Geometry(*lat.dims)
    s, R = mk_list(geo, K, k)
    return lowest_distinct(np.linalg.eigvalsh(gen_full_ham_sym_adapt(geo, K, bonds, s, R, k)), n)


REQS = [(wl.with_disorder(wl.chain(12), 1), 3, None), (wl.with_disorder(wl.square(4), 2, per_bond=False), 2, (1, 0, 0)),
        (wl.with_disorder(wl.chain(16), 3, per_bond=False), 1, (3, 0, 0)), (wl.with_disorder(wl.cube(3), 4), 2, None),
        (wl.with_disorder(wl.square(4), 5), 4, None), (wl.with_disorder(wl.chain(10), 6, per_bond=False), 3, (0, 0, 0))]


def test_served_results_match_dense(qs3, ctx):
    srv = qs3.Server(ctx, max_active=4)
    tickets = [srv.submit(lat, K, k, nev=3, seed=11) for (lat, K, k) in REQS]
    for t, (lat, K, k) in zip(tickets, REQS):
        r = srv.wait(t)
        assert r.status == 0, r.status
        ref = dense_levels(lat, K, k, 3)
        got = np.array(r.evals[:r.n_found])
        assert r.n_found == len(ref)
        assert np.allclose(got, ref, rtol=1e-10, atol=1e-12)
        assert r.t_submit <= r.t_start <= r.t_done
    srv.close()


def test_alone_equals_mixed_bitwise(qs3, ctx):
    probe = (wl.with_disorder(wl.square(6), 21, per_bond=False), 3, (2, 1, 0))
    srv = qs3.Server(ctx, max_active=1)
    alone = srv.wait(srv.submit(*probe, nev=3, seed=5))
    srv.close()
    srv = qs3.Server(ctx, max_active=6)
    others = [srv.submit(lat, K, k, nev=3, seed=2) for (lat, K, k) in REQS]
    t = srv.submit(*probe, nev=3, seed=5)
    others += [srv.submit(lat, K, k, nev=2, seed=3) for (lat, K, k) in REQS[:3]]
    mixed = srv.wait(t)
    for o in others:
        srv.wait(o)
    srv.close()
    assert alone.status == 0 and mixed.status == 0
    assert list(alone.evals[:alone.n_found]) == list(mixed.evals[:mixed.n_found])   # bit-identical
    assert alone.n_matvec == mixed.n_matvec


def test_admission_rejects_oversize_and_cancel(qs3, ctx):
    srv = qs3.Server(ctx, max_active=2)
    big = wl.cube(10)
    t_big = srv.submit(big, 4, None, nev=1)   # C(1000, 4) = 4.1e10 rows: ~9 TB of Krylov vectors
    r = srv.wait(t_big)
    assert r.status == qs3.QS3_ENOMEM
    assert r.footprint_bytes > 1e12
    # cancel a queued request behind a running one
    t1 = srv.submit(wl.square(10), 4, None, nev=1, seed=1)
    t2 = srv.submit(wl.square(10), 4, None, nev=1, seed=2)
    t3 = srv.submit(wl.square(10), 4, None, nev=1, seed=3)
    srv.cancel(t3)
    r3 = srv.wait(t3)
    assert r3.status in (qs3.QS3_ECANCELED, 0)
    assert srv.wait(t1).status == 0 and srv.wait(t2).status == 0
    with pytest.raises(qs3.QS3Error):
        srv.poll(999999)
    srv.close()


def test_tight_budget_large_momentum_requests(qs3):
    """Several large momentum requests (10^3 cube, N_down = 3: a 1.3 GB rank
    table and per-representative hop lists each) under a context budget that
    holds two of them: the footprint used for admission covers every store
    the structure build makes, so no request fails for memory -- all finish
    with QS3_OK, at most two at a time, with the levels of an unconstrained
    run."""
    lat = wl.cube(10)
    ks = [(0, 0, 0), (1, 0, 0), (3, 6, 0), (5, 5, 5), (2, 7, 1)]
    probe_ctx = qs3.Context(0)
    srv = qs3.Server(probe_ctx, max_active=1)
    ref = {}
    for k in ks:
        r = srv.wait(srv.submit(lat, 3, k, nev=1, seed=4))
        assert r.status == 0
        ref[k] = (r.evals[0], r.footprint_bytes)
    srv.close()
    probe_ctx.close()
    F = max(f for _, f in ref.values())
    tight = qs3.Context(0, budget_bytes=int(2.3 * F))
    srv = qs3.Server(tight, max_active=4)
    tickets = [srv.submit(lat, 3, k, nev=1, seed=4) for k in ks]
    res = [srv.wait(t) for t in tickets]
    srv.close()
    for k, r in zip(ks, res):
        assert r.status == 0, (k, r.status, qs3.lib().qs3_last_error())
        assert abs(r.evals[0] - ref[k][0]) <= 1e-12 * abs(ref[k][0])
    # never more than two running at once
    ev = sorted([(r.t_start, 1) for r in res] + [(r.t_done, -1) for r in res])
    run = peak = 0
    for _, d in ev:
        run += d
        peak = max(peak, run)
    assert peak <= 2
    tight.close()
