"""Execution schedules that must not change results: thick-restart cycles
replayed from captured HIP graphs, and autotuned schedules of the batched
momentum H.v (lanes per row, blocks per CU).  Every combination gives the
same eigenvalues bit for bit, and graphs are replayed several times within
a solve with the solver's own host work between the replays."""
import numpy as np
import pytest

import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qs3():
    from paper_2107_00872_amd import qs3 as q
    assert torch.cuda.is_available()
    return q


def _ctx(qs3, graphs, tune):
    c = qs3.Context(0)
    c.set_schedule(graphs, tune)
    return c


def test_graph_replay_equals_eager_fixed_n_down(qs3):
    st = torch.cuda.Stream()
    out = {}
    for graphs in (False, True):
        ctx = _ctx(qs3, graphs, True)
        sec = qs3.Sector(qs3.Lattice.of(ctx, wl.square(10)), 3)
        runs = []
        for seed in (1, 2, 3):
            r = sec.eigs(nev=2, seed=seed, stream=st)
            assert r.status == qs3.QS3_OK
            runs.append((r.evals.tolist(), r.info.n_matvec, r.info.graph_cycles))
            # eager work on the same stream between solves
            v = torch.empty(sec.dim, dtype=torch.float64, device="cuda")
            sec.start_vector(seed, v, stream=st)
        out[graphs] = runs
        sec.close()
        ctx.close()
    for (e0, m0, g0), (e1, m1, g1) in zip(out[False], out[True]):
        assert e0 == e1 and m0 == m1
        assert g0 == 0 and g1 > 0


def test_graphs_and_autotune_equal_plain_batch(qs3):
    """The 10x10 N_down = 4 batch of 100 sectors (lowest 5 levels) and the
    10^3 N_down = 2 batch of 1000 sectors under all four combinations."""
    st = torch.cuda.Stream()
    for lat, K, nev in [(wl.square(10), 4, 5), (wl.cube(10), 2, 1)]:
        ks = wl.all_momenta(lat)
        res = {}
        for graphs in (False, True):
            for tune in (False, True):
                ctx = _ctx(qs3, graphs, tune)
                bat = qs3.Batch(qs3.Lattice.of(ctx, lat), K, ks)
                ev, infos, rc = bat.eigs(nev=nev, seed=3, stream=st)
                assert rc == qs3.QS3_OK
                res[(graphs, tune)] = (ev.copy(), [i.n_matvec for i in infos],
                                       sum(i.graph_cycles for i in infos))
                bat.close()
                ctx.close()
        base = res[(False, False)]
        for key, (ev, mv, gc) in res.items():
            assert np.array_equal(ev, base[0], equal_nan=True), key
            assert mv == base[1], key
            assert (gc > 0) == key[0], key


def test_autotuned_matvec_equals_default(qs3):
    """Single batched products: tuned schedules against the default rule,
    bit for bit, for batches whose width classes differ."""
    st = torch.cuda.Stream()
    for lat, K in [(wl.square(10), 3), (wl.cube(10), 2), (wl.square(12), 2)]:
        ks = wl.all_momenta(lat)
        outs = []
        for tune in (False, True):
            ctx = _ctx(qs3, True, tune)
            L = qs3.Lattice.of(ctx, lat)
            for B in (len(ks), 3, 37):
                bat = qs3.Batch(L, K, ks[:B])
                g = torch.Generator().manual_seed(B)
                v = torch.complex(torch.rand(bat.rows, bat.B, generator=g, dtype=torch.float64),
                                  torch.rand(bat.rows, bat.B, generator=g, dtype=torch.float64)).cuda()
                w = torch.empty_like(v)
                for _ in range(2):                  # the first product may tune
                    bat.matvec(v, w, stream=st)
                st.synchronize()
                outs.append(w.cpu())
                bat.close()
            ctx.close()
        n = len(outs) // 2
        for a, b in zip(outs[:n], outs[n:]):
            assert torch.equal(a, b)
