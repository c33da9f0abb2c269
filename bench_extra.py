"""The other workloads of bench.py (python bench.py --workload c1|c2|c4|c5|...).

c1  periodic chain N=16, N_down=3 (dim 560): 100-step float64 Lanczos, lowest 4
    distinct levels; solve latency p50/p99 over repeated solves.
c2  periodic 10x10 square, N_down=4: full-sector ground state, all 100 momentum
    sectors (lowest 5 levels, batched), <S_i.S_j> and S(q) of the ground state.
c4  periodic 10x10 square, N_down=3 ground state (lowest over the 100 sectors),
    S^-(q, omega) for all 100 q into N_down=4: 300 continued-fraction Lanczos
    levels, eta=0.05, 2000 omega points in [0, 8], field h = 4 (the saturation
    field of the square lattice); float64 and float32-matvec.
pg  periodic 10x10 square, N_down = 5 and 6, k = 0: the four one-dimensional
    C4v sectors (translations x point operations) against the momentum sector
    holding the same ground state: block build, ELL H.v rate and bytes, solve
    times; and at N_down = 4 the 10^3 cube's O_h A1g sector and the 12 x 12
    kagome lattice's C6v A1 sector against their momentum sectors.
c5  serving: Poisson arrivals of random solve requests (workloads.serving_stream),
    rate 0.8 / (mean one-at-a-time service time); p50/p99 latency and solves/s
    against the same requests run one at a time.
"""
from __future__ import annotations

import hashlib
import math
import os
import re
import sys
import time

import numpy as np
import torch

import workloads as wl
from paper_2107_00872_amd import qs3

ROOT = os.path.dirname(os.path.abspath(__file__))


def _ctx():
    torch.cuda.set_device(0)
    return qs3.Context(0)


def _pct(x, p):
    return float(np.percentile(np.asarray(x), p))


def c1(args):
    ctx = _ctx()
    lat = wl.chain(16)
    sec = qs3.Sector(qs3.Lattice.of(ctx, lat), 3)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        sec.eigs(nev=4, alg=qs3.ALG_LANCZOS, steps=100, seed=1, stream=stream)
    lat_s = []
    reps = max(20, args.steps * 20)
    for r in range(reps):
        t0 = time.perf_counter()
        res = sec.eigs(nev=4, alg=qs3.ALG_LANCZOS, steps=100, seed=1 + r, stream=stream)
        lat_s.append(time.perf_counter() - t0)
    out = {"metric": "Lanczos solve latency (100 steps, lowest 4 distinct levels)", "workload": "c1",
           "value": _pct(lat_s, 50) * 1e3, "unit": "ms p50", "p99_ms": _pct(lat_s, 99) * 1e3,
           "rows_per_s": 100 * sec.dim / _pct(lat_s, 50), "evals": [float(x) for x in res.evals],
           "dim": sec.dim, "note": "latency bound (d = 560)"}
    try:
        from oracle import native as orc
        from oracle.lanczos import lanczos, ritz, lowest_distinct
        from oracle.rng import start_vector
        orc.build(force=False)
        B = orc.Bonds.of(lat)
        v0 = start_vector(1, np.arange(sec.dim), complex_=False)
        t0 = time.perf_counter()
        a, b, _ = lanczos(lambda x: orc.hv_u1(16, 3, B, x, nthreads=1), v0, 100)
        e, res_, _ = ritz(a, b)
        out["cpu_baseline"] = {"value": (time.perf_counter() - t0) * 1e3, "unit": "ms per solve",
                               "cores": 1, "kind": "oracle", "sample": "one 100-step solve"}
    except Exception as exc:  # the CPU leg is informative only
        out["cpu_baseline_error"] = str(exc)
    return out


def _cells_run(lat, K):
    """All momenta of a lattice with several sites per cell in one batch:
    batched H.v rate, batched float64 ground states, a sample one sector at a
    time, and the cross-check min_k E_0(k) = E_0 of the fixed-N_down sector."""
    ctx = _ctx()
    L = qs3.Lattice.of(ctx, lat)
    ks = wl.all_momenta(lat)
    NT = lat.lx * lat.ly * lat.lz
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    bat = qs3.Batch(L, K, ks)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    v = torch.zeros(bat.rows, bat.B, dtype=torch.complex128, device="cuda")
    v.real.uniform_(-1, 1)
    w = torch.empty_like(v)
    bat.matvec(v, w, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(10):
        bat.matvec(v, w, stream=stream)
    e1.record(stream)
    e1.synchronize()
    t_mv = e0.elapsed_time(e1) / 10e3
    # off-diagonal entries per row: the mean over the sector's states,
    # N_b 2K(N-K) / (N(N-1)); per row and sector 16 B for each gathered
    # entry, the row's own v and its w
    N = lat.n_sites
    nhops_row = lat.n_bonds * 2 * K * (N - K) / (N * (N - 1))
    alg_bytes = 16.0 * (2 + nhops_row) * bat.rows * bat.B
    del v, w
    torch.cuda.empty_cache()
    out = {"metric": f"batched E(k), {lat.name} N_down={K}, {len(ks)} momenta", "workload": "cells",
           "sites": lat.n_sites, "rows": bat.rows, "sectors": bat.B, "setup_s": t_setup,
           "matvec_ms": t_mv * 1e3, "matvec_sector_rows_per_s": bat.rows * bat.B / t_mv,
           "matvec_alg_GBs": alg_bytes / t_mv / 1e9, "hops_per_row": nhops_row}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    print(f"{lat.name}: {bat.rows} rows x {bat.B} sectors, set-up {t_setup:.2f}s, H.v {t_mv * 1e3:.2f} ms",
          file=sys.stderr, flush=True)
    ev, infos, rc = bat.eigs(nev=1, seed=1, stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"{lat.name}: batched solve {dt:.2f}s", file=sys.stderr, flush=True)
    mv = np.array([i.n_matvec for i in infos])
    out["f64"] = {"seconds": dt, "solves_per_s": bat.B / dt, "matvecs_max": int(mv.max()),
                  "matvecs_p50": float(np.median(mv)), "converged": int(sum(i.converged for i in infos)),
                  "rc": rc, "E_min": float(ev[:, 0].min())}
    sample = sorted(np.random.default_rng(7).choice(len(ks), 10, replace=False).tolist())
    secs = [qs3.Sector(L, K, ks[b]) for b in sample]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev_s = [secs[i].eigs(nev=1, seed=1 + b, stream=stream) for i, b in enumerate(sample)]
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t0
    for sc in secs:
        sc.close()
    e_s = np.array([r.evals[0] for r in ev_s])
    out["f64_one_at_a_time"] = {"seconds": t_s, "solves_per_s": len(sample) / t_s,
                                "max_rel_diff_vs_batched": float(np.max(np.abs(e_s - ev[sample, 0]) / np.abs(e_s)))}
    full = qs3.Sector(L, K)
    r = full.eigs(nev=1, seed=1, stream=stream)
    out["E0_fixed_N_down"] = float(r.evals[0])
    out["min_k_E0_minus_E0"] = float(ev[:, 0].min() - r.evals[0])
    out["value"] = out["f64"]["solves_per_s"]
    out["unit"] = "sector solves/s (float64)"
    full.close()
    bat.close()
    L.close()
    ctx.close()
    return out


def cells(args):
    """Several sites per unit cell: the 12 x 12 kagome lattice (432 sites,
    4 neighbours, 144 momenta, about 92k representatives each) and the
    6 x 6 x 6 pyrochlore lattice (864 sites, 6 neighbours, 216 momenta, about
    496k representatives each), J = Delta = 1, N_down = 3."""
    which = getattr(args, "cells", "both")
    if which == "pyrochlore":
        return _cells_run(wl.pyrochlore(6), 3)
    out = _cells_run(wl.kagome(12, 12), 3)
    if which == "both":
        torch.cuda.empty_cache()
        out["pyrochlore"] = _cells_run(wl.pyrochlore(6), 3)
    return out


def c4(args):
    ctx = _ctx()
    lat = wl.square(10)
    L = qs3.Lattice.of(ctx, lat)
    ks = wl.all_momenta(lat)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    bat = qs3.Batch(L, 3, ks)
    ev, infos, rc = bat.eigs(nev=1, seed=1, stream=stream)
    order = sorted(range(len(ks)), key=lambda b: (round(ev[b, 0], 9), ks[b][0], ks[b][1]))
    k0 = ks[order[0]]
    gs = qs3.Sector(L, 3, k0)
    X = torch.empty(gs.dim, dtype=torch.complex128, device="cuda")
    # S depends on the ground-state vector to first order: converge it to a
    # residual of 1e-13 x the Ritz spread
    r = gs.eigs(nev=1, evecs=X, seed=1, tol=1e-13, stream=stream)
    torch.cuda.synchronize()
    t_gs = time.perf_counter() - t0
    omega = np.linspace(0.0, 8.0, 2000)
    out = {"metric": "S^-(q, omega) for all 100 q", "workload": "c4", "k0": list(k0), "E0": float(r.evals[0]),
           "degenerate_k": int(sum(abs(ev[b, 0] - r.evals[0]) < 1e-10 for b in range(len(ks)))),
           "gs_seconds": t_gs}
    S = {}
    for prec, ro, name in [(qs3.PREC_F64, qs3.REORTH_FULL, "f64"), (qs3.PREC_F32MV, qs3.REORTH_FULL, "f32mv"),
                           (qs3.PREC_F64, qs3.REORTH_PARTIAL, "f64_partial"),
                           (qs3.PREC_F32MV, qs3.REORTH_PARTIAL, "f32mv_partial")]:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Sq, a, b, w = gs.dsf(X, r.evals[0], ks, omega, steps=300, eta=0.05, field=4.0, precision=prec,
                             reorth=ro, stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        S[name] = (Sq, a, b)
        out[name] = {"seconds": dt, "q_per_s": len(ks) / dt, "sum_weights": float(w.sum()),
                     "integral_check": float(np.trapezoid(Sq, omega, axis=1).sum())}
    ref, ra, rb = S["f64"]
    out["max_S"] = float(np.abs(ref).max())
    for name in ("f32mv", "f64_partial", "f32mv_partial"):
        Sq, a, b = S[name]
        out[name]["max_abs_dS_vs_f64"] = float(np.abs(Sq - ref).max())
    for name in ("f64_partial",):
        Sq, a, b = S[name]
        out[name]["max_abs_dalpha_vs_full"] = float(np.abs(a - ra).max())
        out[name]["max_abs_dbeta_vs_full"] = float(np.abs(b - rb).max())
    out["value"] = out["f64"]["q_per_s"]
    out["unit"] = "q/s (300-level continued fraction, float64)"
    return out


def szq(args):
    """Longitudinal and raising structure factors of the 10x10 square at
    N_down = 2 (the paper's Sec. 4.2 demonstration): ground state over the 100
    momenta, then S^z(q, omega) with the trivial q = 0 part subtracted and
    S^+(q, omega) for all 100 q (300 levels, eta = 0.05, omega in [-2, 8])."""
    ctx = _ctx()
    lat = wl.square(10)
    L = qs3.Lattice.of(ctx, lat)
    ks = wl.all_momenta(lat)
    stream = torch.cuda.current_stream()
    K = 2
    t0 = time.perf_counter()
    bat = qs3.Batch(L, K, ks)
    ev, infos, rc = bat.eigs(nev=1, seed=1, stream=stream)
    order = sorted(range(len(ks)), key=lambda b: (round(ev[b, 0], 9), ks[b][0], ks[b][1]))
    k0 = ks[order[0]]
    gs = qs3.Sector(L, K, k0)
    X = torch.empty(gs.dim, dtype=torch.complex128, device="cuda")
    r = gs.eigs(nev=1, evecs=X, seed=1, tol=1e-13, stream=stream)
    torch.cuda.synchronize()
    t_gs = time.perf_counter() - t0
    omega = np.linspace(-2.0, 8.0, 2000)
    N = lat.n_sites
    M = N / 2 - K
    out = {"metric": "S^z(q, omega) and S^+(q, omega) for all 100 q", "workload": "szq", "k0": list(k0),
           "E0": float(r.evals[0]), "gs_seconds": t_gs}
    for op, name in [(qs3.OP_SZ, "sz"), (qs3.OP_SPLUS, "sp")]:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Sq, a, b, w = gs.dsf(X, r.evals[0], ks, omega, steps=300, eta=0.05, field=0.0, op=op,
                             subtract_trivial=(op == qs3.OP_SZ), stream=stream)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"seconds": dt, "q_per_s": len(ks) / dt, "sum_weights": float(w.sum()),
                     "static_q0": float(w[ks.index((0, 0, 0))]), "max_S": float(np.abs(Sq).max())}
    out["sz"]["sum_rule"] = N / 4
    out["sz"]["trivial_weight"] = M * M / N
    out["sp"]["sum_rule"] = K
    out["value"] = out["sz"]["q_per_s"]
    out["unit"] = "q/s (300-level continued fraction, float64)"
    return out


def thermal(args):
    """Full diagonalisation near saturation (Sec. 3.4): every momentum sector of
    the periodic 10x10 square with N_down <= 3 (dims 1, 1, 50/49, 1617 per k),
    then Z, energy, specific heat and magnetisation (Eq. (ens)) over a
    temperature grid at the saturation field h = 4 and just below it."""
    ctx = _ctx()
    lat = wl.square(10)
    L = qs3.Lattice.of(ctx, lat)
    ks = wl.all_momenta(lat)
    N = lat.n_sites
    E, Sz = [], []
    t0 = time.perf_counter()
    nsec, tmax = 0, 0.0
    for K in range(4):
        for k in ks:
            sec = qs3.Sector(L, K, k)
            if sec.dim:
                ts = time.perf_counter()
                ev = sec.full_diag()
                tmax = max(tmax, time.perf_counter() - ts)
                E += list(ev)
                Sz += [N / 2 - K] * len(ev)
                nsec += 1
            sec.close()
    t_diag = time.perf_counter() - t0
    T = np.linspace(0.05, 2.0, 40)
    out = {"metric": "full diagonalisation of all sectors with N_down <= 3 + thermal averages", "workload": "thermal",
           "sectors": nsec, "levels": len(E), "seconds": t_diag, "max_sector_s": tmax,
           "value": nsec / t_diag, "unit": "sectors/s (full diagonalisation, float64)"}
    for h in (3.5, 4.0):
        t = qs3.thermal(E, Sz, 1.0 / T, h)
        out[f"h{h}"] = {"T": T[::8].tolist(), "mag_per_site": (t["mag"][::8] / N).tolist(),
                        "heat_per_site": (t["heat"][::8] / N).tolist()}
    # the oracle's dense eigensolver on one N_down = 3 sector (host), for scale
    try:
        from oracle.translation import Geometry, gen_full_ham_sym_adapt, mk_list
        from oracle.hamiltonian import bonds_1based
        geo = Geometry(*lat.dims)
        s_, R_ = mk_list(geo, 3, (1, 0, 0))
        Hk = gen_full_ham_sym_adapt(geo, 3, bonds_1based(lat.bi, lat.bj, lat.jxy, lat.jz), s_, R_, (1, 0, 0))
        tc = time.perf_counter()
        np.linalg.eigvalsh(Hk)
        out["cpu_baseline"] = {"value": time.perf_counter() - tc, "unit": "s per N_down = 3 sector (eigenvalues)",
                               "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
                               "kind": "oracle", "sample": "numpy eigvalsh of the oracle's dense k = (1,0) block"}
    except Exception as exc:
        out["cpu_baseline_error"] = str(exc)
    return out


def c5(args):
    import sys
    ctx = _ctx()
    n = int(getattr(args, "requests", 0) or 200)
    probe = wl.serving_stream(n, seed=7, rate=1.0)
    # one-at-a-time service times (FP64, same requests)
    srv = qs3.Server(ctx, max_active=1)
    service, results_alone = [], {}
    for q in probe:
        t0 = time.perf_counter()
        r = srv.wait(srv.submit(q["lattice"], q["n_down"], q["K"], nev=3, seed=1 + q["id"]))
        service.append(time.perf_counter() - t0)
        results_alone[q["id"]] = (r.status, list(r.evals[:r.n_found]))
        print(f"alone {q['id']} {q['lattice'].name} K={q['n_down']} k={q['K']} dim={r.dim} "
              f"status={r.status} {service[-1]:.3f}s", file=sys.stderr, flush=True)
    srv.close()
    ok_service = [s for s, q in zip(service, probe) if results_alone[q["id"]][0] == 0]
    mean_s = float(np.mean(ok_service))
    rate = 0.8 / mean_s
    stream = wl.serving_stream(n, seed=7, rate=rate)
    # serial FIFO queue with the measured service times = one-at-a-time latencies
    t_free, lat_serial = 0.0, []
    for q, s in zip(stream, service):
        start = max(t_free, q["t_arrive"])
        t_free = start + s
        lat_serial.append(t_free - q["t_arrive"])
    serial_makespan = t_free
    # served with continuous batching
    srv = qs3.Server(ctx, max_active=8)
    t_base = time.perf_counter()
    tickets = []
    for q in stream:
        while time.perf_counter() - t_base < q["t_arrive"]:
            time.sleep(0.0005)
        tickets.append(srv.submit(q["lattice"], q["n_down"], q["K"], nev=3, seed=1 + q["id"]))
    res = []
    for t in tickets:
        res.append(srv.wait(t))
        print(f"served {len(res)}/{n} status={res[-1].status}", file=sys.stderr, flush=True)
    makespan = time.perf_counter() - t_base
    srv.close()
    lat_served = [r.t_done - r.t_submit for r in res]
    same = sum(1 for q, r in zip(stream, res)
               if r.status == results_alone[q["id"]][0] and list(r.evals[:r.n_found]) == results_alone[q["id"]][1])
    statuses = {}
    for r in res:
        statuses[str(r.status)] = statuses.get(str(r.status), 0) + 1
    # per lattice family (chain / square / cube)
    classes = {}
    for fam in ("chain", "square", "cube"):
        idx = [i for i, q in enumerate(stream) if q["lattice"].name.startswith(fam)]
        if idx:
            classes[fam] = {"requests": len(idx),
                            "p50_ms": _pct([lat_served[i] for i in idx], 50) * 1e3,
                            "p99_ms": _pct([lat_served[i] for i in idx], 99) * 1e3,
                            "serial_p50_ms": _pct([lat_serial[i] for i in idx], 50) * 1e3,
                            "serial_p99_ms": _pct([lat_serial[i] for i in idx], 99) * 1e3}
    # burst: every request at t = 0 (throughput bound), against the sum of
    # the one-at-a-time service times
    srv = qs3.Server(ctx, max_active=8)
    t_base = time.perf_counter()
    tickets = [srv.submit(q["lattice"], q["n_down"], q["K"], nev=3, seed=1 + q["id"]) for q in stream]
    res_b = []
    for t in tickets:
        res_b.append(srv.wait(t))
    makespan_b = time.perf_counter() - t_base
    srv.close()
    print(f"burst {makespan_b:.3f}s", file=sys.stderr, flush=True)
    same_b = sum(1 for q, r in zip(stream, res_b)
                 if r.status == results_alone[q["id"]][0] and list(r.evals[:r.n_found]) == results_alone[q["id"]][1])
    return {"metric": "served solves/s and latency vs one-at-a-time FP64", "workload": "c5",
            "value": n / makespan, "unit": "solves/s",
            "requests": n, "rate_per_s": rate, "mean_service_s": mean_s,
            "p50_ms": _pct(lat_served, 50) * 1e3, "p99_ms": _pct(lat_served, 99) * 1e3,
            "serial_p50_ms": _pct(lat_serial, 50) * 1e3, "serial_p99_ms": _pct(lat_serial, 99) * 1e3,
            "serial_solves_per_s": n / serial_makespan, "per_family": classes, "status_counts": statuses,
            "identical_to_alone": same,
            "burst": {"solves_per_s": n / makespan_b, "serial_solves_per_s": n / float(np.sum(service)),
                      "p50_ms": _pct([r.t_done - r.t_submit for r in res_b], 50) * 1e3,
                      "p99_ms": _pct([r.t_done - r.t_submit for r in res_b], 99) * 1e3,
                      "identical_to_alone": same_b}}


def _pg_vs_momentum(ctx, lat, ops, chars, name, stream, K=4):
    """Build and ground state of one point-group sector against the momentum
    sector k = 0 of the same lattice and N_down."""
    Lc = qs3.Lattice.of(ctx, lat)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sec = qs3.PGSector(Lc, K, (0, 0, 0), ops, chars)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    t0 = time.perf_counter()
    ra = sec.eigs(nev=1, seed=1, stream=stream)
    torch.cuda.synchronize()
    t_a = time.perf_counter() - t0
    mom = qs3.Sector(Lc, K, (0, 0, 0))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rm = mom.eigs(nev=1, seed=1, stream=stream)
    torch.cuda.synchronize()
    t_m = time.perf_counter() - t0
    print(f"pg {lat.name} N_down={K} {name} dim {sec.dim} solve {t_a:.3f}s, momentum {mom.dim} {t_m:.3f}s",
          file=sys.stderr, flush=True)
    out = {name: {"dim": sec.dim, "build_s": t_b, "solve_s": t_a, "E0": float(ra.evals[0]),
                  "matvecs": ra.info.n_matvec, "rc": ra.status},
           "momentum": {"dim": mom.dim, "solve_s": t_m, "E0": float(rm.evals[0]), "matvecs": rm.info.n_matvec},
           "sector_minus_momentum_E0": float(ra.evals[0] - rm.evals[0]), "momentum_over_sector_solve": t_m / t_a}
    sec.close()
    mom.close()
    Lc.close()
    return out


def pg(args):
    """Point-group sectors of the 10 x 10 periodic square (J = Delta = 1) at
    k = 0 for N_down = 5 and 6: per one-dimensional C4v representation the
    block build, the ELL H.v (time over 20 calls; bytes: the packed ELL
    slots, 4 B each, plus 64 B a row) and the
    float64 ground-state solve; the momentum sector k = 0 solved beside it,
    whose ground level the A1 block must reproduce."""
    ctx = _ctx()
    lat = wl.square(10)
    L = qs3.Lattice.of(ctx, lat)
    ops = wl.c4v_ops(10)
    stream = torch.cuda.current_stream()
    out = {"metric": "point-group sector build, H.v and solve vs the momentum sector", "workload": "pg",
           "lattice": lat.name, "group": "C4v x translations", "by_n_down": {}}
    for K in (5, 6):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mom = qs3.Sector(L, K, (0, 0, 0))
        torch.cuda.synchronize()
        t_mom_build = time.perf_counter() - t0
        t0 = time.perf_counter()
        rm = mom.eigs(nev=1, seed=1, stream=stream)
        torch.cuda.synchronize()
        t_mom = time.perf_counter() - t0
        res = {"momentum": {"dim": mom.dim, "build_s": t_mom_build, "solve_s": t_mom, "E0": float(rm.evals[0]),
                            "matvecs": rm.info.n_matvec}}
        mom.close()
        width = K * 4
        for name, chars in wl.C4V_CHARS.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sec = qs3.PGSector(L, K, (0, 0, 0), ops, chars)
            torch.cuda.synchronize()
            t_build = time.perf_counter() - t0
            v = torch.empty(sec.dim, dtype=torch.float64, device="cuda")
            sec.start_vector(1, v, stream=stream)
            w = torch.empty_like(v)
            sec.matvec(v, w, stream=stream)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(20):
                sec.matvec(v, w, stream=stream)
            e1.record(stream)
            e1.synchronize()
            t_mv = e0.elapsed_time(e1) / 20e3
            # one exchange constant: 4 B slots, diagonal, x_a, 1/R_a, y_a, each
            # gathered R_b x_b once, and the R o x staging (read R, x, write)
            nbytes = sec.dim * (4.0 * width + 64.0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            r = sec.eigs(nev=1, seed=1, stream=stream)
            torch.cuda.synchronize()
            t_solve = time.perf_counter() - t0
            res[name] = {"dim": sec.dim, "build_s": t_build, "matvec_us": t_mv * 1e6,
                         "matvec_GBs": nbytes / t_mv / 1e9, "solve_s": t_solve, "E0": float(r.evals[0]),
                         "matvecs": r.info.n_matvec, "rc": r.status}
            if name == "A1":
                # float32 products, float64 recurrences
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r32 = sec.eigs(nev=1, seed=1, precision=qs3.PREC_F32MV, tol=1e-5, stream=stream)
                torch.cuda.synchronize()
                res[name]["f32mv"] = {"solve_s": time.perf_counter() - t0, "matvecs": r32.info.n_matvec,
                                      "rel_err_vs_f64": float(abs(r32.evals[0] - r.evals[0]) / abs(r.evals[0]))}
            del v, w
            sec.close()
            print(f"pg K={K} {name} dim {res[name]['dim']} solve {t_solve:.3f}s", file=sys.stderr, flush=True)
        res["A1_minus_momentum_E0"] = res["A1"]["E0"] - res["momentum"]["E0"]
        res["momentum_over_A1_solve"] = t_mom / res["A1"]["solve_s"]
        out["by_n_down"][K] = res
        torch.cuda.empty_cache()
    L.close()
    # the cube's O_h (48 operations) at 10^3 and the kagome lattice's C6v at
    # 12 x 12, N_down = 4, k = 0: the trivial sector against the momentum sector
    out["cube10_N4_Oh"] = _pg_vs_momentum(ctx, wl.cube(10), wl.oh_ops(10), wl.oh_chars()["A1g"], "A1g", stream)
    out["kagome12_N4_C6v"] = _pg_vs_momentum(ctx, wl.kagome(12, 12), wl.kagome_c6v_ops(12), wl.C6V_CHARS["A1"],
                                             "A1", stream)
    ctx.close()
    return out


# ------------------------------------------------------------------ c2
# counter profile of the fixed-N_down H.v (10x10, N_down = 4) and the sources
# that define that kernel: the profile's traffic holds while they are unchanged
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hv_u1_square10x10_N4.md")
KERNEL_SOURCES = ["paper_2107_00872_amd/csrc/hv_kernels.h", "paper_2107_00872_amd/csrc/qs3_device.h",
                  "paper_2107_00872_amd/csrc/hv_inst.hip", "paper_2107_00872_amd/csrc/qs3_hv.h"]


def kernel_sources_digest():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic():
    """HBM bytes per launch of the fixed-N_down H.v from the committed counter
    profile (FETCH_SIZE + WRITE_SIZE, each scaled by the calibration copy), or
    None when the kernel's sources changed since the counters were taken."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            text = fh.read()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_launch:\s*(\d+)\s+kernel_sources:\s*([0-9a-f]+)", text)
    if not m or m.group(2) != kernel_sources_digest():
        return None
    return int(m.group(1))


def hops_u1(lat, K):
    """Off-diagonal elements of the fixed-N_down matrix: every bond contributes
    one for each state with exactly one end down, 2 * C(N-2, K-1) states."""
    return lat.n_bonds * 2 * math.comb(lat.n_sites - 2, K - 1)


def c2_cpu_baseline(lat, K, budget_s=20.0):
    """The oracle (plain C, Alg. 9 with OpenMP over rows) on the host cores:
    full fixed-N_down H.v of the same sector, repeated within the time budget,
    plus Alg. 9 in one momentum sector."""
    import numpy as np
    from oracle import native as orc
    orc.build(force=False)
    B = orc.Bonds.of(lat)
    d = math.comb(lat.n_sites, K)
    v = np.random.default_rng(0).uniform(-1, 1, size=d)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    reps = 0
    while True:
        orc.hv_u1(lat.n_sites, K, B, v, nthreads=cores)
        reps += 1
        if time.perf_counter() - t0 > budget_s * 0.6:
            break
    t_u1 = (time.perf_counter() - t0) / reps
    sigma, R = orc.mk_list(lat.dims, K, (1, 0, 0), nthreads=cores)
    phi = np.ones(len(sigma), dtype=np.complex128)
    t1 = time.perf_counter()
    orc.hv_k(lat.dims, K, (1, 0, 0), B, sigma, R, phi, nthreads=cores)
    t_k = time.perf_counter() - t1
    return {
        "value": d / t_u1, "unit": "H.v rows/s", "cores": cores, "kind": "oracle",
        "sample": f"{reps} full fixed-N_down H.v of the 10x10 N_down=4 sector "
                  f"({d} rows, {t_u1:.3f} s each); momentum-sector H.v "
                  f"(k=(1,0), {len(sigma)} rows): {len(sigma) / t_k:.3e} rows/s",
        "k_sector_rows_per_s": len(sigma) / t_k,
    }


def c2(args):
    """The 10x10 square at N_down = 4: one step is the full fixed-N_down
    sector's ground state (thick-restart Lanczos, float64), all 100 momentum
    sectors' lowest 5 levels in one batch, and <S_i.S_j> for all pairs and the
    static structure factors of the ground state.  value = H.v rows per second
    over the step; roofline of the fixed-N_down H.v on the full sector."""
    HBM_PEAK_GBS = 8000.0
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)

    lat = wl.square(10)
    K = 4
    ctx = qs3.Context(0)
    L = qs3.Lattice.of(ctx, lat)
    t_setup = time.perf_counter()
    full = qs3.Sector(L, K)
    ks = wl.all_momenta(lat)
    bat = qs3.Batch(L, K, ks)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    d = full.dim
    n_hops = hops_u1(lat, K)
    pairs = [(i, j) for i in range(lat.n_sites) for j in range(lat.n_sites)]
    qs = np.array([[2 * np.pi * kx / lat.lx, 2 * np.pi * ky / lat.ly, 0.0] for (kx, ky, kz) in ks])
    gs_vec = torch.empty(d, dtype=torch.float64, device="cuda")

    t_batch = []

    def one_step(seed):
        rows = 0
        r1 = full.eigs(nev=1, alg=qs3.ALG_TRL, seed=seed, evecs=gs_vec, stream=stream)
        rows += r1.info.n_matvec * d
        tb = time.perf_counter()
        ev, infos, rc = bat.eigs(nev=5, alg=qs3.ALG_TRL, seed=seed, stream=stream)
        t_batch.append(time.perf_counter() - tb)
        # each sector's rows count for the steps it took (converged sectors
        # are masked out of the later launches)
        rows += sum(int(i.n_matvec) * int(dm) for i, dm in zip(infos, bat.dims))
        zz, pm = full.sisj(gs_vec, [p[0] for p in pairs], [p[1] for p in pairs], stream=stream)
        sq = full.sq(gs_vec, qs, stream=stream)
        obs = (zz, pm, sq)
        return rows, r1, ev, infos, obs

    for w in range(args.warmup):
        one_step(100 + w)
    torch.cuda.synchronize()
    times, rows_tot = [], 0
    last = None
    t_all0 = time.perf_counter()
    for s in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rows, r1, ev, infos, obs = one_step(1 + s)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        rows_tot += rows
        last = (r1, ev, infos, obs)
    t_all = time.perf_counter() - t_all0
    ms_per_step = 1e3 * t_all / args.steps

    # ---- roofline of the fixed-N_down H.v on the full sector (the method's hot
    # operation; in the step its kernel time is a minority share beside the
    # multi-dot and Gram-Schmidt kernels of the reorthogonalisation), timed
    # with events recorded on the stream the kernel runs on
    v = torch.empty(d, dtype=torch.float64, device="cuda")
    w = torch.empty_like(v)
    full.start_vector(7, v, stream=stream)
    for _ in range(5):
        full.matvec(v, w, stream=stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.matvec_reps):
        full.matvec(v, w, stream=stream)
    e1.record(stream)
    e1.synchronize()
    t_mv = e0.elapsed_time(e1) / 1e3 / args.matvec_reps
    # a plain device copy of 2^26 float64 (512 MiB read, 512 MiB written) from a
    # buffer larger than the L2 caches: the reference dispatch that scales the
    # FETCH_SIZE / WRITE_SIZE counters of a profiled run to bytes
    cal_src = torch.empty(1 << 26, dtype=torch.float64, device="cuda")
    cal_src.fill_(1.0)
    cal_dst = torch.empty_like(cal_src)
    cal_dst.copy_(cal_src)
    del cal_src, cal_dst
    alg_bytes = 8.0 * (2 * d + n_hops)
    achieved = alg_bytes / t_mv / 1e9
    # float32-row variant of the same kernel
    v32 = v.float()
    w32 = torch.empty_like(v32)
    for _ in range(3):
        full.matvec(v32, w32, stream=stream)
    e0.record(stream)
    for _ in range(args.matvec_reps):
        full.matvec(v32, w32, stream=stream)
    e1.record(stream)
    e1.synchronize()
    t_mv32 = e0.elapsed_time(e1) / 1e3 / args.matvec_reps
    # batched momentum H.v (all 100 sectors in one launch)
    vb = torch.zeros(bat.rows, bat.B, dtype=torch.complex128, device="cuda")
    vb.real.uniform_(-1, 1)
    wb = torch.empty_like(vb)
    for _ in range(3):
        bat.matvec(vb, wb, stream=stream)
    e0.record(stream)
    for _ in range(args.matvec_reps):
        bat.matvec(vb, wb, stream=stream)
    e1.record(stream)
    e1.synchronize()
    t_bat = e0.elapsed_time(e1) / 1e3 / args.matvec_reps

    # ---- the same 100 momentum solves one at a time (plain float64 path, the
    # sectors created beforehand), seeds as in the batch of the last step
    r1, ev, infos, obs = last
    serial = None
    if not args.no_one_at_a_time:
        secs = [qs3.Sector(L, K, k) for k in ks]
        torch.cuda.synchronize()
        ts = time.perf_counter()
        ev_serial = [secs[b].eigs(nev=5, alg=qs3.ALG_TRL, seed=args.steps + b, stream=stream).evals
                     for b in range(len(ks))]
        torch.cuda.synchronize()
        t_serial = time.perf_counter() - ts
        for sc in secs:
            sc.close()
        ev_serial = np.array(ev_serial)
        both = np.isfinite(ev_serial) & np.isfinite(ev)
        serial = {"solves_per_s": len(ks) / t_serial, "seconds": t_serial,
                  "batched_solves_per_s": bat.B / t_batch[-1], "batched_seconds": t_batch[-1],
                  "max_rel_diff": float(np.max(np.abs(ev_serial[both] - ev[both]) / np.abs(ev[both])))}
    out = {
        "metric": "H.v rows/s (whole solve step) + %HBM roofline of the H.v kernel",
        "value": rows_tot / t_all,
        "unit": "H.v rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "10x10 periodic square Heisenberg J=Delta=1, N_down=4: full sector "
                               "(dim 3921225) ground state + all 100 momentum sectors lowest 5 levels "
                               "(batched) + <S_i.S_j>, S(q)",
                   "sectors_per_step": 1 + bat.B, "full_dim": d, "k_rows": bat.rows},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": profiled_traffic(),
                     "kernel": "k_hv_u1<4,uint32,double,double>",
                     "alg_bytes_per_launch": alg_bytes, "launch_s": t_mv},
        "matvec": {"u1_f64_rows_per_s": d / t_mv, "u1_f32_rows_per_s": d / t_mv32,
                   "u1_f32_ms": t_mv32 * 1e3, "u1_f64_ms": t_mv * 1e3,
                   "batch100_rows_per_s": bat.rows * bat.B / t_bat, "batch100_ms": t_bat * 1e3},
        "solves_per_s": (1 + bat.B) / (t_all / args.steps),
        "k_sectors_one_at_a_time": serial,
        "step_ms_p50": 1e3 * float(np.percentile(times, 50)),
        "step_ms_max": 1e3 * float(np.max(times)),
        "setup_s": t_setup,
        "results": {"E0_full": float(r1.evals[0]), "full_matvecs": r1.info.n_matvec,
                    "full_restarts": r1.info.n_restarts, "min_k_E0": float(np.nanmin(ev[:, 0])),
                    "batch_matvecs": infos[0].n_matvec,
                    "all_converged": bool(r1.status == 0 and all(i.converged for i in infos))},
    }
    out["workload"] = "c2"
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = c2_cpu_baseline(lat, K)
    return out


def c2_summary(ctx, stream, steps=3):
    """Secondary figures of the 10x10 square at N_down = 4 for the headline
    line: the step of c2 (full-sector ground state, 100 momentum sectors'
    lowest 5 levels, all-pairs correlations and S(q)) timed over a few steps,
    and the fixed-N_down H.v on the full sector against the HBM roofline."""
    lat = wl.square(10)
    K = 4
    L = qs3.Lattice.of(ctx, lat)
    full = qs3.Sector(L, K)
    ks = wl.all_momenta(lat)
    bat = qs3.Batch(L, K, ks)
    d = full.dim
    pairs = [(i, j) for i in range(lat.n_sites) for j in range(lat.n_sites)]
    qs = np.array([[2 * np.pi * kx / lat.lx, 2 * np.pi * ky / lat.ly, 0.0] for (kx, ky, kz) in ks])
    gs_vec = torch.empty(d, dtype=torch.float64, device="cuda")

    def one_step(seed):
        r1 = full.eigs(nev=1, seed=seed, evecs=gs_vec, stream=stream)
        ev, infos, rc = bat.eigs(nev=5, seed=seed, stream=stream)
        full.sisj(gs_vec, [p[0] for p in pairs], [p[1] for p in pairs], stream=stream)
        full.sq(gs_vec, qs, stream=stream)
        rows = r1.info.n_matvec * d + sum(int(i.n_matvec) * int(dm) for i, dm in zip(infos, bat.dims))
        return rows, r1, ev

    one_step(100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rows = 0
    for s_ in range(steps):
        r, r1, ev = one_step(1 + s_)
        rows += r
    torch.cuda.synchronize()
    t_step = (time.perf_counter() - t0) / steps
    v = torch.empty(d, dtype=torch.float64, device="cuda")
    w = torch.empty_like(v)
    full.start_vector(7, v, stream=stream)
    for _ in range(3):
        full.matvec(v, w, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(20):
        full.matvec(v, w, stream=stream)
    e1.record(stream)
    e1.synchronize()
    t_mv = e0.elapsed_time(e1) / 1e3 / 20
    alg = 8.0 * (2 * d + hops_u1(lat, K))
    out = {"workload": "10x10 square J=Delta=1, N_down=4: full sector ground state + 100 momentum sectors "
                       "lowest 5 levels + <S_i.S_j>, S(q)",
           "step_ms": 1e3 * t_step, "rows_per_s": rows / steps / t_step, "E0_full": float(r1.evals[0]),
           "min_k_E0": float(np.nanmin(ev[:, 0])),
           "k_hv_u1": {"launch_us": t_mv * 1e6, "achieved_GBs": alg / t_mv / 1e9,
                       "frac": alg / t_mv / 8e12, "alg_bytes_per_launch": alg}}
    bat.close()
    full.close()
    L.close()
    return out
