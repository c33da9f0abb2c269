"""Benchmark of the XXZ H.v + thick-restart Lanczos hot path on one MI355X.

Default workload: the periodic 10x10x10 cube, isotropic Heisenberg
(J = Delta = 1), N_down = 3 -- C(1000, 3) = 166,167,000 states, 1000 momentum
sectors of 166,167 representatives each.  One step is the ground level E_0(k)
of all 1000 sectors in one batched thick-restart solve (float64, default
solver settings; every H.v of the solve is one batched launch over the
sectors still iterating).
  value        H.v sector-rows per second over the step (each sector's rows
               counted for every H.v it took)
  roofline     the batched momentum H.v over all 1000 sectors (the method's
               hot operation, k_hv_batch): algorithmic bytes per launch =
               16 B x (2 x rows x sectors + hops per sector x sectors), the
               launch time from HIP events on the stream it runs on
  one_at_a_time  the plain float64 path on a seeded sample of sectors, one
               solve after the other: solves/s and per-solve latency p50/p99
  f32mv        one batched solve with float32 products (float64 recurrences)
               and its largest eigenvalue error against the float64 step
  accuracy     E_0 of the sectors stored by the oracle (tests/golden) against
               the step's values
  c2           the 10x10 square, N_down = 4 step (full sector + 100 momentum
               sectors + correlations) as secondary figures
  cpu_baseline the oracle's cached-structure momentum H.v (plain C, OpenMP
               over rows) on a seeded sample of sectors, all host cores and
               one core

Other workloads print their own line: --workload c1|c2|c4|c5|szq|thermal|cells|pg
(bench_extra.py).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# counter profile of the batched momentum H.v on this workload and the sources
# that define that kernel: the profile's traffic holds while they are unchanged
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hv_batch_cube10_N3_1000k.md")
KERNEL_SOURCES = ["paper_2107_00872_amd/csrc/hv_kernels.h", "paper_2107_00872_amd/csrc/qs3_device.h",
                  "paper_2107_00872_amd/csrc/hv_inst.hip", "paper_2107_00872_amd/csrc/qs3_hv.h"]
GOLDEN = os.path.join(ROOT, "tests", "golden", "full_size_levels.json")


def kernel_sources_digest():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic():
    """HBM bytes per launch of the batched H.v from the committed counter
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


def hops_per_sector(lat, K):
    """Off-diagonal elements of one momentum block of a lattice whose orbits
    are all full (every stabiliser trivial): the fixed-N_down count
    N_b * 2 * C(N-2, K-1) divided over the N translations."""
    return lat.n_bonds * 2 * math.comb(lat.n_sites - 2, K - 1) / lat.n_sites


def cpu_baseline(lat, K, ks, n_sample=20, budget_s=20.0):
    """The oracle's cached-structure momentum H.v (plain C: every hop of every
    representative resolved once by the search over all translations, then
    reused for every momentum; OpenMP over rows) on a seeded sample of the
    1000 sectors -- Gamma, X, M, R and 16 random momenta -- on all host cores,
    and on one core for two of them.  The structure build is timed apart."""
    import numpy as np
    from oracle import native as orc
    orc.build(force=False)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    t0 = time.perf_counter()
    S = orc.KStruct(lat.dims, K, orc.Bonds.of(lat), nthreads=cores)
    t_build = time.perf_counter() - t0
    rng = np.random.default_rng(2021)
    fixed = [(0, 0, 0), (5, 0, 0), (5, 5, 0), (5, 5, 5)]
    rest = [k for k in ks if k not in fixed]
    sample = fixed + [rest[i] for i in rng.choice(len(rest), n_sample - len(fixed), replace=False)]
    rows, t_all = 0, 0.0
    t_end = time.perf_counter() + budget_s
    done = 0
    for Kv in sample:
        mem, sig, R = S.sector(Kv)
        phi = rng.uniform(-1, 1, len(mem)) + 1j * rng.uniform(-1, 1, len(mem))
        t1 = time.perf_counter()
        S.hv(Kv, mem, R, phi, nthreads=cores)
        t_all += time.perf_counter() - t1
        rows += len(mem)
        done += 1
        if time.perf_counter() > t_end:
            break
    r1, t1c = 0, 0.0
    for Kv in sample[:2]:
        mem, sig, R = S.sector(Kv)
        phi = np.ones(len(mem), dtype=np.complex128)
        t1 = time.perf_counter()
        S.hv(Kv, mem, R, phi, nthreads=1)
        t1c += time.perf_counter() - t1
        r1 += len(mem)
    S.close()
    return {"value": rows / t_all, "unit": "H.v sector-rows/s", "cores": cores, "kind": "oracle",
            "sample": f"one H.v in each of {done} sectors (Gamma, X, M, R and seeded random momenta), "
                      f"{rows} rows, {t_all:.2f} s; cached structure (166,167 representatives, all hops "
                      f"resolved once) built in {t_build:.1f} s on {cores} threads",
            "one_core_value": r1 / t1c, "structure_build_s": t_build}


def accuracy_vs_golden(ks, e0):
    """Relative errors of the step's E_0(k) against the oracle's stored values."""
    try:
        with open(GOLDEN) as fh:
            gold = json.load(fh)["c3"]["sectors"]
    except (OSError, KeyError):
        return None
    errs = {}
    for s in gold:
        b = ks.index(tuple(s["k"]))
        errs[str(tuple(s["k"]))] = abs(e0[b] - s["levels"][0]) / abs(s["levels"][0])
    return {"sectors": len(errs), "max_rel_err": max(errs.values()), "per_sector": errs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--matvec-reps", type=int, default=10)
    ap.add_argument("--no-one-at-a-time", action="store_true",
                    help="skip the one-sector-at-a-time comparison (shorter profiles)")
    ap.add_argument("--no-c2", action="store_true", help="skip the secondary 10x10 figures")
    ap.add_argument("--krylov-only", action="store_true",
                    help="only two restart cycles of the batched solve at full width (every sector "
                         "iterating) and the calibration copy (counter profiles of the Krylov kernels)")
    ap.add_argument("--matvec-only", action="store_true",
                    help="only the batched H.v launches and the calibration copy (counter profiles)")
    ap.add_argument("--requests", type=int, default=0, help="c5: number of requests (default 200)")
    ap.add_argument("--cells", default="both", choices=["kagome", "pyrochlore", "both"],
                    help="cells: which unit-cell lattice to run (default both)")
    ap.add_argument("--workload", default="c3",
                    choices=["c1", "c2", "c3", "c4", "c5", "szq", "thermal", "cells", "pg"],
                    help="c3 (default) is the headline configuration; the others print their own line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (independent "
              "sectors would shard across GPUs with no exchange; one sector by rank range "
              "with an all-gather of v per step)", file=sys.stderr)
        sys.exit(2)
    if args.workload != "c3":
        import bench_extra
        print(json.dumps(getattr(bench_extra, args.workload)(args)))
        return

    import numpy as np
    import torch

    import workloads as wl
    from paper_2107_00872_amd import qs3

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    torch.cuda.set_stream(stream)

    lat = wl.cube(10)
    K = 3
    ctx = qs3.Context(0)
    L = qs3.Lattice.of(ctx, lat)
    ks = wl.all_momenta(lat)
    t_setup = time.perf_counter()
    bat = qs3.Batch(L, K, ks)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    dims = bat.dims.astype(np.int64)

    def one_step(seed):
        ev, infos, rc = bat.eigs(nev=1, seed=seed, stream=stream)
        rows = sum(int(i.n_matvec) * int(dm) for i, dm in zip(infos, dims))
        return rows, ev, infos, rc

    print(f"c3: {bat.rows} representatives x {bat.B} sectors, set-up {t_setup:.2f} s", file=sys.stderr,
          flush=True)
    if args.krylov_only:
        # two thick-restart cycles (at most one restart) of the float64 solve,
        # twice: the first call also times the H.v schedules
        for rep in range(2):
            t0 = time.perf_counter()
            ev, infos, rc = bat.eigs(nev=1, seed=1, stream=stream, max_restarts=1)
            torch.cuda.synchronize()
            print(f"two cycles: {time.perf_counter() - t0:.3f} s, {max(int(i.n_matvec) for i in infos)} steps",
                  file=sys.stderr, flush=True)
        cal_src = torch.empty(1 << 26, dtype=torch.float64, device="cuda")
        cal_src.fill_(1.0)
        cal_dst = torch.empty_like(cal_src)
        cal_dst.copy_(cal_src)
        torch.cuda.synchronize()
        print(json.dumps({"workload": "c3 Krylov cycles only"}))
        return
    if args.matvec_only:
        args.steps = args.warmup = 0
    for w in range(args.warmup):
        one_step(100 + w)
        print(f"warmup {w + 1}/{args.warmup}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    times, rows_tot, last = [], 0, None
    t_all0 = time.perf_counter()
    for s in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rows, ev, infos, rc = one_step(1 + s)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        rows_tot += rows
        last = (ev, infos, rc)
        print(f"step {s + 1}/{args.steps}: {times[-1]:.2f} s", file=sys.stderr, flush=True)
    t_all = time.perf_counter() - t_all0

    # ---- roofline of the batched H.v over all 1000 sectors, timed with events
    # recorded on the stream the kernel runs on
    v = torch.zeros(bat.rows, bat.B, dtype=torch.complex128, device="cuda")
    v.real.uniform_(-1, 1)
    w = torch.empty_like(v)
    for _ in range(2):
        bat.matvec(v, w, stream=stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.matvec_reps):
        bat.matvec(v, w, stream=stream)
    e1.record(stream)
    e1.synchronize()
    t_mv = e0.elapsed_time(e1) / 1e3 / args.matvec_reps
    # a plain device copy of 2^26 float64 (512 MiB read, 512 MiB written) from a
    # buffer larger than the L2 and MALL caches: the reference dispatch that
    # scales the FETCH_SIZE / WRITE_SIZE counters of a profiled run to bytes
    cal_src = torch.empty(1 << 26, dtype=torch.float64, device="cuda")
    cal_src.fill_(1.0)
    cal_dst = torch.empty_like(cal_src)
    cal_dst.copy_(cal_src)
    del cal_src, cal_dst, v, w
    torch.cuda.empty_cache()
    nh = hops_per_sector(lat, K)
    # the product runs as `ngr` equal launches over `gw` sectors each (wide
    # batches of long vectors go in groups of at most 256 sectors)
    ngr, gw = bat.groups()
    alg_bytes = 16.0 * (2 * bat.rows + nh) * gw
    t_launch = t_mv / ngr
    achieved = alg_bytes / t_launch / 1e9
    G, bpc = bat.schedule()
    per = -(-gw // G)
    bpl, npass = (per, 1) if per <= 8 else (8, -(-per // 8))
    bpl = 1 << (bpl - 1).bit_length()
    roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": profiled_traffic(),
                "kernel": f"k_hv_batch<3,uint32,double,double,HOP_LISTS,{bpl},{npass}>",
                "schedule": {"lanes_per_row": G, "blocks_per_cu": bpc, "launches_per_product": ngr,
                             "sectors_per_launch": gw},
                "alg_bytes_per_launch": alg_bytes, "launch_s": t_launch, "product_s": t_mv}
    # the single-sector product (one lane per row) on one of the sectors
    one = qs3.Sector(L, K, (3, 6, 0))
    v1 = torch.empty(one.dim, dtype=torch.complex128, device="cuda")
    one.start_vector(1, v1, stream=stream)
    w1 = torch.empty_like(v1)
    for _ in range(2):
        one.matvec(v1, w1, stream=stream)
    e0.record(stream)
    for _ in range(20):
        one.matvec(v1, w1, stream=stream)
    e1.record(stream)
    e1.synchronize()
    t1 = e0.elapsed_time(e1) / 1e3 / 20
    # per row: own v and w, one gather per hop (16 B each), the representative
    # rank (8 B) and stabiliser size (2 B)
    alg1 = (16.0 * (2 + nh / bat.rows) + 10.0) * one.dim
    one_sector = {"kernel": "k_hv_one_lists<double,double,18>", "rows": one.dim, "launch_us": t1 * 1e6,
                  "achieved_GBs": alg1 / t1 / 1e9, "frac": alg1 / t1 / 1e9 / HBM_PEAK_GBS,
                  "alg_bytes_per_launch": alg1}
    one.close()
    del v1, w1
    if args.matvec_only:
        print(json.dumps({"workload": "c3 batched H.v only", "roofline": roofline, "one_sector_hv": one_sector}))
        return
    ms_per_step = 1e3 * t_all / args.steps
    ev, infos, rc = last
    mv = np.array([i.n_matvec for i in infos])

    # ---- the plain float64 path one sector at a time on a seeded sample, the
    # batch's seeds (sector b of the batch uses seed + b)
    serial = None
    if not args.no_one_at_a_time:
        sample = sorted(np.random.default_rng(2021).choice(len(ks), 20, replace=False).tolist())
        secs = [qs3.Sector(L, K, ks[b]) for b in sample]
        torch.cuda.synchronize()
        lat_s, e_s = [], []
        for i, b in enumerate(sample):
            t0 = time.perf_counter()
            r = secs[i].eigs(nev=1, seed=args.steps + b, stream=stream)
            lat_s.append(time.perf_counter() - t0)
            e_s.append(r.evals[0])
        for sc in secs:
            sc.close()
        e_s = np.array(e_s)
        serial = {"sample": len(sample), "solves_per_s": len(sample) / sum(lat_s),
                  "latency_ms_p50": 1e3 * float(np.percentile(lat_s, 50)),
                  "latency_ms_p99": 1e3 * float(np.percentile(lat_s, 99)),
                  "max_rel_diff_vs_batched": float(np.max(np.abs(e_s - ev[sample, 0]) / np.abs(e_s))),
                  "batched_speedup": (bat.B / (t_all / args.steps)) / (len(sample) / sum(lat_s))}
        print(f"one at a time: {serial['solves_per_s']:.1f} solves/s", file=sys.stderr, flush=True)

    # ---- the float32-matvec variant (float64 recurrences): one batched solve
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev32, infos32, rc32 = bat.eigs(nev=1, seed=1, precision=qs3.PREC_F32MV, stream=stream)
    torch.cuda.synchronize()
    t32 = time.perf_counter() - t0
    f32mv = {"seconds": t32, "solves_per_s": bat.B / t32, "rc": rc32,
             "max_rel_err_vs_f64": float(np.max(np.abs(ev32[:, 0] - ev[:, 0]) / np.abs(ev[:, 0])))}

    out = {
        "metric": "H.v rows/s + %HBM roofline of the batched H.v; sector solves/s vs plain float64 one at a time",
        "value": rows_tot / t_all,
        "unit": "H.v sector-rows/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "10x10x10 periodic cube Heisenberg J=Delta=1, N_down=3: ground level E_0(k) of "
                               "all 1000 momentum sectors (166,167 representatives each) in one batched "
                               "thick-restart solve, float64",
                   "sectors": bat.B, "rows_per_sector": int(bat.rows)},
        "roofline": roofline,
        "solves_per_s": bat.B / (t_all / args.steps),
        "step_ms_p50": 1e3 * float(np.percentile(times, 50)),
        "step_ms_max": 1e3 * float(np.max(times)),
        "setup_s": t_setup,
        "matvecs_per_sector": {"max": int(mv.max()), "p50": float(np.median(mv))},
        "results": {"E_min": float(ev[:, 0].min()), "E_gamma": float(ev[ks.index((0, 0, 0)), 0]),
                    "all_converged": bool(rc == 0 and all(i.converged for i in infos))},
        "one_at_a_time_f64": serial,
        "one_sector_hv": one_sector,
        "f32mv": f32mv,
        "accuracy_vs_oracle": accuracy_vs_golden(ks, ev[:, 0]),
    }
    del bat
    torch.cuda.empty_cache()
    if not args.no_c2:
        import bench_extra
        out["c2"] = bench_extra.c2_summary(ctx, stream)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(lat, K, ks)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
