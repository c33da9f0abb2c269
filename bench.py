"""Benchmark of the XXZ H.v + Lanczos hot path on one MI355X.

Default workload (10x10 periodic square-lattice Heisenberg, J = Delta = 1,
N_down = 4): one step is
  * the full fixed-N_down sector (dim C(100,4) = 3,921,225): thick-restart
    Lanczos ground state, float64;
  * all 100 momentum sectors (about 39.2k states each) in one batch: the
    lowest 5 distinct levels per sector by thick-restart Lanczos, float64;
  * observables of the full-sector ground state: <S_i.S_j> for all pairs and
    the static structure factors at all 100 momenta.
value = H.v rows processed per second over the whole step (matvec rows summed
over every sector and every Lanczos step, divided by the step's wall time).

The roofline object is for the dominant H.v kernel, the fixed-N_down pull
kernel on the full sector: algorithmic bytes per launch = 8 B x (own row read
+ row write + one gather per off-diagonal element) = 8 (2 d + n_hops) with
n_hops = N_b * 2 * C(N-2, K-1), divided by the kernel's average duration from
HIP events on the stream it runs on.

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


# counter profile of the fixed-N_down H.v (10x10, N_down = 4) and the sources
# that define that kernel: the profile's traffic holds while they are unchanged
ROOT = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "hv_u1_square10x10_N4.md")
KERNEL_SOURCES = ["paper_2107_00872_amd/csrc/hv_kernels.h", "paper_2107_00872_amd/csrc/qs3_device.h",
                  "paper_2107_00872_amd/csrc/hv_inst.hip"]


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


def cpu_baseline(lat, K, budget_s=20.0):
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--matvec-reps", type=int, default=50)
    ap.add_argument("--no-one-at-a-time", action="store_true",
                    help="skip the one-sector-at-a-time comparison (shorter profiles)")
    ap.add_argument("--requests", type=int, default=0, help="c5: number of requests (default 40)")
    ap.add_argument("--cells", default="both", choices=["kagome", "pyrochlore", "both"],
                    help="cells: which unit-cell lattice to run (default both)")
    ap.add_argument("--workload", default="c2", choices=["c1", "c2", "c3", "c4", "c5", "szq", "thermal", "cells", "pg"],
                    help="c2 (default) is the headline configuration; the others print their own line")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (independent "
              "sectors would shard across GPUs with no exchange; one sector by rank range "
              "with an all-gather of v per step)", file=sys.stderr)
        sys.exit(2)
    if args.workload != "c2":
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
        obs = None
        try:
            zz, pm = full.sisj(gs_vec, [p[0] for p in pairs], [p[1] for p in pairs], stream=stream)
            sq = full.sq(gs_vec, qs, stream=stream)
            obs = (zz, pm, sq)
        except qs3.QS3Error:
            pass
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

    # ---- roofline of the dominant kernel: fixed-N_down H.v on the full sector,
    # timed with events recorded on the stream the kernel runs on
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
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(lat, K)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
