"""Writes tests/golden/full_size_levels.json: oracle values at the full sizes
of the benchmark workloads.  Calls only oracle/ (and numpy / scipy as library
steps); nothing here reads a value computed by the HIP library.

  c2_full  10x10 periodic square, J = Delta = 1, N_down = 4, fixed N_down
           (3,921,225 rows): lowest distinct levels
  c2_k     the same lattice, three momentum sectors: lowest 5 distinct levels
  c3       10x10x10 periodic cube, N_down = 3, nine momentum sectors (among
           them sectors whose lowest two levels are split by ~2e-6 at
           E ~ 734, 3e-9 relative): lowest distinct levels
  c4       10x10 square, N_down = 3 ground state (lowest level over the 100
           momenta, dense diagonalisation of every block) and S^-(q, omega)
           for three q: S^-_q by the scatter of Sec. 3.8 into N_down = 4,
           300 fully reorthogonalised Lanczos levels (Alg. 10), the continued
           fraction of Eq. (cfe) at eta = 0.05, h = 4, omega = linspace(0, 8, 2000)

Eigenvalues come from two solvers on the same oracle operator (the row-by-row
Alg. 9 of the plain C oracle, or its cached-structure variant): the oracle's
fully reorthogonalised Lanczos and scipy's eigsh (ARPACK); both must agree to
1e-11 relative on every stored level.

Usage: python tests/golden/make_goldens.py [c2_full] [c2_k] [c3] [c4] [--threads N]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np
from scipy.sparse.linalg import LinearOperator, eigsh

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import native as orc  # noqa: E402
from oracle.dynamics import continued_fraction  # noqa: E402
from oracle.lanczos import lanczos, lowest_distinct, ritz  # noqa: E402

OUT = os.path.join(HERE, "full_size_levels.json")
AGREE = 1e-11


def log(*a):
    print(*a, flush=True)


def two_solvers(matvec, d, dtype, n_levels, k_eigsh, ncv, steps, seed):
    """Lowest n_levels distinct levels by eigsh and by the oracle's Lanczos
    (full reorthogonalisation, `steps` steps; a level counts when its Ritz
    residual is below 1e-11 max(1, |E|))."""
    rng = np.random.default_rng(seed)
    v0 = rng.uniform(-1, 1, size=d)
    if dtype == np.complex128:
        v0 = v0 + 1j * rng.uniform(-1, 1, size=d)
    cnt = [0]

    def mv(x):
        cnt[0] += 1
        return matvec(np.ascontiguousarray(x.ravel(), dtype=dtype))
    t0 = time.time()
    w = eigsh(LinearOperator((d, d), matvec=mv, dtype=dtype), k=k_eigsh, which="SA", tol=1e-14,
              ncv=ncv, v0=v0, maxiter=100000, return_eigenvectors=False)
    lv_e = lowest_distinct(np.sort(w), n_levels)
    t_e, n_e = time.time() - t0, cnt[0]
    t0 = time.time()
    a, b, _ = lanczos(matvec, v0.astype(dtype), steps)
    e, res, _ = ritz(a, b)
    lv_l = lowest_distinct(e, n_levels, residuals=res, res_rel=1e-11)
    t_l = time.time() - t0
    n = min(len(lv_e), len(lv_l))
    diff = max(abs(x - y) / max(1.0, abs(x)) for x, y in zip(lv_e[:n], lv_l[:n]))
    log(f"  eigsh {lv_e} ({n_e} matvecs, {t_e:.0f} s)\n  lanczos {lv_l} ({len(a)} steps, {t_l:.0f} s)"
        f"  max rel diff {diff:.2e}")
    assert n == n_levels and diff <= AGREE, "the two oracle solvers disagree"
    return {"levels": lv_e, "eigsh": lv_e, "lanczos": lv_l, "lanczos_steps": int(len(a)),
            "eigsh_matvecs": n_e, "max_rel_diff": diff}


def c2_full(out, nt):
    lat = wl.square(10)
    B = orc.Bonds.of(lat)
    d = math.comb(100, 4)
    log("c2_full", d)
    r = two_solvers(lambda x: orc.hv_u1(100, 4, B, x, nthreads=nt), d, np.float64, 2, 4, 30, 300, 1)
    out["c2_full"] = {"lattice": "square 10x10 periodic, J = Delta = 1", "n_down": 4, "dim": d, **r}


def c2_k(out, nt):
    lat = wl.square(10)
    ks = orc.KStruct(lat.dims, 4, orc.Bonds.of(lat), nthreads=nt)
    res = []
    for Kv in [(0, 0, 0), (1, 0, 0), (5, 5, 0)]:
        mem, sig, R = ks.sector(Kv)
        log("c2_k", Kv, len(mem))
        r = two_solvers(lambda x: ks.hv(Kv, mem, R, x, nthreads=nt), len(mem), np.complex128, 5, 16, 64,
                        900, 2)
        res.append({"k": list(Kv), "dim": int(len(mem)), **r})
    out["c2_k"] = {"lattice": "square 10x10 periodic, J = Delta = 1", "n_down": 4, "sectors": res}


C3_SECTORS = [(3, 6, 0), (3, 2, 0), (0, 2, 3), (5, 0, 9), (7, 8, 0), (0, 6, 8), (0, 0, 0), (5, 5, 5),
              (1, 0, 0)]


def c3(out, nt):
    lat = wl.cube(10)
    t0 = time.time()
    ks = orc.KStruct(lat.dims, 3, orc.Bonds.of(lat), nthreads=nt)
    log(f"c3 structure {time.time() - t0:.0f} s: {ks.nrep} representatives, {ks.nhops} hops")
    res = []
    for Kv in C3_SECTORS:
        mem, sig, R = ks.sector(Kv)
        log("c3", Kv, len(mem))
        r = two_solvers(lambda x: ks.hv(Kv, mem, R, x, nthreads=nt), len(mem), np.complex128, 2, 4, 40,
                        700, 3)
        res.append({"k": list(Kv), "dim": int(len(mem)), **r})
    out["c3"] = {"lattice": "cube 10x10x10 periodic, J = Delta = 1", "n_down": 3, "sectors": res}


C4_Q = [(1, 0, 0), (5, 5, 0), (3, 7, 0)]


def c4(out, nt):
    lat = wl.square(10)
    B = orc.Bonds.of(lat)
    ks3 = orc.KStruct(lat.dims, 3, B, nthreads=nt)
    ks4 = orc.KStruct(lat.dims, 4, B, nthreads=nt)
    # ground state: dense diagonalisation of every N_down = 3 block
    best = None
    lows = {}
    for Kv in wl.all_momenta(lat):
        mem, sig, R = ks3.sector(Kv)
        d = len(mem)
        H = np.zeros((d, d), dtype=np.complex128)
        e = np.zeros(d, dtype=np.complex128)
        for j in range(d):
            e[:] = 0
            e[j] = 1
            H[:, j] = ks3.hv(Kv, mem, R, e, nthreads=nt)
        assert np.abs(H - H.conj().T).max() < 1e-12
        w, V = np.linalg.eigh(H)
        lows[Kv] = w[:3]
        # READING: the lowest level over the momenta, ties to the smallest (Kx, Ky)
        if best is None or w[0] < best[0] - 1e-10:
            best = (w[0], Kv, V[:, 0], sig, R, w)
    e0, k0, phi, sig, R, w = best
    gap = float(w[1] - w[0])
    ties = [list(Kv) for Kv, lw in lows.items() if abs(lw[0] - e0) <= 1e-10 * abs(e0)]
    log(f"c4 ground state E0 = {e0:.12f} at k0 = {k0}, next level in the sector +{gap:.3e}, "
        f"momenta within 1e-10: {ties}")
    omega = np.linspace(0.0, 8.0, 2000)
    eta, h, steps = 0.05, 4.0, 300
    qs = []
    for Qv in C4_Q:
        kq = tuple((k0[i] + Qv[i]) % lat.dims[i] for i in range(3))
        mem1, sig1, R1 = ks4.sector(kq)
        psi = orc.smq(lat.dims, 3, k0, sig, R, phi, sig1, R1, Qv, nthreads=nt)
        wq = float(np.vdot(psi, psi).real)
        a, b, _ = lanczos(lambda x: ks4.hv(kq, mem1, R1, x, nthreads=nt), psi, steps)
        S = continued_fraction(a, b, wq, omega, e0, eta, h, "-")
        log(f"  q = {Qv}: |S^-_q phi|^2 = {wq:.12f}, max S = {S.max():.6f}")
        qs.append({"q": list(Qv), "k_plus_q": list(kq), "dim": int(len(mem1)), "weight": wq,
                   "alpha": a.tolist(), "beta": b.tolist(), "S": S.tolist()})
    out["c4"] = {"lattice": "square 10x10 periodic, J = Delta = 1", "n_down": 3, "E0": float(e0),
                 "k0": list(k0), "gap_in_k0": gap, "lowest_by_k": {str(k): [float(x) for x in v]
                                                                  for k, v in lows.items()},
                 "eta": eta, "field": h, "steps": steps, "omega": [0.0, 8.0, 2000], "q": qs}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("parts", nargs="*", default=["c2_full", "c2_k", "c3", "c4"])
    ap.add_argument("--threads", type=int, default=os.cpu_count() or 1)
    args = ap.parse_args()
    orc.build(force=False)
    out = json.load(open(OUT)) if os.path.exists(OUT) else {}
    out["citation"] = ("oracle values (plain C Alg. 9 / cached structure, oracle Lanczos with full "
                       "reorthogonalisation and scipy eigsh; dense diagonalisation and Sec. 3.8-3.9 "
                       "for S(q, omega)) written by tests/golden/make_goldens.py")
    for p in args.parts:
        globals()[p](out, args.threads)
        with open(OUT, "w") as fh:
            json.dump(out, fh, indent=1)
        log("wrote", p)


if __name__ == "__main__":
    main()
