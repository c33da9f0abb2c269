"""Expectation values (Sec. 3.6) and static structure factors (Sec. 4.2), from the
definitions, on U(1)-basis amplitudes phi[a-1] (a = rank of Eq. (a_of_n)).

A momentum-sector vector is first expanded to U(1) amplitudes with
translation.expand_to_u1; for an eigenstate of T the paper's translation-
averaged operators (1/N) sum_j T^j O T^-j give exactly <O>, so no separate
averaging is needed here.

s^z on a basis state is +1/2 on up sites and -1/2 on down sites;
s^+_i s^-_j (i != j) moves the down spin at i to j.
"""
from __future__ import annotations

import itertools

import numpy as np

from .cns import C, F


def all_tuples(N: int, K: int):
    """Every ascending 1-based tuple in rank order (rank = position + 1)."""
    tups = sorted(itertools.combinations(range(1, N + 1), K), key=F)
    return tups


def sz(phi: np.ndarray, N: int, K: int) -> np.ndarray:
    """<s^z_r> for r = 1..N (returned 0-based)."""
    p = np.abs(phi) ** 2
    nrm = p.sum()
    out = np.full(N, 0.5)
    for a, n in enumerate(all_tuples(N, K)):
        for r in n:
            out[r - 1] -= p[a] / nrm
    return out


def corr_zz(phi: np.ndarray, N: int, K: int) -> np.ndarray:
    """<s^z_i s^z_j> for all pairs (0-based matrix)."""
    p = np.abs(phi) ** 2
    p = p / p.sum()
    out = np.zeros((N, N))
    for a, n in enumerate(all_tuples(N, K)):
        s = np.full(N, 0.5)
        for r in n:
            s[r - 1] = -0.5
        out += p[a] * np.outer(s, s)
    return out


def corr_pm(phi: np.ndarray, N: int, K: int) -> np.ndarray:
    """<s^+_i s^-_j> for all pairs (0-based matrix); i == j gives <1/2 + s^z_i>."""
    nrm = np.vdot(phi, phi).real
    tups = all_tuples(N, K)
    out = np.zeros((N, N), dtype=np.complex128)
    for a, n in enumerate(tups):
        if phi[a] == 0:
            continue
        ns = set(n)
        for i in n:                          # s^+_i needs i down
            for j in range(1, N + 1):        # s^-_j needs j up
                if j in ns:
                    continue
                n2 = tuple(sorted((ns - {i}) | {j}))
                out[i - 1, j - 1] += np.conj(phi[F(n2) - 1]) * phi[a]
    out /= nrm
    szv = sz(phi, N, K)
    out[np.arange(N), np.arange(N)] = 0.5 + szv
    return out


def positions(lx: int, ly: int, lz: int) -> np.ndarray:
    """Integer coordinates R_r of sites r = 1..N (row r-1)."""
    N = lx * ly * lz
    i = np.arange(N)
    return np.stack([i % lx, (i // lx) % ly, i // (lx * ly)], axis=1).astype(np.float64)


def structure_factors(zz: np.ndarray, pm: np.ndarray, szv: np.ndarray, R: np.ndarray,
                      qs: np.ndarray):
    """S^zz(q), S^{+-}(q) and S(q) = <S_{-q} . S_q> with
    S^a_q = N^{-1/2} sum_r e^{-i q.R_r} s^a_r (Sec. 3.8 and Sec. 4.2):
      S^zz(q)  = (1/N) sum_{r,r'} e^{i q.(R_r - R_r')} <s^z_r s^z_r'>
      S^{+-}(q) = (1/N) sum_{r,r'} e^{i q.(R_r - R_r')} <s^+_r s^-_r'>
      S^{-+}(q) uses <s^-_r s^+_r'> = <s^+_r' s^-_r> (r != r') and 1/2 - <s^z_r> (r = r')
      S(q) = S^zz(q) + (S^{+-}(q) + S^{-+}(q)) / 2.
    """
    N = zz.shape[0]
    mp = pm.T.copy()                     # <s^-_r s^+_r'> = <s^+_r' s^-_r>
    mp[np.arange(N), np.arange(N)] = 0.5 - szv
    out = []
    for q in qs:
        ph = np.exp(1j * (R @ q))
        M = np.outer(ph, np.conj(ph))    # e^{i q.(R_r - R_r')}
        szz = np.real(np.sum(M * zz)) / N
        spm = np.real(np.sum(M * pm)) / N
        smp = np.real(np.sum(M * mp)) / N
        out.append((szz, spm, szz + 0.5 * (spm + smp)))
    return np.array(out)
