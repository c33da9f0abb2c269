"""XXZ Hamiltonian in the fixed-N_down basis (Sec. 3.2; model of Eq. (xxz_hamiltonian)).

H = sum_b { Jxy_b (s^x_r s^x_r' + s^y_r s^y_r') + Jz_b s^z_r s^z_r' };  the Zeeman
term is a constant in a fixed-N_down sector and is left out (Sec. 3.2).
Bonds are given 0-based (as written by workloads.py) and converted to the
paper's 1-based sites here.

READING: J > 0 is antiferromagnetic (the model equation taken literally).
READING: Alg. 4 assigns the off-diagonal element while Alg. 8 adds it; here it
is always added, so a repeated bond entry sums.
READING: a bond with r > r' is swapped to r < r'; r = r' is rejected.
"""
from __future__ import annotations

import numpy as np

from .cns import C, F, f_bar, hop


def bonds_1based(bi, bj, jxy, jz):
    out = []
    for i, j, a, b in zip(bi, bj, jxy, jz):
        r, rp = int(i) + 1, int(j) + 1
        if r == rp:
            raise ValueError("bond with r == r'")
        if r > rp:
            r, rp = rp, r
        out.append((r, rp, float(a), float(b)))
    return out


def row_terms(n, bonds):
    """All terms of row F(n), bond by bond (the row loop of Alg. 4 / Alg. 9):
    returns (diag, [(n', Jxy/2), ...]).  A bond with both ends alike adds
    +Jz/4 to the diagonal; a bond with one end down adds -Jz/4 and the state
    n' in which that down spin has moved to the other end."""
    diag = 0.0
    offs = []
    for (r, rp, jxy, jz) in bonds:
        if (r in n) == (rp in n):
            diag += jz / 4.0
        else:
            diag -= jz / 4.0
            offs.append((hop(n, r, rp), jxy / 2.0))
    return diag, offs


def gen_full_ham(N: int, K: int, bonds) -> np.ndarray:
    """Alg. 4: the dense real symmetric matrix of the sector, H[a-1, a'-1]."""
    dim = C(N, K)
    H = np.zeros((dim, dim))
    for a in range(1, dim + 1):
        n = f_bar(a, K, N)
        diag, offs = row_terms(n, bonds)
        H[a - 1, a - 1] += diag
        for (np_, c) in offs:
            H[a - 1, F(np_) - 1] += c
    return H


def ham_to_vec_u1(N: int, K: int, bonds, phi: np.ndarray) -> np.ndarray:
    """Alg. 9 without translations (sigma = all ranks, R = 1, k = 0): psi = H phi."""
    dim = C(N, K)
    psi = np.zeros(dim, dtype=np.result_type(phi.dtype, np.float64))
    for a in range(1, dim + 1):
        n = f_bar(a, K, N)
        diag, offs = row_terms(n, bonds)
        acc = diag * phi[a - 1]
        for (np_, c) in offs:
            acc = acc + c * phi[F(np_) - 1]
        psi[a - 1] = acc
    return psi


def row_pattern_u1(N: int, K: int, bonds, a: int):
    """Diagonal value and the off-diagonal (column rank, value) pairs of row a,
    in bond order (0-based columns)."""
    n = f_bar(a, K, N)
    diag, offs = row_terms(n, bonds)
    return diag, [(F(np_) - 1, c) for (np_, c) in offs]
