"""Momentum (translation-symmetry) basis, Sec. 3.3: Alg. 5 (check_state),
Alg. 6 (mk_list), Alg. 7 (representative), Alg. 8 (dense k-block) and Alg. 9
(on-the-fly H.v in the k basis).

The paper writes the chain; the lattice here is Lx x Ly x Lz unit cells of
S sites each, with periodic boundaries and the translation group
Z_Lx x Z_Ly x Z_Lz acting on the cells (S > 1 is the multi-site unit cell the
paper names as future work, Sec. 5).
READING: site r (1-based) has sublattice s and cell coordinates (x, y, z) with
r - 1 = s + S*(x + Lx*(y + Ly*z)) (S = 1: x-fastest as before); translation
number j = 1..N_T (N_T = Lx Ly Lz) is the vector t_j = cell coordinates of
j mod N_T, so j = N_T is the identity, as T^N = 1 on the chain; a
translation keeps the sublattice.  k = 2*pi*(Kx/Lx, Ky/Ly, Kz/Lz) and
k.t = 2*pi*(Kx tx/Lx + Ky ty/Ly + Kz tz/Lz); the orbit normalisation is over
the N_T translations.
"""
from __future__ import annotations

import cmath
import math

import numpy as np

from .cns import C, F, f_bar, is_down, spin_exchange
from .hamiltonian import row_terms


class Geometry:
    def __init__(self, lx: int, ly: int = 1, lz: int = 1, ns: int = 1, basis=None):
        self.lx, self.ly, self.lz, self.ns = lx, ly, lz, ns
        self.NT = lx * ly * lz          # translations
        self.N = ns * self.NT           # sites
        # place s of a cell sits at the cell's coordinates + basis[s] (cell-vector units)
        self.basis = [tuple(map(float, b)) for b in basis] if basis else [(0.0, 0.0, 0.0)] * ns

    def position(self, r: int):
        """1-based site -> position (cell coordinates + the place's offset)."""
        x, y, z = self.coords(r)
        b = self.basis[self.sublattice(r)]
        return x + b[0], y + b[1], z + b[2]

    def coords(self, r: int):
        """1-based site -> cell coordinates (x, y, z)."""
        c = (r - 1) // self.ns
        return c % self.lx, (c // self.lx) % self.ly, c // (self.lx * self.ly)

    def sublattice(self, r: int) -> int:
        return (r - 1) % self.ns

    def site(self, x, y, z, s: int = 0) -> int:
        return 1 + s + self.ns * ((x % self.lx) + self.lx * ((y % self.ly) + self.ly * (z % self.lz)))

    def t(self, j: int):
        """Translation vector of translation number j = 1..N_T (j = N_T: identity)."""
        c = j % self.NT
        return c % self.lx, (c // self.lx) % self.ly, c // (self.lx * self.ly)

    def shift_func(self, n, t):
        """The tuple of T^t|n>: every down spin moves by t (unsorted)."""
        out = []
        for r in n:
            x, y, z = self.coords(r)
            out.append(self.site(x + t[0], y + t[1], z + t[2], self.sublattice(r)))
        return out

    def kdot(self, K, t) -> float:
        return 2.0 * math.pi * (K[0] * t[0] / self.lx + K[1] * t[1] / self.ly + K[2] * t[2] / self.lz)


def insertion_sort(v):
    """Ascending insertion sort (the paper's choice for O(1) lengths, Alg. 5)."""
    v = list(v)
    for i in range(1, len(v)):
        x = v[i]
        j = i - 1
        while j >= 0 and v[j] > x:
            v[j + 1] = v[j]
            j -= 1
        v[j + 1] = x
    return tuple(v)


def check_state(geo: Geometry, a: int, K: int, Kvec) -> float:
    """Alg. 5: N_{a,k} = |c*|^2 N / n_c if a is the minimum rank of its orbit, else 0.

    READING: N_{a,k} is tested against 1e-8 instead of 0, since a vanishing
    character sum is only zero up to rounding in floating point.
    """
    n = f_bar(a, K, geo.N)
    cstar = 0j
    nc = 0
    for j in range(1, geo.NT + 1):
        t = geo.t(j)
        a2 = F(insertion_sort(geo.shift_func(n, t)))
        if a2 < a:
            return 0.0
        if a2 == a:
            cstar += cmath.exp(1j * geo.kdot(Kvec, t))
            nc += 1
    Nak = abs(cstar) ** 2 * geo.NT / nc
    return Nak if Nak > 1e-8 else 0.0


def mk_list(geo: Geometry, K: int, Kvec):
    """Alg. 6: representative ranks sigma (ascending) and R = sqrt(N_{a,k})."""
    sigma, R = [], []
    for a in range(1, C(geo.N, K) + 1):
        Nak = check_state(geo, a, K, Kvec)
        if Nak > 0:
            sigma.append(a)
            R.append(math.sqrt(Nak))
    return sigma, R


def representative(geo: Geometry, a_n: int, K: int):
    """Alg. 7: (min rank over the orbit of a_n, l) with T^{t_l} a_n = rep.
    Ties keep the last j (the printed "<=")."""
    rep = a_n
    ell = geo.NT
    n = f_bar(a_n, K, geo.N)
    for j in range(1, geo.NT + 1):
        a = F(insertion_sort(geo.shift_func(n, geo.t(j))))
        if a <= rep:
            rep, ell = a, j
    return rep, ell


def _bsearch_sorted(sigma, x):
    """(index 1-based, found) of x in ascending sigma (Alg. 2 on the list)."""
    lo, hi = 0, len(sigma)
    while lo < hi:
        mid = (lo + hi) // 2
        if sigma[mid] < x:
            lo = mid + 1
        else:
            hi = mid
    if lo < len(sigma) and sigma[lo] == x:
        return lo + 1, True
    return lo, False


def row_terms_k(geo: Geometry, K: int, bonds, sigma, R, Kvec, alpha: int):
    """Terms of row alpha (1-based) of the k block in the order of Alg. 8/9:
    (diag, [(alpha', coefficient), ...]).

    READING: the printed factor sqrt(R_{alpha'}/R_alpha) with R = sqrt(N_{a,k})
    would be (N'/N)^(1/4); the matrix element of Eq. (hak2) and of the H.v
    equation is sqrt(N_{a'}/N_a) = R_{alpha'}/R_alpha, which is used here.
    The row (pull) element carries e^{+i k.t_l}, as printed in Alg. 8/9.
    """
    n = f_bar(sigma[alpha - 1], K, geo.N)
    diag, offs = row_terms(n, bonds)
    out = []
    for (np_, jhalf) in offs:
        rep, ell = representative(geo, F(np_), K)
        ap, found = _bsearch_sorted(sigma, rep)
        if found:
            coef = jhalf * cmath.exp(1j * geo.kdot(Kvec, geo.t(ell))) * (R[ap - 1] / R[alpha - 1])
            out.append((ap, coef))
    return diag, out


def gen_full_ham_sym_adapt(geo: Geometry, K: int, bonds, sigma, R, Kvec) -> np.ndarray:
    """Alg. 8: dense complex k block (tiny inputs only)."""
    d = len(sigma)
    H = np.zeros((d, d), dtype=np.complex128)
    for alpha in range(1, d + 1):
        diag, offs = row_terms_k(geo, K, bonds, sigma, R, Kvec, alpha)
        H[alpha - 1, alpha - 1] += diag
        for (ap, c) in offs:
            H[alpha - 1, ap - 1] += c
    return H


def ham_to_vec_k(geo: Geometry, K: int, bonds, sigma, R, Kvec, phi: np.ndarray) -> np.ndarray:
    """Alg. 9: psi = H phi in the k basis, row by row on the fly."""
    d = len(sigma)
    psi = np.zeros(d, dtype=np.complex128)
    for alpha in range(1, d + 1):
        diag, offs = row_terms_k(geo, K, bonds, sigma, R, Kvec, alpha)
        acc = diag * phi[alpha - 1]
        for (ap, c) in offs:
            acc += c * phi[ap - 1]
        psi[alpha - 1] = acc
    return psi


def expand_to_u1(geo: Geometry, K: int, sigma, R, Kvec, phi: np.ndarray) -> np.ndarray:
    """The U(1)-basis amplitudes of sum_alpha phi_alpha |sigma_alpha, k>, from the
    definition Eq. (akstate): |a,k> = N_{a,k}^{-1/2} sum_j e^{-i k.t_j} T^j |a>."""
    out = np.zeros(C(geo.N, K), dtype=np.complex128)
    for alpha, a in enumerate(sigma):
        n = f_bar(a, K, geo.N)
        for j in range(1, geo.NT + 1):
            t = geo.t(j)
            b = F(insertion_sort(geo.shift_func(n, t)))
            out[b - 1] += phi[alpha] * cmath.exp(-1j * geo.kdot(Kvec, t)) / R[alpha]
    return out
