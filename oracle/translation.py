"""Momentum (translation-symmetry) basis, Sec. 3.3, written from its
definitions: the orbit of a state under translations, its representative
(the minimum rank of the orbit), the normalisation N_{a,k} of Eq. (akstate),
the list of representatives of a sector (what Alg. 5/6 compute), the
representative search of a hop's target (Alg. 7's result), the dense k-block
(Alg. 8) and the row-by-row H.v in the k basis (Alg. 9).

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

from .cns import C, F, f_bar
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


def translate(geo: Geometry, n, t):
    """T^t n as an ascending tuple: every down spin moved by the vector t."""
    return tuple(sorted(geo.shift_func(n, t)))


def orbit(geo: Geometry, n):
    """[(j, rank of T^{t_j} n)] for translation numbers j = 1..N_T."""
    return [(j, F(translate(geo, n, geo.t(j)))) for j in range(1, geo.NT + 1)]


def check_state(geo: Geometry, a: int, K: int, Kvec) -> float:
    """N_{a,k}, the squared norm of the sum in Eq. (akstate) for the orbit
    minimum a: N_T sum over the stabiliser {t: T^t a = a} of e^{ik.t}, which is
    N_T |stab| when e^{ik.t} = 1 on the stabiliser and 0 otherwise; 0 when a is
    not the minimum rank of its orbit (it is then not a representative).

    READING: N_{a,k} is tested against 1e-8 instead of 0, since a vanishing
    character sum is only zero up to rounding in floating point.
    """
    n = f_bar(a, K, geo.N)
    s = 0.0
    for j in range(1, geo.NT + 1):
        b = F(translate(geo, n, geo.t(j)))
        if b < a:                    # a is not its orbit's minimum
            return 0.0
        if b == a:                   # t_j is in the stabiliser
            s += math.cos(geo.kdot(Kvec, geo.t(j)))
    Nak = s * geo.NT
    return Nak if Nak > 1e-8 else 0.0


def mk_list(geo: Geometry, K: int, Kvec):
    """Representative ranks sigma (ascending) of the k sector and R = sqrt(N_{a,k})."""
    sigma, R = [], []
    for a in range(1, C(geo.N, K) + 1):
        Nak = check_state(geo, a, K, Kvec)
        if Nak > 0:
            sigma.append(a)
            R.append(math.sqrt(Nak))
    return sigma, R


def representative(geo: Geometry, a_n: int, K: int):
    """(minimum rank over the orbit of a_n, the first translation number l
    with T^{t_l} a_n = that minimum).  READING: any translation reaching the
    minimum would do; they give the same phase for a compatible k."""
    orb = orbit(geo, f_bar(a_n, K, geo.N))
    rep = min(r for _, r in orb)
    ell = next(j for j, r in orb if r == rep)
    return rep, ell


def _bsearch_sorted(sigma, x):
    """(index 1-based, found) of x in the ascending list sigma (the binary
    search of Alg. 9)."""
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
    """Terms of row alpha (1-based) of the k block, bond by bond as Alg. 8/9
    take them: (diag, [(alpha', coefficient), ...]) for the exchanged states
    whose representative is in sigma.

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
            b = F(translate(geo, n, t))
            out[b - 1] += phi[alpha] * cmath.exp(-1j * geo.kdot(Kvec, t)) / R[alpha]
    return out
