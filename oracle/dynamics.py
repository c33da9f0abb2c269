"""S^-_q |phi> (Sec. 3.8, Alg. 11) and the continued-fraction dynamical structure
factor (Sec. 3.9, Eq. (cfe))."""
from __future__ import annotations

import cmath
import math

import numpy as np

from .cns import f_bar, F, is_down
from .translation import Geometry, representative, _bsearch_sorted


def smq_to_vec(geo: Geometry, K: int, sigma, R, Kvec, phi, sigma1, R1, Qvec):
    """Alg. 11: psi' = S^-_q phi from the (N_down = K, k) sector into the
    (K + 1, k + q) sector, as a scatter over sites r and rows alpha.

    READING: the printed factor sqrt(R'_beta / (R_alpha N)) with R = sqrt(N_{a,k})
    is the same garble as in Alg. 8/9; the derivation after Eq. (sq_phi) gives
    sqrt(N'_beta / (N_alpha N)) = R'_beta / (R_alpha sqrt(N)), used here.
    The site phase is e^{-i q.R_r} with R_r the coordinates of site r (site 1 at
    the origin); k + q is taken index-wise modulo (Lx, Ly, Lz).
    """
    d1 = len(sigma1)
    out = np.zeros(d1, dtype=np.complex128)
    kq = tuple(Kvec[i] + Qvec[i] for i in range(3))
    sqN = math.sqrt(geo.N)
    for r in range(1, geo.N + 1):
        Rr = geo.coords(r)
        for alpha, a in enumerate(sigma):
            n = f_bar(a, K, geo.N)
            p, f = is_down(r, n)
            if f:
                continue
            n2 = n[:p] + (r,) + n[p:]
            b = F(n2)
            rep, ell = representative(geo, b, K + 1)
            bi, found = _bsearch_sorted(sigma1, rep)
            if not found:
                continue
            ph = cmath.exp(-1j * (geo.kdot(Qvec, Rr) + geo.kdot(kq, geo.t(ell))))
            out[bi - 1] += (R1[bi - 1] / (R[alpha] * sqN)) * ph * phi[alpha]
    return out


def smq_u1(N: int, K: int, pos: np.ndarray, q: np.ndarray, phi_u1: np.ndarray) -> np.ndarray:
    """S^-_q = N^{-1/2} sum_r e^{-i q.R_r} s^-_r applied to U(1) amplitudes (the
    definition, no translation machinery)."""
    from .observables import all_tuples
    from .cns import C
    out = np.zeros(C(N, K + 1), dtype=np.complex128)
    for a, n in enumerate(all_tuples(N, K)):
        if phi_u1[a] == 0:
            continue
        for r in range(1, N + 1):
            if r in n:
                continue
            n2 = tuple(sorted(n + (r,)))
            out[F(n2) - 1] += cmath.exp(-1j * float(pos[r - 1] @ q)) * phi_u1[a] / math.sqrt(N)
    return out


def continued_fraction(alpha, beta, weight: float, omega: np.ndarray, e0: float,
                       eta: float, h: float = 0.0) -> np.ndarray:
    """Eq. (cfe): S(omega) = -(1/pi) Im[ weight / (z - a_1 - b_1^2/(z - a_2 - ...)) ],
    evaluated from the innermost level outwards with alpha[0:m], beta[0:m-1].

    READING: z = omega + E_0 + i eta (the printed "omega - E_0" contradicts the
    resolvent (omega - H + E_0 + i eta)^-1 the section starts from), and with a
    field h the S^- poles move by +h: z = omega - h + E_0 + i eta.
    """
    m = len(alpha)
    z = omega - h + e0 + 1j * eta
    g = np.zeros_like(z)
    for i in range(m - 1, -1, -1):
        tail = beta[i] ** 2 * g if i < m - 1 else 0.0
        g = 1.0 / (z - alpha[i] - tail)
    return -np.imag(weight * g) / math.pi
