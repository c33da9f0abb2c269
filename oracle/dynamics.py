"""S^alpha_q |phi> for alpha = -, +, z (Sec. 3.8: Alg. 11 for S^-, the same
procedure for S^+ and S^z as the section states) and the continued-fraction
dynamical structure factor (Sec. 3.9, Eq. (cfe))."""
from __future__ import annotations

import cmath
import math

import numpy as np

from .cns import f_bar, F
from .translation import Geometry, representative, _bsearch_sorted


def _flip(op: str, n, r: int):
    """The state and matrix element of s^op_r |n> (op = '-', '+', 'z'): s^- puts a
    down spin at an up site r, s^+ removes the down spin at r, s^z multiplies by
    1/2 - [r down].  Returns (tuple, c) or None when s^op_r |n> = 0."""
    down = r in n
    if op == "-":
        return None if down else (tuple(sorted(n + (r,))), 1.0)
    if op == "+":
        return (tuple(x for x in n if x != r), 1.0) if down else None
    return n, (-0.5 if down else 0.5)


def n_down_after(op: str, K: int) -> int:
    return K + 1 if op == "-" else (K - 1 if op == "+" else K)


def sq_to_vec(geo: Geometry, K: int, sigma, R, Kvec, phi, sigma1, R1, Qvec, op: str = "-"):
    """psi' = S^op_q phi from the (N_down = K, k) sector into the (K', k + q) sector
    (K' = K + 1, K - 1, K for op = '-', '+', 'z'), as the scatter of Alg. 11 over
    sites r and rows alpha: every term s^op_r |sigma_alpha> = c |b> lands on the
    representative of b with the element c sqrt(N'_beta / (N_alpha N))
    e^{-i(q.R_r + (k+q).t_l)}.

    READING: the printed factor sqrt(R'_beta / (R_alpha N)) with R = sqrt(N_{a,k})
    is the same garble as in Alg. 8/9; the derivation after Eq. (sq_phi) gives
    sqrt(N'_beta / (N_alpha N)) = R'_beta / (R_alpha sqrt(N)), used here.
    The site phase is e^{-i q.R_r} with R_r the position of site r (site 1 at
    the origin; with several sites per cell, the cell's coordinates plus the
    place's offset, and q = 2 pi (Qx/Lx, Qy/Ly, Qz/Lz) for the given integers);
    k + q is taken index-wise modulo (Lx, Ly, Lz).  The element's N is the
    number of sites (the N_T of the two orbit normalisations cancel).
    """
    K1 = n_down_after(op, K)
    d1 = len(sigma1)
    out = np.zeros(d1, dtype=np.complex128)
    kq = tuple(Kvec[i] + Qvec[i] for i in range(3))
    sqN = math.sqrt(geo.N)
    for r in range(1, geo.N + 1):
        Rr = geo.position(r)
        for alpha, a in enumerate(sigma):
            n = f_bar(a, K, geo.N)
            fl = _flip(op, n, r)
            if fl is None:
                continue
            n2, c = fl
            b = F(n2)
            rep, ell = representative(geo, b, K1)
            bi, found = _bsearch_sorted(sigma1, rep)
            if not found:
                continue
            ph = cmath.exp(-1j * (geo.kdot(Qvec, Rr) + geo.kdot(kq, geo.t(ell))))
            out[bi - 1] += c * (R1[bi - 1] / (R[alpha] * sqN)) * ph * phi[alpha]
    return out


def smq_to_vec(geo: Geometry, K: int, sigma, R, Kvec, phi, sigma1, R1, Qvec):
    """Alg. 11: psi' = S^-_q phi from the (N_down = K, k) sector into the
    (K + 1, k + q) sector."""
    return sq_to_vec(geo, K, sigma, R, Kvec, phi, sigma1, R1, Qvec, "-")


def sq_u1(N: int, K: int, pos: np.ndarray, q: np.ndarray, phi_u1: np.ndarray, op: str = "-") -> np.ndarray:
    """S^op_q = N^{-1/2} sum_r e^{-i q.R_r} s^op_r applied to U(1) amplitudes (the
    definition, no translation machinery); op = '-', '+', 'z'."""
    from .observables import all_tuples
    from .cns import C
    out = np.zeros(C(N, n_down_after(op, K)), dtype=np.complex128)
    for a, n in enumerate(all_tuples(N, K)):
        if phi_u1[a] == 0:
            continue
        for r in range(1, N + 1):
            if op == "-":
                if r in n:
                    continue
                n2, c = tuple(sorted(n + (r,))), 1.0
            elif op == "+":
                if r not in n:
                    continue
                n2, c = tuple(x for x in n if x != r), 1.0
            else:
                n2, c = n, (-0.5 if r in n else 0.5)
            out[F(n2) - 1] += c * cmath.exp(-1j * float(pos[r - 1] @ q)) * phi_u1[a] / math.sqrt(N)
    return out


def smq_u1(N: int, K: int, pos: np.ndarray, q: np.ndarray, phi_u1: np.ndarray) -> np.ndarray:
    """S^-_q applied to U(1) amplitudes (the definition)."""
    return sq_u1(N, K, pos, q, phi_u1, "-")


def zeeman_shift(op: str, h: float) -> float:
    """Energy a field h adds to the poles of S^op: the Zeeman term -h S^z_tot
    changes by +h when S^- lowers S^z_tot by one, by -h for S^+, 0 for S^z."""
    return h if op == "-" else (-h if op == "+" else 0.0)


def trivial_sz(omega: np.ndarray, eta: float, M: float, N: int) -> np.ndarray:
    """The trivial q = 0 longitudinal component subtracted in Sec. 4.2:
    (M^2 / N) eta / (pi (omega^2 + eta^2)), M = S^z_tot of the ground state."""
    return (M * M / N) * eta / (math.pi * (omega ** 2 + eta ** 2))


def continued_fraction(alpha, beta, weight: float, omega: np.ndarray, e0: float,
                       eta: float, h: float = 0.0, op: str = "-") -> np.ndarray:
    """Eq. (cfe): S(omega) = -(1/pi) Im[ weight / (z - a_1 - b_1^2/(z - a_2 - ...)) ],
    evaluated from the innermost level outwards with alpha[0:m], beta[0:m-1].

    READING: z = omega + E_0 + i eta (the printed "omega - E_0" contradicts the
    resolvent (omega - H + E_0 + i eta)^-1 the section starts from), and with a
    field h the poles move by the Zeeman change of the operator:
    z = omega - zeeman_shift(op, h) + E_0 + i eta.
    """
    m = len(alpha)
    z = omega - zeeman_shift(op, h) + e0 + 1j * eta
    g = np.zeros_like(z)
    for i in range(m - 1, -1, -1):
        tail = beta[i] ** 2 * g if i < m - 1 else 0.0
        g = 1.0 / (z - alpha[i] - tail)
    return -np.imag(weight * g) / math.pi
