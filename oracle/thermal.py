"""Thermal averages from complete spectra (Sec. 3.4, full diagonalisation;
Eq. (ens)): <A>_beta = sum_nu e^{-beta E_nu} <nu|A|nu> / Z(beta) over every
level nu of every symmetry sector included.

With a field h the Zeeman term -h S^z_tot is diagonal in every sector
(S^z_tot = N/2 - N_down), so a level's energy is E_nu - h S^z_nu.  Computed in
float64 with the lowest energy subtracted before exponentiating (the shift
cancels in every ratio and is added back to ln Z).
"""
from __future__ import annotations

import math

import numpy as np


def thermal(E: np.ndarray, Sz: np.ndarray, beta: np.ndarray, h: float = 0.0):
    """For every inverse temperature beta[t]: ln Z, the energy <H - h S^z>,
    the specific heat beta^2 (<E^2> - <E>^2), the magnetisation <S^z_tot> and
    the susceptibility beta (<S^z^2> - <S^z>^2), from the levels E[nu] (without
    the field) and their S^z_tot Sz[nu]."""
    E = np.asarray(E, dtype=np.float64)
    Sz = np.asarray(Sz, dtype=np.float64)
    Eh = E - h * Sz
    e0 = Eh.min()
    out = {"lnZ": [], "energy": [], "heat": [], "mag": [], "chi": []}
    for b in np.atleast_1d(beta):
        w = np.exp(-b * (Eh - e0))
        Z = w.sum()
        p = w / Z
        em = (p * Eh).sum()
        e2 = (p * Eh * Eh).sum()
        m = (p * Sz).sum()
        m2 = (p * Sz * Sz).sum()
        out["lnZ"].append(math.log(Z) - b * e0)
        out["energy"].append(em)
        out["heat"].append(b * b * (e2 - em * em))
        out["mag"].append(m)
        out["chi"].append(b * (m2 - m * m))
    return {k: np.array(v) for k, v in out.items()}
