"""Parity tolerances derived from the arithmetic.

The oracle forms a row of H.v as Alg. 9 does: it runs over all N_b bonds and
accumulates a term per bond (the Ising diagonal +-Jz/4 v_a, and Jxy/2 v_a' for
exchanged bonds), so its running sum reaches |E_FM| |v| with E_FM = sum Jz/4
and its rounding error is at most N_b eps (sum|Jz|/4 + max|Jxy|) max|v|.  The
kernel adds <= 6K terms of the same size, a smaller error.  The tolerance is
four times the oracle's bound.
"""
import numpy as np

EPS64 = 2.220446049250313e-16
EPS32 = 1.1920928955078125e-07


def hv_tol(lat, vmax, eps=EPS64):
    scale = np.abs(lat.jz).sum() / 4.0 + np.abs(lat.jxy).max() + np.abs(lat.jz).max()
    return 4.0 * eps * max(lat.n_bonds, 1) * scale * max(vmax, 1e-300)


def hv_tol32(lat, vmax, n_down):
    """float32 rows: the kernel rounds v to float32 (relative eps32) and adds
    <= z*K + 2 float32 terms, each of size <= (|E_FM| + max|J|) max|v|."""
    scale = np.abs(lat.jz).sum() / 4.0 + np.abs(lat.jxy).max() + np.abs(lat.jz).max()
    return 4.0 * EPS32 * (12 * max(n_down, 1) + 2) * scale * vmax
