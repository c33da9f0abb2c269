"""Lanczos and thick-restart Lanczos (Sec. 3.7, Alg. 10), float64/complex128.

``matvec`` is any callable x -> H x.  diag_tri / diag use numpy's LAPACK-backed
eigh as the library step the paper names (DSTEV-like / ZHEEV-like).
"""
from __future__ import annotations

import numpy as np


def _dot(x, y):
    return np.vdot(x, y)


def mgs(Psi, ncols: int, w):
    """Modified Gram-Schmidt of w against columns 0..ncols-1 of Psi (Alg. 10's
    reorthogonalization, "for example, with the modified Gram-Schmidt procedure")."""
    for j in range(ncols):
        w = w - _dot(Psi[:, j], w) * Psi[:, j]
    return w


def lanczos(matvec, psi1, n_steps: int, reorth: bool = True, reorth_passes: int = 1):
    """Alg. 10, first part (conventional Lanczos): returns (alpha[0:m], beta[0:m],
    Psi[:, 0:m+1]) with beta[x-1] = |psi_{x+1}| as in the algorithm (1-based x).

    Stops early (m < n_steps) if beta vanishes (invariant subspace found)."""
    d = psi1.shape[0]
    dtype = np.result_type(psi1.dtype, np.float64)
    Psi = np.zeros((d, n_steps + 1), dtype=dtype, order="F")   # columns contiguous
    alpha = np.zeros(n_steps)
    beta = np.zeros(n_steps)
    beta_prev = np.sqrt(np.real(_dot(psi1, psi1)))          # beta_0
    Psi[:, 0] = psi1
    for x in range(n_steps):
        Psi[:, x] = Psi[:, x] / beta_prev
        v = matvec(Psi[:, x])
        alpha[x] = np.real(_dot(Psi[:, x], v))
        w = v - alpha[x] * Psi[:, x]
        if x > 0:
            w = w - beta[x - 1] * Psi[:, x - 1]
        if reorth:
            for _ in range(reorth_passes):
                w = mgs(Psi, x + 1, w)
        beta[x] = np.sqrt(np.real(_dot(w, w)))
        Psi[:, x + 1] = w
        beta_prev = beta[x]
        if beta[x] <= 1e-14 * max(1.0, abs(alpha[x])):
            return alpha[:x + 1], beta[:x + 1], Psi[:, :x + 2]
    Psi[:, n_steps] = Psi[:, n_steps] / beta_prev
    return alpha, beta, Psi


def diag_tri(alpha, beta):
    """Eigenpairs (ascending) of the real symmetric tridiagonal matrix with diagonal
    alpha and off-diagonal beta[0:m-1]."""
    m = len(alpha)
    T = np.diag(alpha) + np.diag(beta[:m - 1], 1) + np.diag(beta[:m - 1], -1)
    return np.linalg.eigh(T)


def lowest_distinct(values, n: int, cluster_rel: float = 1e-10, residuals=None,
                    res_rel: float = 1e-8):
    """READING (degenerate levels): a single-start Krylov space holds one vector per
    eigenspace in exact arithmetic, while rounding lets partner copies of
    degenerate levels emerge slowly.  "The n lowest eigenvalues" are therefore
    the n lowest distinct levels among the converged Ritz values: a Ritz value
    counts when its residual estimate |beta_m c_{m,i}| <= res_rel * max(1, |e_i|)
    (when residuals are given), and values within cluster_rel * max(1, |E|) are
    one level (1e-10: levels closer than the accuracy asked of an eigenvalue
    cannot be told apart by it)."""
    vals = np.asarray(values, dtype=np.float64)
    order = np.argsort(vals)
    out = []
    for i in order:
        v = vals[i]
        if residuals is not None and abs(residuals[i]) > res_rel * max(1.0, abs(v)):
            continue
        if out and abs(v - out[-1]) <= cluster_rel * max(1.0, abs(v)):
            continue
        out.append(float(v))
        if len(out) == n:
            break
    return out


def ritz(alpha, beta):
    """Ritz values of the tridiagonal T and their residual estimates
    |beta_m c_{m,i}| (beta_m = beta[-1], the norm of the next Lanczos vector)."""
    e, Cm = diag_tri(alpha, beta)
    return e, np.abs(beta[len(alpha) - 1] * Cm[-1, :]), Cm


def trl(matvec, psi1, NK: int, NM: int, IM: int, eps: float, reorth_passes: int = 1):
    """Alg. 10, thick-restart Lanczos.  Returns (e[0:NK], Psi[:, 0:NK], n_restarts,
    converged).

    Convergence is the paper's: max_y |e'_y / e_y - 1| < eps over the lowest NK
    Ritz values of two successive restarts.  READING: when e_y == 0 the absolute
    change |e'_y - e_y| is used instead of the ratio.
    """
    d = psi1.shape[0]
    dtype = np.result_type(psi1.dtype, np.float64)
    alpha, beta, Psi = lanczos(matvec, psi1, NM, reorth=True, reorth_passes=reorth_passes)
    if len(alpha) < NM:          # the Krylov space closed before NM steps: exact
        e, Cm = diag_tri(alpha, beta)
        k = min(NK, len(e))
        return e[:k], Psi[:, :len(alpha)] @ Cm[:, :k], 0, True
    alpha = alpha.copy()
    beta = beta.copy()
    e, Cm = diag_tri(alpha, beta)
    Psi = Psi.astype(dtype)
    eprev = None
    for I in range(1, IM + 1):
        # Ritz vectors: psi_y := Psi c_y for y <= NK
        PsiK = Psi[:, :NM] @ Cm[:, :NK]
        Psi[:, :NK] = PsiK
        if I > 1:
            ratio = []
            for y in range(NK):
                if e[y] != 0.0:
                    ratio.append(abs(eprev[y] / e[y] - 1.0))
                else:
                    ratio.append(abs(eprev[y] - e[y]))
            if max(ratio) < eps:
                return e[:NK], Psi[:, :NK], I - 1, True
        eprev = e[:NK].copy()
        # arrowhead couplings and the residual vector as psi_{NK+1}
        bcoup = beta[NM - 1] * Cm[NM - 1, :NK]
        alpha[:NK] = e[:NK]
        Psi[:, NK] = Psi[:, NM]
        # lines 6-7 with x = NK+1
        x = NK
        v = matvec(Psi[:, x])
        alpha[x] = np.real(_dot(Psi[:, x], v))
        v = v - Psi[:, :NK] @ bcoup
        w = v - alpha[x] * Psi[:, x]
        for _ in range(reorth_passes):
            w = mgs(Psi, x + 1, w)
        beta[x] = np.sqrt(np.real(_dot(w, w)))
        Psi[:, x + 1] = w
        # lines 4-12 from x = NK+2
        for x in range(NK + 1, NM):
            Psi[:, x] = Psi[:, x] / beta[x - 1]
            v = matvec(Psi[:, x])
            alpha[x] = np.real(_dot(Psi[:, x], v))
            w = v - alpha[x] * Psi[:, x] - beta[x - 1] * Psi[:, x - 1]
            for _ in range(reorth_passes):
                w = mgs(Psi, x + 1, w)
            beta[x] = np.sqrt(np.real(_dot(w, w)))
            Psi[:, x + 1] = w
        Psi[:, NM] = Psi[:, NM] / beta[NM - 1]
        T = np.zeros((NM, NM))
        T[np.arange(NM), np.arange(NM)] = alpha[:NM]
        T[:NK, NK] = bcoup
        T[NK, :NK] = bcoup
        for z in range(NK, NM - 1):
            T[z, z + 1] = beta[z]
            T[z + 1, z] = beta[z]
        e, Cm = np.linalg.eigh(T)
    PsiK = Psi[:, :NM] @ Cm[:, :NK]
    return e[:NK], PsiK, IM, False
