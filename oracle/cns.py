"""Combinatorial-number-system basis of the fixed-N_down sector (Sec. 3.1).

Plain Python integers (exact) and 1-based sites/ranks, as in the paper.
"""
from __future__ import annotations

from math import comb


def C(k: int, m: int) -> int:
    """Binomial coefficient with C(k, m) = 0 for k < m (Sec. 3.1, after Eq. (a_of_n))."""
    if m < 0 or k < m or k < 0:
        return 0
    return comb(k, m)


def F(n) -> int:
    """Rank of an ascending down-spin tuple: a = 1 + sum_m C(r_m - 1, m) (Eq. (a_of_n))."""
    a = 1
    for m, r in enumerate(n, start=1):
        a += C(r - 1, m)
    return a


def binary_search(s0, s, ls: int, le: int):
    """Alg. 2: find p in [ls, le] with s_p <= s0 < s_{p+1} (s_{le+1} = +inf) and
    f = (s_p == s0).  ``s`` is indexed 1-based through ``s(k)`` if callable, else
    ``s[k-1]``.

    READING: the algorithm does not say what p is when s0 < s_ls; here p = ls - 1
    and f = False, which for a down-spin tuple means "insert before n_1".
    """
    get = s if callable(s) else (lambda k: s[k - 1])
    if s0 < get(ls):
        return ls - 1, False
    lo, hi = ls, le          # invariant: get(lo) <= s0, answer in [lo, hi]
    while lo < hi:
        mid = (lo + hi + 1) // 2
        if get(mid) <= s0:
            lo = mid
        else:
            hi = mid - 1
    return lo, get(lo) == s0


def f_bar(a: int, K: int, N: int):
    """Alg. 1: the ascending tuple n with F(n) = a.

    READING: the printed search range {C(k, m)}, 1 <= k <= j cannot return
    j_0 = m - 1, which is needed when the remaining s equals 1 (e.g. a = 1 ->
    n = (1, ..., K)).  The search here runs over k in [m - 1, j - 1] with
    C(m - 1, m) = 0, which always contains the answer.
    """
    if K == 0:
        return ()
    n = [0] * (K + 1)
    s = a
    j = N
    for m in range(K, 1, -1):
        j0, _ = binary_search(s - 1, lambda k: C(k, m), m - 1, j - 1)
        j = j0
        n[m] = j0 + 1
        s -= C(j, m)
    n[1] = s
    return tuple(n[1:])


def is_down(r: int, n):
    """(p, f) := binary_search(r, n, 1, N_down) as used in Alg. 4 and Alg. 9."""
    if len(n) == 0:
        return 0, False
    return binary_search(r, n, 1, len(n))


def spin_exchange(r: int, p: int, f: bool, rp: int, pp: int, n):
    """Alg. 3: apply s^+ s^- + s^- s^+ on the bond (r < r') with exactly one end down.

    f = False: r is up and r' = n_{p'} is down; r is inserted after n_p and n_{p'}
    removed.  f = True: r = n_p is down and r' is up; n_p is removed and r' is
    inserted after n_{p'}.
    READING: the printed f = True branch inserts "r"; the down spin moves from r
    to r', so r' is inserted.
    """
    assert r < rp
    n = list(n)
    if not f:
        out = n[:p] + [r] + n[p:pp - 1] + n[pp:]
    else:
        out = n[:p - 1] + n[p:pp] + [rp] + n[pp:]
    return tuple(out)


def to0(n):
    """1-based tuple -> 0-based tuple."""
    return tuple(r - 1 for r in n)


def from0(c):
    return tuple(r + 1 for r in c)
