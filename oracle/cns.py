"""Combinatorial-number-system basis of the fixed-N_down sector (Sec. 3.1) and
the spin exchange on a bond (Sec. 3.2), written from their definitions.

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
    """Rank of an ascending down-spin tuple: a = 1 + sum_m C(n_m - 1, m) (Eq. (a_of_n))."""
    a = 1
    for m, r in enumerate(n, start=1):
        a += C(r - 1, m)
    return a


def f_bar(a: int, K: int, N: int):
    """The ascending tuple n with F(n) = a (the inverse map of Sec. 3.1).

    a - 1 = sum_m C(n_m - 1, m) with n_1 < ... < n_K is the combinatorial
    number system, whose digits come greedily from the top: n_K - 1 is the
    largest c with C(c, K) <= a - 1, then n_{K-1} - 1 the largest c below it
    with C(c, K-1) <= the remainder, and so on down to m = 1.  (The definition
    also covers the ranks that the search range printed in Alg. 1 cannot
    return, e.g. a = 1 -> (1, ..., K).)
    """
    s = a - 1
    top = N - 1                      # n_m - 1 <= top
    n = [0] * K
    for m in range(K, 0, -1):
        c = top
        while C(c, m) > s:
            c -= 1
        n[m - 1] = c + 1
        s -= C(c, m)
        top = c - 1
    return tuple(n)


def is_down(r: int, n) -> bool:
    """Is site r occupied by a down spin in the tuple n?"""
    return r in n


def hop(n, r: int, rp: int):
    """The exchange term of the bond (r, r') on a state with exactly one end
    down: that down spin moves to the other end -- it is removed and the
    other site inserted, the tuple kept ascending."""
    src, dst = (r, rp) if r in n else (rp, r)
    return tuple(sorted([x for x in n if x != src] + [dst]))


def to0(n):
    """1-based tuple -> 0-based tuple."""
    return tuple(r - 1 for r in n)


def from0(c):
    return tuple(r + 1 for r in c)
