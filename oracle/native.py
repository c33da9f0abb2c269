"""ctypes binding of the plain C oracle (oracle/c/qs3_oracle.c).

Test infrastructure only (see the package docstring).  ``build()`` compiles the
C file with gcc and OpenMP into oracle/c/libqs3_oracle.so.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "c", "qs3_oracle.c")
LIB = os.path.join(_HERE, "c", "libqs3_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_GNU_SOURCE", SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


def build_sanitized(out: str) -> str:
    """The same C file under AddressSanitizer and UndefinedBehaviorSanitizer
    (any report aborts the process); loaded in place of the plain build when
    QS3_ORACLE_LIB names it, in a process that preloads the ASan runtime."""
    subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                           "-D_GNU_SOURCE", SRC, "-o", out, "-lm"])
    return out


def lib():
    global _lib
    if _lib is None:
        path = os.environ.get("QS3_ORACLE_LIB") or LIB
        if path == LIB and not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(path)
        P = ctypes.c_void_p
        i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        L.orc_binom.restype = u64
        L.orc_binom.argtypes = [ctypes.c_int, ctypes.c_int]
        L.orc_f_bar.argtypes = [ctypes.c_int, ctypes.c_int, i64, P, P]
        L.orc_F.argtypes = [ctypes.c_int, ctypes.c_int, i64, P, P]
        L.orc_hv_u1.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, P, P, i64, P, P,
                                ctypes.c_int]
        L.orc_row_u1.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, P, u64, P, P, P]
        L.orc_mk_list.restype = i64
        L.orc_mk_list.argtypes = [ctypes.c_int] * 4 + [P, P, P, ctypes.c_int]
        L.orc_representative.argtypes = [ctypes.c_int] * 4 + [i64, P, P, P]
        L.orc_hv_k.argtypes = [ctypes.c_int] * 4 + [P, ctypes.c_int, P, P, P, P, P, P, i64, P, i64,
                                                    P, P, ctypes.c_int]
        L.orc_row_k.argtypes = [ctypes.c_int] * 4 + [P, ctypes.c_int, P, P, P, P, P, P, i64, i64, P,
                                                     P, P]
        L.orc_smq.argtypes = [ctypes.c_int] * 4 + [P, P, P, i64, P, P, P, i64, P, P, ctypes.c_int]
        L.orc_kstruct_build.restype = P
        L.orc_kstruct_build.argtypes = [ctypes.c_int] * 5 + [P, P, P, P, ctypes.c_int]
        L.orc_kstruct_free.argtypes = [P]
        L.orc_kstruct_nrep.restype = i64
        L.orc_kstruct_nrep.argtypes = [P]
        L.orc_kstruct_nhops.restype = i64
        L.orc_kstruct_nhops.argtypes = [P]
        L.orc_kstruct_sector.restype = i64
        L.orc_kstruct_sector.argtypes = [P, P, P, P, P]
        L.orc_kstruct_hv.argtypes = [P, P, P, P, i64, P, P, ctypes.c_int]
        _lib = L
    return _lib


def _ok(rc):
    if rc < 0:
        raise ValueError("oracle: unsupported size (N <= 4096, N_down <= 31)")
    return rc


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


class Bonds:
    """1-based bond arrays (r < r') for the C routines."""

    def __init__(self, bi, bj, jxy, jz):
        r = np.asarray(bi, dtype=np.int64) + 1
        rp = np.asarray(bj, dtype=np.int64) + 1
        if np.any(r == rp):
            raise ValueError("bond with r == r'")
        lo, hi = np.minimum(r, rp), np.maximum(r, rp)
        self.r = np.ascontiguousarray(lo, dtype=np.int32)
        self.rp = np.ascontiguousarray(hi, dtype=np.int32)
        self.jxy = np.ascontiguousarray(jxy, dtype=np.float64)
        self.jz = np.ascontiguousarray(jz, dtype=np.float64)
        self.n = int(self.r.shape[0])

    @classmethod
    def of(cls, lat):
        return cls(lat.bi, lat.bj, lat.jxy, lat.jz)


def binom(n: int, k: int) -> int:
    return int(lib().orc_binom(n, k))


def f_bar(N: int, K: int, a: np.ndarray) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.uint64)
    out = np.zeros((a.shape[0], K), dtype=np.int32)
    _ok(lib().orc_f_bar(N, K, a.shape[0], _p(a), _p(out)))
    return out


def F(N: int, K: int, n: np.ndarray) -> np.ndarray:
    n = np.ascontiguousarray(n, dtype=np.int32)
    out = np.zeros(n.shape[0], dtype=np.uint64)
    _ok(lib().orc_F(N, K, n.shape[0], _p(n), _p(out)))
    return out


def hv_u1(N: int, K: int, bonds: Bonds, phi: np.ndarray, rows=None, nthreads: int = 0):
    """Alg. 9 in the U(1) basis; rows are 1-based ranks (None = all)."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    if rows is None:
        out = np.zeros(binom(N, K))
        _ok(lib().orc_hv_u1(N, K, bonds.n, _p(bonds.r), _p(bonds.rp), _p(bonds.jxy),
                            _p(bonds.jz), None, 0, _p(phi), _p(out), nthreads))
    else:
        rows = np.ascontiguousarray(rows, dtype=np.uint64)
        out = np.zeros(rows.shape[0])
        _ok(lib().orc_hv_u1(N, K, bonds.n, _p(bonds.r), _p(bonds.rp), _p(bonds.jxy),
                            _p(bonds.jz), _p(rows), rows.shape[0], _p(phi), _p(out), nthreads))
    return out


def row_u1(N: int, K: int, bonds: Bonds, a: int):
    """(diag, cols0[], vals[]) of row a (1-based) in bond order."""
    cols = np.zeros(bonds.n, dtype=np.uint64)
    vals = np.zeros(bonds.n)
    dg = ctypes.c_double()
    c = lib().orc_row_u1(N, K, bonds.n, _p(bonds.r), _p(bonds.rp), _p(bonds.jxy), _p(bonds.jz),
                         a, ctypes.byref(dg), _p(cols), _p(vals))
    return dg.value, cols[:c], vals[:c]


def mk_list(dims, K: int, Kvec, nthreads: int = 0):
    """The k sector's representatives (sigma ascending 1-based ranks) and
    R = sqrt(N_{a,k}), from every rank (what Alg. 5/6 compute)."""
    Kv = np.ascontiguousarray(Kvec, dtype=np.int32)
    d = _ok(lib().orc_mk_list(dims[0], dims[1], dims[2], K, _p(Kv), None, None, nthreads))
    sigma = np.zeros(d, dtype=np.uint64)
    R = np.zeros(d)
    lib().orc_mk_list(dims[0], dims[1], dims[2], K, _p(Kv), _p(sigma), _p(R), nthreads)
    return sigma, R


def representative(dims, K: int, a: np.ndarray):
    a = np.ascontiguousarray(a, dtype=np.uint64)
    rep = np.zeros_like(a)
    ell = np.zeros(a.shape[0], dtype=np.int32)
    _ok(lib().orc_representative(dims[0], dims[1], dims[2], K, a.shape[0], _p(a), _p(rep),
                                 _p(ell)))
    return rep, ell


def hv_k(dims, K: int, Kvec, bonds: Bonds, sigma, R, phi, rows=None, nthreads: int = 0):
    """Alg. 9 in the k basis; rows are 1-based sigma indices (None = all)."""
    Kv = np.ascontiguousarray(Kvec, dtype=np.int32)
    sigma = np.ascontiguousarray(sigma, dtype=np.uint64)
    R = np.ascontiguousarray(R, dtype=np.float64)
    phi = np.ascontiguousarray(phi, dtype=np.complex128)
    d = sigma.shape[0]
    if rows is None:
        out = np.zeros(d, dtype=np.complex128)
        rp, nr = None, 0
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        out = np.zeros(rows.shape[0], dtype=np.complex128)
        rp, nr = _p(rows), rows.shape[0]
    _ok(lib().orc_hv_k(dims[0], dims[1], dims[2], K, _p(Kv), bonds.n, _p(bonds.r), _p(bonds.rp),
                       _p(bonds.jxy), _p(bonds.jz), _p(sigma), _p(R), d, rp, nr, _p(phi), _p(out),
                       nthreads))
    return out


def row_k(dims, K: int, Kvec, bonds: Bonds, sigma, R, alpha: int):
    Kv = np.ascontiguousarray(Kvec, dtype=np.int32)
    cols = np.zeros(bonds.n, dtype=np.int64)
    vals = np.zeros(bonds.n, dtype=np.complex128)
    dg = ctypes.c_double()
    c = lib().orc_row_k(dims[0], dims[1], dims[2], K, _p(Kv), bonds.n, _p(bonds.r), _p(bonds.rp),
                        _p(bonds.jxy), _p(bonds.jz), _p(sigma), _p(R), sigma.shape[0], alpha,
                        ctypes.byref(dg), _p(cols), _p(vals))
    return dg.value, cols[:c], vals[:c]


def smq(dims, K: int, Kvec, sigma, R, phi, sigma1, R1, Qvec, nthreads: int = 0):
    Kv = np.ascontiguousarray(Kvec, dtype=np.int32)
    Qv = np.ascontiguousarray(Qvec, dtype=np.int32)
    phi = np.ascontiguousarray(phi, dtype=np.complex128)
    out = np.zeros(sigma1.shape[0], dtype=np.complex128)
    _ok(lib().orc_smq(dims[0], dims[1], dims[2], K, _p(Kv), _p(sigma), _p(R), sigma.shape[0],
                      _p(phi), _p(sigma1), _p(R1), sigma1.shape[0], _p(Qv), _p(out), nthreads))
    return out


class KStruct:
    """The cached-structure variant: every orbit representative of (lattice,
    N_down) with its stabiliser and its row's hops resolved once (target
    representative and translation, by the search over all translations),
    reused for every momentum and every H.v.  ``sector(K)`` gives a momentum
    sector (positions, 1-based ranks, R); ``hv`` applies H in it."""

    def __init__(self, dims, K: int, bonds: Bonds, nthreads: int = 0):
        self.dims, self.K = tuple(dims), K
        self._h = lib().orc_kstruct_build(dims[0], dims[1], dims[2], K, bonds.n, _p(bonds.r),
                                          _p(bonds.rp), _p(bonds.jxy), _p(bonds.jz), nthreads)
        if not self._h:
            raise ValueError("oracle: structure build failed")
        self.nrep = int(lib().orc_kstruct_nrep(self._h))
        self.nhops = int(lib().orc_kstruct_nhops(self._h))

    def sector(self, Kvec):
        Kv = np.ascontiguousarray(Kvec, dtype=np.int32)
        d = int(lib().orc_kstruct_sector(self._h, _p(Kv), None, None, None))
        mem = np.zeros(d, dtype=np.int64)
        sigma = np.zeros(d, dtype=np.uint64)
        R = np.zeros(d)
        lib().orc_kstruct_sector(self._h, _p(Kv), _p(mem), _p(sigma), _p(R))
        return mem, sigma, R

    def hv(self, Kvec, members, R, phi, nthreads: int = 0):
        Kv = np.ascontiguousarray(Kvec, dtype=np.int32)
        members = np.ascontiguousarray(members, dtype=np.int64)
        R = np.ascontiguousarray(R, dtype=np.float64)
        phi = np.ascontiguousarray(phi, dtype=np.complex128)
        out = np.zeros(members.shape[0], dtype=np.complex128)
        _ok(lib().orc_kstruct_hv(self._h, _p(Kv), _p(members), _p(R), members.shape[0], _p(phi),
                                 _p(out), nthreads))
        return out

    def close(self):
        if self._h:
            lib().orc_kstruct_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
