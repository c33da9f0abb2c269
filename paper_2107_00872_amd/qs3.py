"""Python binding of libqs3 (include/qs3.h): argument marshalling only.

Every computation runs in the HIP library; torch supplies device memory and
streams.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqs3.so")

QS3_OK, QS3_EINVAL, QS3_ENOMEM, QS3_ENOCONV, QS3_ENUMERIC, QS3_EDEVICE = 0, -1, -2, -3, -4, -5
QS3_EBUSY, QS3_ENOTFOUND, QS3_ECANCELED = -6, -7, -8
F64, F32, C128, C64 = 0, 1, 2, 3
ALG_LANCZOS, ALG_TRL = 0, 1
REORTH_NONE, REORTH_FULL, REORTH_PARTIAL = 0, 1, 2
OP_SMINUS, OP_SPLUS, OP_SZ = 0, 1, 2
PREC_F64, PREC_F32MV = 0, 1

P = ctypes.c_void_p
i32, u64, dbl = ctypes.c_int32, ctypes.c_uint64, ctypes.c_double


class EigsOpts(ctypes.Structure):
    _fields_ = [("alg", ctypes.c_int), ("nev", ctypes.c_int), ("nk", ctypes.c_int),
                ("nm", ctypes.c_int), ("max_restarts", ctypes.c_int), ("steps", ctypes.c_int),
                ("tol", dbl), ("seed", u64), ("precision", ctypes.c_int), ("reorth", ctypes.c_int)]


class EigsInfo(ctypes.Structure):
    _fields_ = [("converged", ctypes.c_int), ("n_restarts", ctypes.c_int), ("n_matvec", ctypes.c_int),
                ("n_found", ctypes.c_int), ("max_residual", dbl), ("seconds", dbl),
                ("width", ctypes.c_int), ("graph_cycles", ctypes.c_int)]


class DsfOpts(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int), ("eta", dbl), ("field", dbl), ("precision", ctypes.c_int),
                ("reorth", ctypes.c_int), ("op", ctypes.c_int), ("subtract_trivial", ctypes.c_int)]


class ServerOpts(ctypes.Structure):
    _fields_ = [("max_active", ctypes.c_int), ("budget_bytes", u64)]


class Request(ctypes.Structure):
    _fields_ = [("lx", ctypes.c_int), ("ly", ctypes.c_int), ("lz", ctypes.c_int), ("n_bonds", ctypes.c_int),
                ("bi", P), ("bj", P), ("jxy", P), ("jz", P), ("n_down", ctypes.c_int),
                ("use_k", ctypes.c_int), ("kvec", i32 * 3), ("nev", ctypes.c_int),
                ("precision", ctypes.c_int), ("seed", u64)]


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("n_found", ctypes.c_int), ("evals", dbl * 16), ("dim", u64),
                ("footprint_bytes", u64), ("t_submit", dbl), ("t_start", dbl), ("t_done", dbl),
                ("n_matvec", ctypes.c_int)]


# (name, restype, argtypes) of every entry point of include/qs3.h
SIGNATURES = [
    ("qs3_version", ctypes.c_char_p, []),
    ("qs3_strerror", ctypes.c_char_p, [ctypes.c_int]),
    ("qs3_last_error", ctypes.c_char_p, []),
    ("qs3_ctx_create", ctypes.c_int, [ctypes.c_int, u64, P]),
    ("qs3_ctx_destroy", ctypes.c_int, [P]),
    ("qs3_ctx_memory", ctypes.c_int, [P, P, P]),
    ("qs3_ctx_set_structure_limits", ctypes.c_int, [P, u64, u64]),
    ("qs3_ctx_set_schedule", ctypes.c_int, [P, ctypes.c_int, ctypes.c_int]),
    ("qs3_lattice_create", ctypes.c_int, [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, P, P]),
    ("qs3_lattice_create_cells", ctypes.c_int,
     [P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P, P, P, P]),
    ("qs3_lattice_destroy", ctypes.c_int, [P]),
    ("qs3_lattice_set_basis", ctypes.c_int, [P, P]),
    ("qs3_lattice_info", ctypes.c_int, [P, P, P]),
    ("qs3_sector_create", ctypes.c_int, [P, ctypes.c_int, P, P]),
    ("qs3_sector_destroy", ctypes.c_int, [P]),
    ("qs3_sector_dim", ctypes.c_int, [P, P]),
    ("qs3_sector_basis", ctypes.c_int, [P, P, P]),
    ("qs3_sector_start_vector", ctypes.c_int, [P, u64, P, ctypes.c_int, P]),
    ("qs3_matvec", ctypes.c_int, [P, P, P, ctypes.c_int, P]),
    ("qs3_matvec_noalloc", ctypes.c_int, [P, P, P, ctypes.c_int, P]),
    ("qs3_row", ctypes.c_int, [P, u64, ctypes.c_int, P, P, P, P]),
    ("qs3_eigs", ctypes.c_int, [P, P, P, P, P, P]),
    ("qs3_lanczos", ctypes.c_int, [P, P, ctypes.c_int, ctypes.c_int, ctypes.c_int, u64, P, P, P, P, P]),
    ("qs3_dense", ctypes.c_int, [P, P, P]),
    ("qs3_full_diag", ctypes.c_int, [P, P, P, P]),
    ("qs3_thermal", ctypes.c_int, [u64, P, P, dbl, ctypes.c_int, P, P, P, P, P, P]),
    ("qs3_sz", ctypes.c_int, [P, P, P, P]),
    ("qs3_sisj", ctypes.c_int, [P, P, ctypes.c_int, P, P, P, P, P]),
    ("qs3_sq", ctypes.c_int, [P, P, ctypes.c_int, P, P, P, P, P]),
    ("qs3_smq", ctypes.c_int, [P, P, P, P, P, P]),
    ("qs3_sq_apply", ctypes.c_int, [P, P, P, ctypes.c_int, P, P, P]),
    ("qs3_dsf", ctypes.c_int, [P, P, dbl, ctypes.c_int, P, P, ctypes.c_int, P, P, P, P, P, P]),
    ("qs3_batch_create", ctypes.c_int, [P, ctypes.c_int, ctypes.c_int, P, P]),
    ("qs3_batch_destroy", ctypes.c_int, [P]),
    ("qs3_batch_dims", ctypes.c_int, [P, P, P]),
    ("qs3_batch_schedule", ctypes.c_int, [P, P, P]),
    ("qs3_batch_groups", ctypes.c_int, [P, P, P]),
    ("qs3_batch_matvec", ctypes.c_int, [P, P, P, ctypes.c_int, P]),
    ("qs3_batch_eigs", ctypes.c_int, [P, P, P, P, P]),
    ("qs3_server_create", ctypes.c_int, [P, P, P]),
    ("qs3_server_destroy", ctypes.c_int, [P]),
    ("qs3_submit", ctypes.c_int, [P, P, P]),
    ("qs3_poll", ctypes.c_int, [P, u64, P]),
    ("qs3_wait", ctypes.c_int, [P, u64, P]),
    ("qs3_cancel", ctypes.c_int, [P, u64]),
    ("qs3_server_clock", dbl, [P]),
    ("qs3_pg_sector_create", ctypes.c_int, [P, ctypes.c_int, P, ctypes.c_int, P, P, P]),
    ("qs3_pg_sector_destroy", ctypes.c_int, [P]),
    ("qs3_pg_sector_dim", ctypes.c_int, [P, P]),
    ("qs3_pg_sector_basis", ctypes.c_int, [P, P, P]),
    ("qs3_pg_start_vector", ctypes.c_int, [P, u64, P, P]),
    ("qs3_pg_matvec", ctypes.c_int, [P, P, P, P]),
    ("qs3_pg_eigs", ctypes.c_int, [P, P, P, P, P, P]),
    ("qs3_pg_to_momentum", ctypes.c_int, [P, P, P, P, P]),
]

_lib = None


def lib():
    """The loaded libqs3 (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libqs3.so not found at {LIB_PATH}: run __graft_entry__.build() "
                              "(or python paper_2107_00872_amd/build.py) first")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class QS3Error(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (code {code})")
        self.code = code


def check(rc: int, allow=(QS3_OK,)):
    if rc in allow:
        return rc
    msg = lib().qs3_last_error().decode() or lib().qs3_strerror(rc).decode()
    raise QS3Error(rc, msg)


def _ptr(t):
    """Raw pointer of a torch tensor or numpy array (None -> NULL)."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return ctypes.c_void_p(t.data_ptr())
    return t.ctypes.data_as(ctypes.c_void_p)


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(stream)


def _dtype_code(t):
    import torch
    return {torch.float64: F64, torch.float32: F32, torch.complex128: C128, torch.complex64: C64}[t.dtype]


class Context:
    def __init__(self, device: int = 0, budget_bytes: int = 0):
        h = ctypes.c_void_p()
        check(lib().qs3_ctx_create(device, budget_bytes, ctypes.byref(h)))
        self.h = h
        self.device = device

    def set_structure_limits(self, table_max_bytes: int, hop_list_max_bytes: int):
        """Momentum structures built later use a rank table up to
        table_max_bytes, else hop lists up to hop_list_max_bytes, else
        canonicalise on the fly (0 turns a store off)."""
        check(lib().qs3_ctx_set_structure_limits(self.h, int(table_max_bytes), int(hop_list_max_bytes)))

    def set_schedule(self, use_graphs: bool = True, autotune: bool = True):
        """Graph replay of restart cycles and autotuned batched H.v schedules
        (results do not depend on either)."""
        check(lib().qs3_ctx_set_schedule(self.h, int(use_graphs), int(autotune)))

    def memory(self):
        u, b = u64(), u64()
        check(lib().qs3_ctx_memory(self.h, ctypes.byref(u), ctypes.byref(b)))
        return u.value, b.value

    def close(self):
        if self.h:
            lib().qs3_ctx_destroy(self.h)
            self.h = None


class Lattice:
    def __init__(self, ctx: Context, lx, ly, lz, bi, bj, jxy, jz, ns: int = 1):
        self.ctx = ctx
        self.dims = (int(lx), int(ly), int(lz))
        self.ns = int(ns)
        self._bi = np.ascontiguousarray(bi, dtype=np.int32)
        self._bj = np.ascontiguousarray(bj, dtype=np.int32)
        self._jxy = np.ascontiguousarray(jxy, dtype=np.float64)
        self._jz = np.ascontiguousarray(jz, dtype=np.float64)
        h = ctypes.c_void_p()
        check(lib().qs3_lattice_create_cells(ctx.h, self.ns, self.dims[0], self.dims[1], self.dims[2],
                                             len(self._bi), _ptr(self._bi), _ptr(self._bj), _ptr(self._jxy),
                                             _ptr(self._jz), ctypes.byref(h)))
        self.h = h

    @classmethod
    def of(cls, ctx: Context, lat):
        """From a workloads.Lattice."""
        L = cls(ctx, lat.lx, lat.ly, lat.lz, lat.bi, lat.bj, lat.jxy, lat.jz, getattr(lat, "ns", 1))
        if getattr(lat, "basis", ()):
            L.set_basis(lat.basis)
        return L

    def set_basis(self, offsets):
        """Positions of the places in a cell (ns x 3, cell-vector units)."""
        self._basis = np.ascontiguousarray(offsets, dtype=np.float64).reshape(self.ns, 3)
        check(lib().qs3_lattice_set_basis(self.h, _ptr(self._basis)))

    def info(self):
        n, ti = ctypes.c_int(), ctypes.c_int()
        check(lib().qs3_lattice_info(self.h, ctypes.byref(n), ctypes.byref(ti)))
        return n.value, bool(ti.value)

    def close(self):
        if self.h:
            lib().qs3_lattice_destroy(self.h)
            self.h = None


@dataclass
class EigsResult:
    evals: np.ndarray
    info: EigsInfo
    status: int


def make_opts(alg=ALG_TRL, nev=1, nk=0, nm=0, max_restarts=0, steps=0, tol=0.0, seed=1,
              precision=PREC_F64, reorth=1):
    return EigsOpts(alg, nev, nk, nm, max_restarts, steps, tol, seed, precision, reorth)


class Sector:
    def __init__(self, lattice: Lattice, n_down: int, k=None):
        self.lattice = lattice
        self.n_down = n_down
        self.k = None if k is None else tuple(int(x) for x in k)
        h = ctypes.c_void_p()
        kv = None if k is None else np.array(self.k, dtype=np.int32)
        check(lib().qs3_sector_create(lattice.h, n_down, _ptr(kv), ctypes.byref(h)))
        self.h = h
        d = u64()
        check(lib().qs3_sector_dim(self.h, ctypes.byref(d)))
        self.dim = d.value

    @property
    def is_complex(self):
        return self.k is not None

    def basis(self):
        r = np.zeros(self.dim, dtype=np.uint64)
        s = np.zeros(self.dim, dtype=np.uint32)
        check(lib().qs3_sector_basis(self.h, _ptr(r), _ptr(s)))
        return r, s

    def start_vector(self, seed, out, stream=None):
        check(lib().qs3_sector_start_vector(self.h, seed, _ptr(out), _dtype_code(out), _stream(stream)))
        return out

    def matvec(self, v, w, stream=None):
        check(lib().qs3_matvec(self.h, _ptr(v), _ptr(w), _dtype_code(v), _stream(stream)))
        return w

    def row(self, row: int, cap: int = 512):
        cols = np.zeros(cap, dtype=np.int64)
        vals = np.zeros(2 * cap if self.is_complex else cap)
        dg, nnz = ctypes.c_double(), ctypes.c_int()
        check(lib().qs3_row(self.h, row, cap, _ptr(cols), _ptr(vals), ctypes.byref(dg), ctypes.byref(nnz)))
        n = min(nnz.value, cap)
        v = vals[:2 * n].view(np.complex128) if self.is_complex else vals[:n]
        return dg.value, cols[:n], v

    def eigs(self, nev=1, evecs=None, stream=None, **kw) -> EigsResult:
        o = make_opts(nev=nev, **kw)
        ev = np.zeros(max(nev, 1))
        info = EigsInfo()
        rc = lib().qs3_eigs(self.h, ctypes.byref(o), _ptr(ev), _ptr(evecs), ctypes.byref(info),
                            _stream(stream))
        check(rc, allow=(QS3_OK, QS3_ENOCONV))
        return EigsResult(ev[:nev], info, rc)

    def dense(self, out=None, stream=None):
        """The dense block, column major (a torch tensor dim x dim: out[j, i] = H[i, j])."""
        import torch
        if out is None:
            dt = torch.complex128 if self.is_complex else torch.float64
            out = torch.empty(self.dim, self.dim, dtype=dt, device="cuda")
        check(lib().qs3_dense(self.h, _ptr(out), _stream(stream)))
        return out

    def full_diag(self, evecs=None, stream=None):
        """All eigenvalues (ascending); eigenvectors into evecs (dim x dim column
        major: evecs[j] is eigenvector j) when given."""
        ev = np.zeros(max(self.dim, 1))
        check(lib().qs3_full_diag(self.h, _ptr(ev), _ptr(evecs), _stream(stream)))
        return ev[:self.dim]

    def lanczos(self, steps, v0=None, precision=PREC_F64, reorth=1, seed=1, stream=None):
        a = np.zeros(steps)
        b = np.zeros(steps)
        n0 = ctypes.c_double()
        done = ctypes.c_int()
        check(lib().qs3_lanczos(self.h, _ptr(v0), steps, precision, reorth, seed, _ptr(a), _ptr(b),
                                ctypes.byref(n0), ctypes.byref(done), _stream(stream)))
        return a, b, n0.value, done.value

    def sz(self, vec, stream=None):
        N = self.lattice.info()[0]
        out = np.zeros(N)
        check(lib().qs3_sz(self.h, _ptr(vec), _ptr(out), _stream(stream)))
        return out

    def sisj(self, vec, pairs_i, pairs_j, stream=None):
        pi = np.ascontiguousarray(pairs_i, dtype=np.int32)
        pj = np.ascontiguousarray(pairs_j, dtype=np.int32)
        zz = np.zeros(len(pi))
        pm = np.zeros(2 * len(pi))
        check(lib().qs3_sisj(self.h, _ptr(vec), len(pi), _ptr(pi), _ptr(pj), _ptr(zz), _ptr(pm),
                             _stream(stream)))
        return zz, pm.view(np.complex128)

    def sq(self, vec, qs, stream=None):
        q = np.ascontiguousarray(qs, dtype=np.float64).reshape(-1, 3)
        n = q.shape[0]
        szz, spm, stot = np.zeros(n), np.zeros(n), np.zeros(n)
        check(lib().qs3_sq(self.h, _ptr(vec), n, _ptr(q), _ptr(szz), _ptr(spm), _ptr(stot),
                           _stream(stream)))
        return szz, spm, stot

    def smq(self, vec, to: "Sector", qvec, out, stream=None):
        qv = np.array(qvec, dtype=np.int32)
        check(lib().qs3_smq(self.h, _ptr(vec), to.h, _ptr(qv), _ptr(out), _stream(stream)))
        return out

    def sq_apply(self, vec, to: "Sector", op, qvec, out, stream=None):
        """out = S^op_q vec in the sector `to` (op = OP_SMINUS, OP_SPLUS, OP_SZ)."""
        qv = np.array(qvec, dtype=np.int32)
        check(lib().qs3_sq_apply(self.h, _ptr(vec), to.h, op, _ptr(qv), _ptr(out), _stream(stream)))
        return out

    def dsf(self, gs_vec, e0, qvecs, omega, steps=300, eta=0.05, field=0.0, precision=PREC_F64,
            reorth=1, op=OP_SMINUS, subtract_trivial=False, stream=None):
        qv = np.ascontiguousarray(qvecs, dtype=np.int32).reshape(-1, 3)
        om = np.ascontiguousarray(omega, dtype=np.float64)
        nq, nw = qv.shape[0], om.shape[0]
        S = np.zeros(nq * nw)
        a = np.zeros(nq * steps)
        b = np.zeros(nq * steps)
        w = np.zeros(nq)
        o = DsfOpts(steps, eta, field, precision, reorth, op, 1 if subtract_trivial else 0)
        check(lib().qs3_dsf(self.h, _ptr(gs_vec), e0, nq, _ptr(qv), ctypes.byref(o), nw, _ptr(om),
                            _ptr(S), _ptr(a), _ptr(b), _ptr(w), _stream(stream)))
        return S.reshape(nq, nw), a.reshape(nq, steps), b.reshape(nq, steps), w

    def close(self):
        if self.h:
            lib().qs3_sector_destroy(self.h)
            self.h = None


class Batch:
    def __init__(self, lattice: Lattice, n_down: int, kvecs):
        self.lattice = lattice
        self.n_down = n_down
        self.kvecs = np.ascontiguousarray(kvecs, dtype=np.int32).reshape(-1, 3)
        self.B = self.kvecs.shape[0]
        h = ctypes.c_void_p()
        check(lib().qs3_batch_create(lattice.h, n_down, self.B, _ptr(self.kvecs), ctypes.byref(h)))
        self.h = h
        rows = u64()
        dims = np.zeros(self.B, dtype=np.uint64)
        check(lib().qs3_batch_dims(self.h, ctypes.byref(rows), _ptr(dims)))
        self.rows = rows.value
        self.dims = dims

    def schedule(self):
        """(lanes per row, blocks per CU) of the last batched H.v launch."""
        g, b = ctypes.c_int(), ctypes.c_int()
        check(lib().qs3_batch_schedule(self.h, ctypes.byref(g), ctypes.byref(b)))
        return g.value, b.value

    def groups(self):
        """(launches, sectors per launch) of the last batched H.v."""
        g, b = ctypes.c_int(), ctypes.c_int()
        check(lib().qs3_batch_groups(self.h, ctypes.byref(g), ctypes.byref(b)))
        return g.value, b.value

    def matvec(self, v, w, stream=None):
        check(lib().qs3_batch_matvec(self.h, _ptr(v), _ptr(w), _dtype_code(v), _stream(stream)))
        return w

    def eigs(self, nev=1, stream=None, **kw):
        o = make_opts(nev=nev, **kw)
        ev = np.zeros(self.B * nev)
        infos = (EigsInfo * self.B)()
        rc = lib().qs3_batch_eigs(self.h, ctypes.byref(o), _ptr(ev), infos, _stream(stream))
        check(rc, allow=(QS3_OK, QS3_ENOCONV))
        return ev.reshape(self.B, nev), list(infos), rc

    def close(self):
        if self.h:
            lib().qs3_batch_destroy(self.h)
            self.h = None


class PGSector:
    """Sector of translations x point operations in a one-dimensional real
    representation: perms (n_ops x N site permutations, row 0 the identity),
    chars (+-1 per operation), k with every component 0 or L/2."""

    def __init__(self, lattice: Lattice, n_down: int, k, perms, chars):
        self.lattice = lattice
        self.n_down = n_down
        self.k = tuple(int(x) for x in k)
        self._perms = np.ascontiguousarray(perms, dtype=np.int32)
        self._chars = np.ascontiguousarray(chars, dtype=np.int32)
        kv = np.array(self.k, dtype=np.int32)
        h = ctypes.c_void_p()
        check(lib().qs3_pg_sector_create(lattice.h, n_down, _ptr(kv), self._perms.shape[0], _ptr(self._perms),
                                         _ptr(self._chars), ctypes.byref(h)))
        self.h = h
        d = u64()
        check(lib().qs3_pg_sector_dim(self.h, ctypes.byref(d)))
        self.dim = d.value

    def basis(self):
        """(0-based ranks, N_a) of the representatives."""
        r = np.zeros(self.dim, dtype=np.uint64)
        n = np.zeros(self.dim)
        check(lib().qs3_pg_sector_basis(self.h, _ptr(r), _ptr(n)))
        return r, n

    def start_vector(self, seed, out, stream=None):
        check(lib().qs3_pg_start_vector(self.h, seed, _ptr(out), _stream(stream)))
        return out

    def matvec(self, v, w, stream=None):
        check(lib().qs3_pg_matvec(self.h, _ptr(v), _ptr(w), _stream(stream)))
        return w

    def eigs(self, nev=1, evecs=None, stream=None, **kw) -> EigsResult:
        o = make_opts(nev=nev, **kw)
        ev = np.zeros(max(nev, 1))
        info = EigsInfo()
        rc = lib().qs3_pg_eigs(self.h, ctypes.byref(o), _ptr(ev), _ptr(evecs), ctypes.byref(info),
                               _stream(stream))
        check(rc, allow=(QS3_OK, QS3_ENOCONV))
        return EigsResult(ev[:nev], info, rc)

    def to_momentum(self, v, msec, out=None, stream=None):
        """The vector in the momentum sector msec (same lattice, n_down, k)."""
        import torch
        if out is None:
            out = torch.empty(msec.dim, dtype=torch.complex128, device="cuda")
        check(lib().qs3_pg_to_momentum(self.h, _ptr(v), msec.h, _ptr(out), _stream(stream)))
        return out

    def close(self):
        if self.h:
            lib().qs3_pg_sector_destroy(self.h)
            self.h = None


class Server:
    def __init__(self, ctx: Context, max_active=8, budget_bytes=0):
        self.ctx = ctx
        o = ServerOpts(max_active, budget_bytes)
        h = ctypes.c_void_p()
        check(lib().qs3_server_create(ctx.h, ctypes.byref(o), ctypes.byref(h)))
        self.h = h
        self._keep = {}

    def submit(self, lat, n_down, k=None, nev=3, precision=PREC_F64, seed=1):
        bi = np.ascontiguousarray(lat.bi, dtype=np.int32)
        bj = np.ascontiguousarray(lat.bj, dtype=np.int32)
        jxy = np.ascontiguousarray(lat.jxy, dtype=np.float64)
        jz = np.ascontiguousarray(lat.jz, dtype=np.float64)
        kv = (i32 * 3)(*(k if k is not None else (0, 0, 0)))
        r = Request(lat.lx, lat.ly, lat.lz, len(bi), _ptr(bi), _ptr(bj), _ptr(jxy), _ptr(jz), n_down,
                    0 if k is None else 1, kv, nev, precision, seed)
        t = u64()
        check(lib().qs3_submit(self.h, ctypes.byref(r), ctypes.byref(t)))
        return t.value

    def poll(self, ticket):
        r = Result()
        rc = lib().qs3_poll(self.h, ticket, ctypes.byref(r))
        if rc == QS3_EBUSY:
            return None
        check(rc)
        return r

    def wait(self, ticket):
        r = Result()
        check(lib().qs3_wait(self.h, ticket, ctypes.byref(r)))
        return r

    def cancel(self, ticket):
        return lib().qs3_cancel(self.h, ticket)

    def clock(self):
        return lib().qs3_server_clock(self.h)

    def close(self):
        if self.h:
            lib().qs3_server_destroy(self.h)
            self.h = None


def thermal(E, Sz, beta, h=0.0):
    """Thermal averages (Eq. (ens)) of the levels E with S^z_tot values Sz: a dict
    of arrays over beta (lnZ, energy, heat, mag, chi)."""
    E = np.ascontiguousarray(E, dtype=np.float64)
    Sz = np.ascontiguousarray(Sz, dtype=np.float64)
    b = np.ascontiguousarray(np.atleast_1d(beta), dtype=np.float64)
    out = {k: np.zeros(len(b)) for k in ("lnZ", "energy", "heat", "mag", "chi")}
    check(lib().qs3_thermal(len(E), _ptr(E), _ptr(Sz), float(h), len(b), _ptr(b), _ptr(out["lnZ"]),
                            _ptr(out["energy"]), _ptr(out["heat"]), _ptr(out["mag"]), _ptr(out["chi"])))
    return out
