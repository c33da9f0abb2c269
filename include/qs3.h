/*
 * qs3.h -- C ABI of the MI355X (gfx950) engine for the S=1/2 XXZ model near
 * saturation, after "Quantum spin solver near saturation: QS^3"
 * (Ueda, Yunoki, Shimokawa; arXiv 2107.00872).
 *
 * Model (Sec. 2.2, Eq. (xxz_hamiltonian)):
 *   H = sum_b [ Jxy_b (s^x_i s^x_j + s^y_i s^y_j) + Jz_b s^z_i s^z_j ] - h sum_i s^z_i,
 * J > 0 antiferromagnetic.  The Zeeman term is a constant in a fixed-N_down
 * sector and is never part of H.v; it enters only the dynamical structure
 * factor as a shift of the poles.
 *
 * States are ascending down-spin site tuples c_1 < ... < c_K (0-based sites,
 * K = N_down) indexed by the combinatorial-number-system rank
 *   rank = sum_m C(c_m, m)  in [0, C(N, K))                (Eq. (a_of_n), minus 1)
 * so a vector of the fixed-N_down ("U(1)") sector is indexed by rank.
 * Momentum sectors (Sec. 3.3) use the states
 *   |a,k> = N_{a,k}^{-1/2} sum_t e^{-i k.t} T^t |a>        (Eq. (akstate))
 * over the representatives a (the minimum rank of each translation orbit)
 * compatible with k, in ascending rank order.  k = 2 pi (Kx/Lx, Ky/Ly, Kz/Lz).
 * Site i has coordinates (x, y, z) with i = x + Lx*(y + Ly*z).
 *
 * Conventions of every entry point:
 *  - return 0 (QS3_OK) or a negative QS3_E* code; nothing throws across the
 *    ABI.  qs3_last_error() gives a message for the calling thread.
 *  - "device" pointers are caller-owned HIP device allocations (for example
 *    torch tensors); the library never frees them.  "host" pointers are read
 *    or written during the call only; host inputs are copied.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Calls that
 *    return host results synchronise with the stream before returning;
 *    qs3_matvec and qs3_sector_start_vector only enqueue work.
 *  - handles are opaque and owned by the library; destroy them in the reverse
 *    order of creation (server, batch/sector, lattice, context).
 *  - one context per host thread; a server is internally synchronised.
 */
#ifndef QS3_H
#define QS3_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define QS3_OK        0
#define QS3_EINVAL   -1   /* bad argument: site id, i == j, N_down out of range, k out
                             of range, N != Lx*Ly*Lz, k requested on a lattice whose
                             bond set is not translation invariant, dtype mismatch */
#define QS3_ENOMEM   -2   /* footprint exceeds the context budget or hipMalloc failed */
#define QS3_ENOCONV  -3   /* solver hit its iteration limit: outputs hold the best
                             estimates and info->converged == 0 */
#define QS3_ENUMERIC -4   /* NaN/Inf or a zero start vector */
#define QS3_EDEVICE  -5   /* a HIP call failed */
#define QS3_EBUSY    -6   /* a server ticket is not finished yet */
#define QS3_ENOTFOUND -7  /* unknown server ticket */
#define QS3_ECANCELED -8  /* the request was cancelled */

/* ---- element types of device vectors ----------------------------------- */
#define QS3_F64  0   /* real float64: fixed-N_down sectors (H is real symmetric) */
#define QS3_F32  1   /* real float32 */
#define QS3_C128 2   /* complex float64 (re, im interleaved): momentum sectors */
#define QS3_C64  3   /* complex float32 */

typedef struct qs3_ctx qs3_ctx;
typedef struct qs3_lattice qs3_lattice;
typedef struct qs3_sector qs3_sector;
typedef struct qs3_batch qs3_batch;
typedef struct qs3_server qs3_server;
typedef struct qs3_pg_sector qs3_pg_sector;

const char *qs3_version(void);
const char *qs3_strerror(int code);
const char *qs3_last_error(void);

/* ---- context ----------------------------------------------------------- */
/* Binds HIP device `device`.  hbm_budget_bytes bounds the device memory the
 * library itself allocates (tables, Krylov workspace); 0 = 90% of the free
 * memory at creation.  Allocations beyond it fail with QS3_ENOMEM. */
int qs3_ctx_create(int device, uint64_t hbm_budget_bytes, qs3_ctx **out);
int qs3_ctx_destroy(qs3_ctx *ctx);
int qs3_ctx_memory(const qs3_ctx *ctx, uint64_t *used_bytes, uint64_t *budget_bytes);
/* How momentum structures built later in this context resolve a hop's target
 * (its representative and the translation that reaches it, Sec. 3.3).  Two
 * optional stores, each built when it fits its limit and a quarter of the
 * unused budget (0 turns a store off):
 *  - a rank -> (representative, translation) table, 8 bytes per rank of
 *    C(N, N_down), at most table_max_bytes (default 16 GiB);
 *  - per-representative hop lists, 8 bytes per (representative, hop slot),
 *    N_down * (largest site degree) slots per representative, resolved once
 *    at build, at most hop_list_max_bytes (default 64 GiB).
 * The batched and single-sector H.v use the hop lists when present, else the
 * table; the other kernels use the table; without a store every hop is
 * canonicalised on the fly with a directory search among the
 * representatives.  Structures already built keep their mode. */
/* Execution schedule of the solvers on this context (graphs off and
 * autotuning on by default; with both measured on the benchmark workloads,
 * graphs changed no solve time by more than 3% -- the cycles are bound by
 * kernel time, not by launches -- and autotuning shortened the 1000-sector
 * batch by 5%):
 *  use_graphs  a thick-restart cycle (the launches of N_M - N_K Lanczos steps,
 *              which are the same at every restart of one solve) is captured
 *              into a HIP graph on its first run and replayed afterwards, on
 *              caller streams that can be captured (not the NULL stream);
 *  autotune    the first batched momentum H.v of each width class (batch size
 *              rounded up to a power of two), element type and hop store
 *              times its schedules -- lanes per row and blocks per CU -- and
 *              keeps the fastest for the lattice's structure.
 * Neither changes results: every schedule sums each sector's hops in the
 * same order, and a replayed cycle runs the captured launches unchanged. */
int qs3_ctx_set_schedule(qs3_ctx *ctx, int use_graphs, int autotune);
int qs3_ctx_set_structure_limits(qs3_ctx *ctx, uint64_t table_max_bytes, uint64_t hop_list_max_bytes);

/* ---- lattice (Sec. 2.2 model; bond list as in the paper's FILExxz) ------ */
/* n_sites = lx*ly*lz (<= 4096).  Bond b couples sites bi[b] != bj[b] (0-based)
 * with exchange jxy[b] and Ising jz[b]; repeated bonds add.  Arrays are host,
 * copied.  The lattice records whether the bond set (with couplings) is
 * invariant under every translation of Z_lx x Z_ly x Z_lz; only then can
 * momentum sectors be built on it. */
int qs3_lattice_create(qs3_ctx *ctx, int lx, int ly, int lz, int n_bonds, const int32_t *bi,
                       const int32_t *bj, const double *jxy, const double *jz,
                       qs3_lattice **out);
/* Unit cells of n_sub sites (1 <= n_sub <= 4; the multi-site unit cell that
 * Sec. 5 names as future work, e.g. kagome 3, honeycomb 2): n_sites = n_sub *
 * lx*ly*lz with site = s + n_sub*(x + lx*(y + ly*z)) for place s of cell
 * (x, y, z).  Translations move whole cells and keep s, so momentum sectors
 * are over the lx*ly*lz cell translations (orbit normalisation N_T s_a with
 * N_T = lx*ly*lz).  Every entry point takes such lattices: momentum-sector
 * correlations are averaged over cell translations per pair of places, and
 * S^a_q uses the sites' positions (qs3_lattice_set_basis) with q = 2 pi
 * (Qx/lx, Qy/ly, Qz/lz), Q taken modulo the lengths.  qs3_lattice_create is
 * this call with n_sub = 1. */
int qs3_lattice_create_cells(qs3_ctx *ctx, int n_sub, int lx, int ly, int lz, int n_bonds,
                             const int32_t *bi, const int32_t *bj, const double *jxy,
                             const double *jz, qs3_lattice **out);
/* Positions of the n_sub places within a cell, in units of the cell vectors
 * (offsets: host, n_sub x 3, copied; default all 0).  Site s + n_sub*(x +
 * lx*(y + ly*z)) sits at (x, y, z) + offsets[s]; qs3_sq uses these positions
 * in e^{-i q.R}. */
int qs3_lattice_set_basis(qs3_lattice *lat, const double *offsets);
int qs3_lattice_destroy(qs3_lattice *lat);
int qs3_lattice_info(const qs3_lattice *lat, int *n_sites, int *translation_invariant);

/* ---- sectors (Sec. 3.1 fixed N_down; Sec. 3.3 momentum) ------------------ */
/* kvec = NULL: the fixed-N_down sector, dimension C(N, K), real vectors
 * (QS3_F64/QS3_F32).  kvec = {Kx, Ky, Kz} with 0 <= K_a < L_a: the momentum
 * sector, complex vectors (QS3_C128/QS3_C64) over its representatives.
 * 0 <= n_down <= min(N, 8); momentum sectors need n_down <= 6.  Building a
 * momentum sector canonicalises every state of the fixed-N_down sector once
 * on the device (the structure is shared by all sectors and batches of the
 * same lattice and n_down). */
int qs3_sector_create(qs3_lattice *lat, int n_down, const int32_t *kvec, qs3_sector **out);
int qs3_sector_destroy(qs3_sector *sec);
int qs3_sector_dim(const qs3_sector *sec, uint64_t *dim);
/* Host copy of the basis: ranks[i] = 0-based rank of the i-th basis state
 * (the representative for momentum sectors, ascending) and stab[i] = size of
 * its stabiliser under translations (1 for fixed-N_down sectors), so that
 * N_{a,k} = N * stab (Alg. 5).  Either pointer may be NULL. */
int qs3_sector_basis(const qs3_sector *sec, uint64_t *ranks, uint32_t *stab);
/* Start vector of the Lanczos iteration (Alg. 10's random_vec): element i is
 * 2u - 1 with u the top 53 bits of SplitMix64(seed, counter) / 2^53, counter
 * = ranks[i] (real) or 2*ranks[i] and 2*ranks[i]+1 (re, im).  v: device. */
int qs3_sector_start_vector(qs3_sector *sec, uint64_t seed, void *v, int dtype, void *stream);

/* w = H v (Alg. 9, matrix free, one output row per gather).  v, w: device,
 * dim elements of `dtype`, not aliased.  QS3_F32/QS3_C64 accumulate each row
 * in float32. */
int qs3_matvec(qs3_sector *sec, const void *v, void *w, int dtype, void *stream);

/* One row of H exactly as the device kernel forms it: the diagonal element
 * and the off-diagonal (column, value) pairs in the order the kernel visits
 * them (down spins ascending, then the site's bonds in bond order).  cols are
 * basis indices; vals is re/im interleaved for momentum sectors.  *nnz may
 * exceed cap (then only cap entries are written).  Host outputs. */
/* The same product as qs3_matvec, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid allocation): it allocates nothing.  A momentum sector whose basis is
 * smaller than the union of representatives is multiplied through two
 * union-layout vectors; qs3_matvec allocates them on the sector's first call,
 * this entry point takes them from one device array of 64 MiB that the
 * library holds on every device it runs on until the process ends.  Sectors
 * of more than 2,097,152 representatives return QS3_EINVAL (nothing is
 * launched); fixed-N_down sectors, and momentum sectors in QS3_C128 whose
 * basis is the whole union, need no scratch.  Every call on a device shares
 * that device's array and leaves its last contents there: calls that overlap
 * on one GPU (two streams, two threads) race, so serialise them.  Same
 * arguments, layouts and results as qs3_matvec (bit for bit). */
int qs3_matvec_noalloc(qs3_sector *sec, const void *v, void *w, int dtype, void *stream);

int qs3_row(qs3_sector *sec, uint64_t row, int cap, int64_t *cols, double *vals, double *diag,
            int *nnz);

/* ---- eigensolver (Sec. 3.7, Alg. 10) ------------------------------------ */
#define QS3_ALG_LANCZOS 0   /* conventional Lanczos, `steps` steps, no restart */
#define QS3_ALG_TRL     1   /* thick-restart Lanczos */
#define QS3_REORTH_NONE    0  /* three-term recurrence only */
#define QS3_REORTH_FULL    1  /* classical Gram-Schmidt against every earlier
                                 vector at every step, a second pass where the
                                 first cancelled more than half the norm */
#define QS3_REORTH_PARTIAL 2  /* plain Lanczos only (thick restart and sectors
                                 small enough for one workgroup run FULL):
                                 Simon's recurrence estimates the overlaps of
                                 each new vector with the earlier ones, and a
                                 Gram-Schmidt pass against all of them runs at
                                 the steps where an estimate exceeds sqrt(eps)
                                 and at the step after (semi-orthogonality) */
#define QS3_PREC_F64    0   /* float64 everywhere */
#define QS3_PREC_F32MV  1   /* float32 matvec (float32 row accumulation), float64
                               recurrence, reorthogonalisation and eigensolves */

typedef struct {
    int alg;            /* QS3_ALG_LANCZOS or QS3_ALG_TRL */
    int nev;            /* wanted number of distinct lowest levels */
    int nk;             /* TRL: kept Ritz vectors N_K (0 = max(nev + 5, 8)) */
    int nm;             /* TRL: Krylov size N_M (0 = max(2 nk, 24)) */
    int max_restarts;   /* TRL: I_M (0 = 2000) */
    int steps;          /* LANCZOS: number of steps (0 = 100) */
    double tol;         /* residual tolerance, relative to the scale below
                           (0 = 1e-10; 1e-6 with QS3_PREC_F32MV) */
    uint64_t seed;      /* start vector seed */
    int precision;      /* QS3_PREC_* */
    int reorth;         /* QS3_REORTH_* (TRL: FULL or PARTIAL, both full) */
} qs3_eigs_opts;

typedef struct {
    int converged;      /* 1 if every wanted level met tol */
    int n_restarts;
    int n_matvec;
    int n_found;        /* distinct levels returned (<= nev) */
    double max_residual;
    double seconds;     /* wall time of the call */
    int width;          /* columns of the launches that ran the last restart
                           (1 for a sector; in a batch the batch size, or fewer
                           once the solver narrowed to the sectors still
                           iterating) */
    int graph_cycles;   /* restart cycles replayed from a captured graph */
} qs3_eigs_info;

/* Lowest `nev` distinct levels (Alg. 10): a Ritz value counts when its
 * residual estimate |beta_m c_{m,i}| <= tol * min(max(1, |e_i|), max(1, w)),
 * w the width of the current Ritz spectrum (a scale that a constant offset of
 * H does not change, so near-degenerate levels are resolved to about tol * w),
 * and values closer than 1e-10 * max(1, |e|) are one level (1e-6 with
 * QS3_PREC_F32MV, whose rounding splits degenerate levels by ~1e-8).  evals: host, nev doubles (unfound =
 * NaN).  evecs: device, dim x nev (vector y at offset y*dim) of the sector's
 * float64 type (QS3_F64 / QS3_C128), or NULL. */
int qs3_eigs(qs3_sector *sec, const qs3_eigs_opts *opts, double *evals, void *evecs,
             qs3_eigs_info *info, void *stream);

/* Plain Lanczos coefficients from v0 (device, float64 type of the sector; or
 * NULL for the seeded start vector), reorth = QS3_REORTH_*: alpha[0..steps-1], beta[0..steps-1]
 * (beta[x] = norm of the (x+2)-th vector before normalisation) and
 * *norm0 = |v0|.  Host outputs.  Stops early at an invariant subspace: *done
 * receives the number of steps taken.  QS3_ENUMERIC when v0 is zero or not
 * finite (or a coefficient turns non-finite); the outputs are then left
 * untouched. */
int qs3_lanczos(qs3_sector *sec, const void *v0, int steps, int precision, int reorth,
                uint64_t seed, double *alpha, double *beta, double *norm0, int *done,
                void *stream);

/* ---- full diagonalisation and thermal averages (Sec. 3.4, Eq. (ens)) ----- */
/* The dense Hamiltonian block of the sector (the matrix of Alg. 4 / Alg. 8),
 * formed on the device from the same hop rules as qs3_matvec: H (device,
 * caller-owned) receives dim x dim elements of the sector's float64 type
 * (QS3_F64 fixed N_down, QS3_C128 momentum), column major (element (i, j) at
 * j*dim + i).  dim <= 46340. */
int qs3_dense(qs3_sector *sec, void *H, void *stream);
/* Every eigenvalue of the sector, ascending (evals: host, dim doubles), and
 * when evecs is not NULL the eigenvectors as its columns (device, dim x dim
 * column major, the sector's float64 type), by the ROCm library's dense
 * Hermitian eigensolver (divide and conquer; the paper uses LAPACK's) on the
 * block of qs3_dense.  dim <= 46340; QS3_ENUMERIC if the solver fails. */
int qs3_full_diag(qs3_sector *sec, double *evals, void *evecs, void *stream);
/* Thermal averages over n levels (Eq. (ens)): energies E (without the field)
 * and S^z_tot values Sz (N/2 - N_down of each level's sector), field h (the
 * Zeeman term -h S^z_tot).  For each inverse temperature beta[t] >= 0: ln Z,
 * energy <H - h S^z_tot>, specific heat beta^2 (<E^2> - <E>^2),
 * magnetisation <S^z_tot>, susceptibility beta (<S^z^2> - <S^z>^2).  Host
 * arrays; outputs may be NULL.  Sectors left out (e.g. large N_down near
 * saturation) are simply absent from the sums. */
int qs3_thermal(uint64_t n, const double *E, const double *Sz, double h, int n_beta, const double *beta,
                double *lnZ, double *energy, double *heat, double *mag, double *chi);

/* ---- observables (Sec. 3.6 and Sec. 4.2) -------------------------------- */
/* <s^z_i> for i = 0..N-1 of the state vec (device, float64 type, any norm;
 * the result is normalised).  In a momentum sector the translation-averaged
 * operator gives M/N on every site. */
int qs3_sz(qs3_sector *sec, const void *vec, double *out, void *stream);
/* <s^z_i s^z_j> and <s^+_i s^-_j> for n_pairs host pairs (i[p], j[p]); in a
 * momentum sector the translation average (1/N_T) sum_t of the pair moved by
 * the cell translation t (Sec. 3.6).  pm is complex (re, im interleaved, 2*n_pairs doubles).  i == j
 * gives 1/4 and 1/2 + <s^z_i>. */
int qs3_sisj(qs3_sector *sec, const void *vec, int n_pairs, const int32_t *i, const int32_t *j,
             double *zz, double *pm, void *stream);
/* Static structure factors at n_q momenta q (host, 3 doubles each):
 * S^zz(q), S^{+-}(q) = <(S^-_q)^+ S^-_q> and S(q) = <S_{-q}.S_q> with
 * S^a_q = N^{-1/2} sum_r e^{-i q.R_r} s^a_r, R_r the site position (cell
 * coordinates plus the place's offset, qs3_lattice_set_basis).  In a
 * momentum sector the sum runs over the translation-averaged correlations
 * with displacements taken within one period, which equals the definition for
 * q on the lattice's momentum grid 2 pi (Kx/lx, Ky/ly, Kz/lz). */
int qs3_sq(qs3_sector *sec, const void *vec, int n_q, const double *q, double *szz,
           double *spm, double *stot, void *stream);
/* psi' = S^-_q phi (Sec. 3.8, Alg. 11) from `from` (N_down = K, momentum k)
 * into `to` (K + 1, momentum k + q), computed as a gather over the rows of
 * `to`.  qvec: host {Qx, Qy, Qz}.  Vectors: device complex float64. */
int qs3_smq(qs3_sector *from, const void *vec_from, qs3_sector *to, const int32_t *qvec,
            void *vec_to, void *stream);

/* The Fourier-transformed spin operators S^a_q = N^{-1/2} sum_r e^{-i q.R_r} s^a_r
 * (Sec. 3.8; the paper's spsmsz = 2, 1, 3). */
#define QS3_OP_SMINUS 0   /* lowers S^z: N_down -> N_down + 1, poles move by +h */
#define QS3_OP_SPLUS  1   /* raises S^z: N_down -> N_down - 1, poles move by -h */
#define QS3_OP_SZ     2   /* N_down unchanged, no field shift */

/* psi' = S^op_q phi from `from` (N_down = K, momentum k) into `to` (K + 1, K - 1
 * or K for op = QS3_OP_SMINUS, QS3_OP_SPLUS, QS3_OP_SZ; momentum k + q), as a
 * gather over the rows of `to` (S^z_q is diagonal in the representatives).
 * Same vector conventions as qs3_smq; QS3_EINVAL when the sectors do not
 * match the operator. */
int qs3_sq_apply(qs3_sector *from, const void *vec_from, qs3_sector *to, int op, const int32_t *qvec,
                 void *vec_to, void *stream);

/* ---- dynamical structure factor (Sec. 3.9, Eq. (cfe)) -------------------- */
typedef struct {
    int steps;          /* Lanczos levels of the continued fraction (0 = 300) */
    double eta;         /* Lorentzian broadening */
    double field;       /* h of the Zeeman term -h S^z_tot: the poles move by +h
                           (S^-), -h (S^+) or 0 (S^z) */
    int precision;      /* QS3_PREC_* */
    int reorth;         /* QS3_REORTH_* */
    int op;             /* QS3_OP_SMINUS (0, default), QS3_OP_SPLUS or QS3_OP_SZ */
    int subtract_trivial; /* S^z only: subtract the trivial q = 0 part
                           (M^2/N) eta / (pi (omega^2 + eta^2)), M = N/2 - K (Sec. 4.2) */
} qs3_dsf_opts;

/* S^a(q, omega) = -(1/pi) Im <psi'| (z - H)^-1 |psi'> with psi' = S^a_q |gs>,
 * a = opts->op, z = omega - shift + E_0 + i eta (shift = +h, -h, 0 for S^-,
 * S^+, S^z), for n_q momenta qvecs (host, 3 ints each), by the continued
 * fraction of the Lanczos coefficients started from psi'/|psi'|; all q run in
 * one batch of target sectors k_0 + q.  gs: momentum sector of the ground
 * state, gs_vec: device complex float64 (any norm).  Outputs (host):
 * S[n_q*n_omega], alpha/beta [n_q*steps], weight[n_q] = |psi'|^2/|gs|^2, the
 * static structure factor <(S^a_q)^+ S^a_q>. */
int qs3_dsf(qs3_sector *gs, const void *gs_vec, double e0, int n_q, const int32_t *qvecs,
            const qs3_dsf_opts *opts, int n_omega, const double *omega, double *S,
            double *alpha, double *beta, double *weight, void *stream);

/* ---- batches of momentum sectors (one persistent launch per H.v) --------- */
/* Every momentum kvecs[3*b..3*b+2] (b < n_sectors) of one lattice and n_down.
 * Batch vectors use the layout [row][sector] over the union of all
 * representatives (rows = union size), complex; entries of representatives
 * incompatible with a sector are ignored on input and zero on output. */
int qs3_batch_create(qs3_lattice *lat, int n_down, int n_sectors, const int32_t *kvecs,
                     qs3_batch **out);
int qs3_batch_destroy(qs3_batch *bat);
/* rows: union size; dims[b]: dimension of sector b.  Host outputs. */
int qs3_batch_dims(const qs3_batch *bat, uint64_t *rows, uint64_t *dims);
/* The schedule of the batch's last batched H.v launch (see
 * qs3_ctx_set_schedule): lanes per representative row and blocks per CU; 0
 * before the first launch and for a batch of one sector (one lane per row). */
int qs3_batch_schedule(const qs3_batch *bat, int *lanes_per_row, int *blocks_per_cu);
/* How the batch's last batched H.v was split: `groups` consecutive launches
 * over at most `sectors_per_group` sectors each (a wide batch of long
 * vectors runs in groups of at most 256 sectors, whose share of v the caches
 * serve better; every sector's sum is the same either way); 0 before the
 * first launch.  Host outputs, either may be null. */
int qs3_batch_groups(const qs3_batch *bat, int *groups, int *sectors_per_group);
int qs3_batch_matvec(qs3_batch *bat, const void *v, void *w, int dtype, void *stream);
/* Per-sector lowest levels (evals[b*nev + y]) and info[b]; every sector runs
 * its own Lanczos state inside the shared launches and stops updating when it
 * converges. */
int qs3_batch_eigs(qs3_batch *bat, const qs3_eigs_opts *opts, double *evals,
                   qs3_eigs_info *info, void *stream);

/* ---- point-group sectors (Sec. 5: point groups beyond translations) ------ */
/* The sector of the space group G = {T^t P_p} (cell translations t, point
 * operations p) in a one-dimensional representation with real characters:
 * chi(T^t P_p) = chars[p] e^{i k.t}, built like the momentum sector of
 * Sec. 3.3 (Eqs. (ak)-(hak2)) with G in place of the translations.  The
 * representative of an orbit is its minimum rank, its norm N_a = |sum over the
 * stabiliser of chi|^2 |G| / |stabiliser|; orbits whose character sum vanishes
 * are not in the sector.  Vectors are real float64 over the representatives.
 *  - lat: translation invariant (point operations may exchange the places of
 *    a cell); 1 <= n_down <= min(N, 6);
 *  - kvec: host, 3 ints, each component 0 or L_a / 2 (k.t = 0 or pi);
 *  - perms: host, n_ops x N (row p: site r -> perms[p*N + r]), 1 <= n_ops <= 48,
 *    row 0 the identity; every row a permutation that keeps the couplings,
 *    conjugates translations into translations with the same e^{i k.t}, and
 *    the rows closed under composition up to translations, no two differing
 *    by a translation;
 *  - chars: host, n_ops values +-1 (chars[0] = 1) that form a representation
 *    of G together with e^{i k.t}.
 * Anything else returns QS3_EINVAL before any device work.  The sector's
 * block is built once on the device (one ELL row of resolved hops per
 * representative); an empty sector (dim 0) is valid. */
int qs3_pg_sector_create(qs3_lattice *lat, int n_down, const int32_t *kvec, int n_ops,
                         const int32_t *perms, const int32_t *chars, qs3_pg_sector **out);
int qs3_pg_sector_destroy(qs3_pg_sector *sec);
int qs3_pg_sector_dim(const qs3_pg_sector *sec, uint64_t *dim);
/* Representatives (0-based ranks, ascending) and N_a, host arrays of dim
 * entries (either may be NULL). */
int qs3_pg_sector_basis(const qs3_pg_sector *sec, uint64_t *ranks, double *norms);
/* v (device, dim float64) := entries uniform in [-1, 1) from seed. */
int qs3_pg_start_vector(qs3_pg_sector *sec, uint64_t seed, double *v, void *stream);
/* w := H v, device float64, dim entries each, no aliasing.  With a single
 * exchange constant the product stages R o v in a buffer of the sector, so
 * products (and solves) on one sector must not overlap. */
int qs3_pg_matvec(qs3_pg_sector *sec, const double *v, double *w, void *stream);
/* The same states in the momentum sector: out (device, complex float64,
 * msec's dim) := sum_a v_a |a, k, chi> in msec's basis, msec the momentum
 * sector of the same lattice handle, n_down and k (else QS3_EINVAL).  Each
 * term of the space-group sum is grouped by point operation: P_p a is a
 * translate T^{-t} u of a representative u, contributing chi(p) e^{i k.t}
 * sqrt(N_T s_u / N_a) to u (Eq. (akstate) for u).  Every momentum-sector
 * observable, S^a_q and S(q, omega) then applies to point-group states. */
int qs3_pg_to_momentum(qs3_pg_sector *sec, const double *v, qs3_sector *msec, void *out, void *stream);
/* As qs3_eigs (QS3_PREC_F64, or QS3_PREC_F32MV: float32 products with the
 * float32 row sums, float64 recurrences); evecs: device, dim x nev (vector y
 * at y*dim), or NULL. */
int qs3_pg_eigs(qs3_pg_sector *sec, const qs3_eigs_opts *opts, double *evals, double *evecs,
                qs3_eigs_info *info, void *stream);

/* ---- serving: continuous batching of solve requests ---------------------- */
typedef struct {
    int max_active;          /* concurrent requests on the device (0 = 8) */
    uint64_t budget_bytes;   /* device memory for admitted requests (0 = ctx budget) */
} qs3_server_opts;

typedef struct {
    int lx, ly, lz, n_bonds;
    const int32_t *bi, *bj;
    const double *jxy, *jz;
    int n_down;
    int use_k;              /* 0: fixed-N_down sector; 1: momentum kvec */
    int32_t kvec[3];
    int nev;
    int precision;          /* QS3_PREC_* */
    uint64_t seed;
} qs3_request;

typedef struct {
    int status;             /* QS3_OK, QS3_ENOCONV, QS3_ENOMEM (not admissible), ... */
    int n_found;
    double evals[16];
    uint64_t dim;
    uint64_t footprint_bytes;
    double t_submit, t_start, t_done;   /* seconds on the server clock */
    int n_matvec;
} qs3_result;

/* A server owns a worker thread that admits queued requests when their device
 * footprint fits the budget and a slot is free, runs every admitted request's
 * Lanczos state on its own stream (their kernels overlap on the device) and
 * retires requests as they converge, so new requests join while others run.
 * A request's result does not depend on what else is running. */
int qs3_server_create(qs3_ctx *ctx, const qs3_server_opts *opts, qs3_server **out);
int qs3_server_destroy(qs3_server *srv);
int qs3_submit(qs3_server *srv, const qs3_request *req, uint64_t *ticket);
/* QS3_OK with the result once done, QS3_EBUSY while queued or running. */
int qs3_poll(qs3_server *srv, uint64_t ticket, qs3_result *out);
int qs3_wait(qs3_server *srv, uint64_t ticket, qs3_result *out);
int qs3_cancel(qs3_server *srv, uint64_t ticket);
double qs3_server_clock(qs3_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* QS3_H */
