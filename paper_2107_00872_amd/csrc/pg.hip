// Point-group sectors: translations combined with point operations (Sec. 5
// names point-group symmetry as future work; the construction is that of
// Sec. 3.3, Eqs. (ak)-(hak2), with the space group G = {T^t P_p} in place of
// the translation group).
//
// Point operations may exchange the places of a unit cell (translations act
// on cells).  Only one-dimensional representations with real characters are
// built: chi(p)
// = +-1 on the point operations and momenta k with e^{i k.t} = +-1 (each
// component 0 or pi), so that chi(T^t P_p) = chi(p) e^{i k.t} and the sector
// is real.  The representative of an orbit is its minimum rank; its norm is
// N_a = |sum_{g in stab(a)} chi(g)|^2 |G| / |stab(a)| and the pull-form
// element between representatives a and b = g(n') is (J/2) chi(g)
// sqrt(N_b / N_a).
//
// Work split: the translation representatives of (lattice, N_down) are the
// existing momentum structure; one kernel classifies each of them under the
// point operations (minimum over P_p followed by the K^D-candidate
// translation canonicalisation), the host keeps those with a non-zero
// character sum, and a second kernel resolves every row's hops once into an
// ELL block (the sectors are |G| times smaller than the fixed-N_down sector,
// so storing the block costs less than canonicalising |P| images per hop in
// every product).  H.v is then one pass over the ELL arrays; with one
// exchange constant the slots shrink to 4 bytes (column and the character's
// sign), the norm ratio sqrt(N_b / N_a) factored into R_b x_b and 1 / R_a
// (R o x staged in a per-sector buffer, so products on one sector must not
// overlap).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <map>
#include <memory>
#include <vector>

#include "qs3_device.h"
#include "qs3_impl.h"
#include "qs3_krylov.h"

using namespace qs3;

struct qs3_pg_sector {
    qs3_lattice *lat = nullptr;
    int K = 0;
    int kv[3] = {0, 0, 0};
    int n_ops = 0;
    uint64_t dim = 0;
    int width = 0;  // ELL slots per row: N_down * most neighbours of a site
    std::shared_ptr<KStructure> ks;
    std::shared_ptr<BinomTable> bt;
    std::vector<uint64_t> h_reps;  // ascending ranks
    std::vector<double> h_norm;    // N_a
    DevBuf perm;   // uint16 [n_ops * N]
    DevBuf chi;    // int32 [n_ops]
    DevBuf reps;   // uint64 [dim]
    DevBuf rnorm;  // double [dim]: sqrt(N_a)
    // ELL block, slot w of row a at w * dim + a.  Uniform exchange (packed):
    // col holds b | sign << 31 (sign of chi(g)), padding 0xffffffff, and
    // H_ab = scale_a * sign * R_b with scale_a = (J/2) / R_a.  Otherwise col
    // holds b (padding a) and val the element.
    bool packed = false;
    DevBuf col;    // uint32 [width * dim]
    DevBuf val;    // double [width * dim] (not packed)
    DevBuf scale;  // double [dim] (packed)
    DevBuf xr;     // double [dim] (packed): R o x of the product in progress
    DevBuf xr32;   // float [dim] (packed): the same for float32 products
    DevBuf diag;   // double [dim]
};

namespace {

struct PgArgs {
    int N, n_ops;
    const uint16_t *perm;
    const int32_t *chi;
    int kpi[3];  // 1 where the momentum component is pi
    Geom g;
};

// e^{i k.t} for k components in {0, pi}
__device__ __forceinline__ int kchar(const PgArgs &P, int tx, int ty, int tz) {
    return ((P.kpi[0] & tx) ^ (P.kpi[1] & ty) ^ (P.kpi[2] & tz)) & 1 ? -1 : 1;
}

// The minimum rank over the G-orbit of the (unsorted) tuple c and an element
// (p, t) with T^t P_p c = that minimum.
template <int K, typename RT>
__device__ __forceinline__ RT pg_canon(const int (&c)[K], const PgArgs &P, const Binom<RT> &Bn, int *bp,
                                       int *btx, int *bty, int *btz) {
    RT best = 0;
    for (int p = 0; p < P.n_ops; ++p) {
        int img[K], can[K];
#pragma unroll
        for (int m = 0; m < K; ++m) img[m] = P.perm[p * P.N + c[m]];
        sortK<K>(img);
        int tx, ty, tz;
        canonicalize<K>(img, P.g, can, tx, ty, tz);
        const RT r = rank_of<K, RT>(can, Bn);
        if (p == 0 || r < best) {
            best = r;
            *bp = p;
            *btx = tx;
            *bty = ty;
            *btz = tz;
        }
    }
    return best;
}

// Per translation representative u: csum = sum over the point operations p
// whose image P_p a is a translate of a of chi(p) e^{i k.t_p} (T^{t_p} P_p a =
// a), nmatch = their number; csum = 0 when a is not the minimum of its
// G-orbit or its translation stabiliser is incompatible with k.
template <int K, typename RT>
__global__ void k_pg_classify(PgArgs P, const RT *binom_g, const uint64_t *__restrict__ treps,
                              const uint16_t *__restrict__ tstab, const int32_t *__restrict__ nt_of,
                              const uint8_t *__restrict__ nt_ok, uint64_t n, int32_t *csum, int32_t *nmatch) {
    const uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    Binom<RT> Bn{binom_g, binom_shift(P.N)};
    const RT R = (RT)treps[u];
    int c[K];
    unrank<K, RT>(R, P.N, Bn, c);
    int cs = 0, nm = 0;
    bool keep = tstab[u] <= 1 || nt_ok[nt_of[u]];
    for (int p = 0; p < P.n_ops && keep; ++p) {
        int img[K], can[K];
#pragma unroll
        for (int m = 0; m < K; ++m) img[m] = P.perm[p * P.N + c[m]];
        sortK<K>(img);
        int tx, ty, tz;
        canonicalize<K>(img, P.g, can, tx, ty, tz);
        const RT r = rank_of<K, RT>(can, Bn);
        if (r < R) keep = false;
        if (r == R) {
            cs += P.chi[p] * kchar(P, tx, ty, tz);
            ++nm;
        }
    }
    csum[u] = keep ? cs : 0;
    nmatch[u] = nm;
}

// Row a of the sector: diagonal and the resolved hops in ELL slots
// (slot w of row a at w * dim + a).
template <int K, typename RT, bool PACKED>
__global__ void k_pg_ell(PgArgs P, LatArgs L, const RT *binom_g, const uint64_t *__restrict__ reps,
                         const double *__restrict__ rnorm, uint64_t dim, int width, uint32_t *col, double *val,
                         double *scale, double *diag) {
    const uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= dim) return;
    Binom<RT> Bn{binom_g, binom_shift(P.N)};
    int c[K];
    unrank<K, RT>((RT)reps[a], P.N, Bn, c);
    const double inv_ra = 1.0 / rnorm[a];
    int w = 0;
    double dz = 0;
    for (int m = 0; m < K; ++m) {
        for (int e = L.ptr[c[m]]; e < L.ptr[c[m] + 1]; ++e) {
            const int j = L.nbr[e];
            bool occ = false;
#pragma unroll
            for (int t = 0; t < K; ++t) occ |= c[t] == j;
            if (occ) continue;
            dz += L.jz_h[e];
            int np[K];
#pragma unroll
            for (int t = 0; t < K; ++t) np[t] = t == m ? j : c[t];
            int p, tx, ty, tz;
            const RT rb = pg_canon<K, RT>(np, P, Bn, &p, &tx, &ty, &tz);
            // the representative's index among the sector's ranks
            uint64_t lo = 0, hi = dim;
            while (lo < hi) {
                const uint64_t mid = (lo + hi) >> 1;
                if (reps[mid] < (uint64_t)rb) lo = mid + 1; else hi = mid;
            }
            if (lo == dim || reps[lo] != (uint64_t)rb) continue;  // its character sum vanishes
            const int sgn = P.chi[p] * kchar(P, tx, ty, tz);
            if (PACKED) {
                col[(uint64_t)w * dim + a] = (uint32_t)lo | (sgn < 0 ? 0x80000000u : 0u);
            } else {
                col[(uint64_t)w * dim + a] = (uint32_t)lo;
                val[(uint64_t)w * dim + a] = L.jxy_h[e] * (double)sgn * rnorm[lo] * inv_ra;
            }
            ++w;
        }
    }
    for (; w < width; ++w) {
        col[(uint64_t)w * dim + a] = PACKED ? 0xffffffffu : (uint32_t)a;
        if (!PACKED) val[(uint64_t)w * dim + a] = 0.0;
    }
    if (PACKED) scale[a] = L.u_jxy_h * inv_ra;
    diag[a] = L.ez4 - dz;
}

// Slots are taken eight at a time: the column loads of a chunk, then its
// gathers, so that each thread keeps eight gathers in flight.
constexpr int PG_CH = 8;

__global__ void k_pg_spmv(const uint32_t *__restrict__ col, const double *__restrict__ val,
                          const double *__restrict__ diag, uint64_t dim, int width,
                          const double *__restrict__ x, double *__restrict__ y) {
    const uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= dim) return;
    double acc = diag[a] * x[a];
    for (int w0 = 0; w0 < width; w0 += PG_CH) {
        uint32_t cb[PG_CH];
        double v[PG_CH], t[PG_CH];
#pragma unroll
        for (int i = 0; i < PG_CH; ++i) {
            const bool in = w0 + i < width;
            cb[i] = in ? col[(uint64_t)(w0 + i) * dim + a] : (uint32_t)a;
            v[i] = in ? val[(uint64_t)(w0 + i) * dim + a] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < PG_CH; ++i) t[i] = x[cb[i]];
#pragma unroll
        for (int i = 0; i < PG_CH; ++i) acc += v[i] * t[i];
    }
    y[a] = acc;
}

// xr = R o x (the packed form gathers R_b x_b in one load)
__global__ void k_pg_prescale(const double *__restrict__ rnorm, uint64_t dim, const double *__restrict__ x,
                              double *__restrict__ xr) {
    const uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a < dim) xr[a] = rnorm[a] * x[a];
}

// Packed form: y_a = diag_a x_a + scale_a * sum over slots of +-xr_b.
__global__ void k_pg_spmv_packed(const uint32_t *__restrict__ col, const double *__restrict__ xr,
                                 const double *__restrict__ scale, const double *__restrict__ diag, uint64_t dim,
                                 int width, const double *__restrict__ x, double *__restrict__ y) {
    const uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= dim) return;
    double acc = 0.0;
    for (int w0 = 0; w0 < width; w0 += PG_CH) {
        uint32_t cb[PG_CH];
        double t[PG_CH];
#pragma unroll
        for (int i = 0; i < PG_CH; ++i) cb[i] = w0 + i < width ? col[(uint64_t)(w0 + i) * dim + a] : 0xffffffffu;
#pragma unroll
        for (int i = 0; i < PG_CH; ++i) t[i] = cb[i] == 0xffffffffu ? 0.0 : xr[cb[i] & 0x7fffffffu];
#pragma unroll
        for (int i = 0; i < PG_CH; ++i) acc += (cb[i] >> 31) ? -t[i] : t[i];
        if (cb[PG_CH - 1] == 0xffffffffu) break;  // slots fill from 0: the rest is padding
    }
    y[a] = diag[a] * x[a] + scale[a] * acc;
}

// The packed product with every slot of a row in flight at once (WM >= width
// slots, padding dropped by a select): the row's column loads, then all of its
// gathers, so a row waits for two memory round trips instead of two per chunk
// of eight.  XT: element type of x and the staged R o x, AT: accumulator (the
// float32 form accumulates in float32); same terms and order as the chunked
// kernels.
template <typename XT, typename AT, int WM>
__global__ __launch_bounds__(256) void k_pg_spmv_packed_w(const uint32_t *__restrict__ col,
                                                          const XT *__restrict__ xr,
                                                          const double *__restrict__ scale,
                                                          const double *__restrict__ diag, uint64_t dim, int width,
                                                          const XT *__restrict__ x, double *__restrict__ y) {
    const uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= dim) return;
    uint32_t cb[WM];
#pragma unroll
    for (int i = 0; i < WM; ++i) cb[i] = i < width ? col[(uint64_t)i * dim + a] : 0xffffffffu;
    XT t[WM];
#pragma unroll
    for (int i = 0; i < WM; ++i) t[i] = xr[cb[i] == 0xffffffffu ? 0u : (cb[i] & 0x7fffffffu)];
    AT acc = 0;
#pragma unroll
    for (int i = 0; i < WM; ++i) {
        const AT v = (AT)t[i];
        acc = cb[i] == 0xffffffffu ? acc : acc + ((cb[i] >> 31) ? -v : v);
    }
    if constexpr (sizeof(AT) == 8) y[a] = diag[a] * (double)x[a] + scale[a] * (double)acc;
    else y[a] = (double)((float)diag[a] * (float)x[a] + (float)scale[a] * (float)acc);
}

// The momentum-sector amplitudes of sum_a x_a |a, k, chi>: grouping the
// space-group sum by point operation, T-sum of P_p a = T^{-t} u is
// e^{i k.t} sqrt(N_T s_u) |u, k>, so u (compact index i) receives
// x_a / sqrt(N_a) * chi(p) e^{i k.t} sqrt(N_T s_u).  Different
// representatives a have disjoint orbits, so every i is written by one thread.
template <int K, typename RT>
__global__ void k_pg_expand(PgArgs P, const RT *binom_g, const uint64_t *__restrict__ reps,
                            const double *__restrict__ rnorm, uint64_t dim, const double *__restrict__ x,
                            const uint64_t *__restrict__ kreps, const uint16_t *__restrict__ kstab,
                            const int64_t *__restrict__ comp2u, uint64_t kdim, double n_t, double2 *out) {
    const uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= dim) return;
    Binom<RT> Bn{binom_g, binom_shift(P.N)};
    int c[K];
    unrank<K, RT>((RT)reps[a], P.N, Bn, c);
    const double xa = x[a] / rnorm[a];
    for (int p = 0; p < P.n_ops; ++p) {
        int img[K], can[K];
#pragma unroll
        for (int m = 0; m < K; ++m) img[m] = P.perm[p * P.N + c[m]];
        sortK<K>(img);
        int tx, ty, tz;
        canonicalize<K>(img, P.g, can, tx, ty, tz);
        const uint64_t r = (uint64_t)rank_of<K, RT>(can, Bn);
        uint64_t lo = 0, hi = kdim;
        while (lo < hi) {
            const uint64_t mid = (lo + hi) >> 1;
            if (kreps[comp2u[mid]] < r) lo = mid + 1; else hi = mid;
        }
        if (lo == kdim || kreps[comp2u[lo]] != r) continue;  // not reached for a valid pair of sectors
        const double sgn = (double)(P.chi[p] * kchar(P, tx, ty, tz));
        out[lo].x += xa * sgn * sqrt(n_t * (double)kstab[comp2u[lo]]);
    }
}

__global__ void k_pg_zero2(uint64_t n, double2 *p) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = make_double2(0.0, 0.0);
}

// float32 products (float64 recurrences around them): float32 inputs, the
// staged R o x and the row sums in float32, the result stored as float64
__global__ void k_pg_prescale_f32(const double *__restrict__ rnorm, uint64_t dim, const float *__restrict__ x,
                                  float *__restrict__ xr) {
    const uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a < dim) xr[a] = (float)(rnorm[a] * (double)x[a]);
}

__global__ void k_pg_spmv_packed_f32(const uint32_t *__restrict__ col, const float *__restrict__ xr,
                                     const double *__restrict__ scale, const double *__restrict__ diag, uint64_t dim,
                                     int width, const float *__restrict__ x, double *__restrict__ y) {
    const uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= dim) return;
    float acc = 0.0f;
    for (int w0 = 0; w0 < width; w0 += PG_CH) {
        uint32_t cb[PG_CH];
        float t[PG_CH];
#pragma unroll
        for (int i = 0; i < PG_CH; ++i) cb[i] = w0 + i < width ? col[(uint64_t)(w0 + i) * dim + a] : 0xffffffffu;
#pragma unroll
        for (int i = 0; i < PG_CH; ++i) t[i] = cb[i] == 0xffffffffu ? 0.0f : xr[cb[i] & 0x7fffffffu];
#pragma unroll
        for (int i = 0; i < PG_CH; ++i) acc += (cb[i] >> 31) ? -t[i] : t[i];
        if (cb[PG_CH - 1] == 0xffffffffu) break;
    }
    y[a] = (double)((float)diag[a] * x[a] + (float)scale[a] * acc);
}

__global__ void k_pg_spmv_f32(const uint32_t *__restrict__ col, const double *__restrict__ val,
                              const double *__restrict__ diag, uint64_t dim, int width,
                              const float *__restrict__ x, double *__restrict__ y) {
    const uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a >= dim) return;
    float acc = (float)diag[a] * x[a];
    for (int w0 = 0; w0 < width; w0 += PG_CH) {
        uint32_t cb[PG_CH];
        float v[PG_CH], t[PG_CH];
#pragma unroll
        for (int i = 0; i < PG_CH; ++i) {
            const bool in = w0 + i < width;
            cb[i] = in ? col[(uint64_t)(w0 + i) * dim + a] : (uint32_t)a;
            v[i] = in ? (float)val[(uint64_t)(w0 + i) * dim + a] : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < PG_CH; ++i) t[i] = x[cb[i]];
#pragma unroll
        for (int i = 0; i < PG_CH; ++i) acc += v[i] * t[i];
    }
    y[a] = (double)acc;
}

__global__ void k_pg_start(const uint64_t *__restrict__ reps, uint64_t dim, uint64_t seed, double *v) {
    const uint64_t a = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (a < dim) v[a] = u01_pm1(splitmix64(seed, reps[a]));
}

inline unsigned blocks_for(uint64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

PgArgs pg_args(const qs3_pg_sector *sec) {
    const qs3_lattice *lat = sec->lat;
    PgArgs P;
    P.N = lat->N;
    P.n_ops = sec->n_ops;
    P.perm = sec->perm.as<uint16_t>();
    P.chi = sec->chi.as<int32_t>();
    for (int d = 0; d < 3; ++d) P.kpi[d] = sec->kv[d] != 0 ? 1 : 0;
    P.g = Geom{lat->lx, lat->ly, lat->lz, lat->lx * lat->ly, lat->d_coords.as<uint32_t>(), lat->ns};
    return P;
}

template <int K, typename RT>
int classify_K(qs3_pg_sector *sec, const DevBuf &nt_ok, DevBuf &cs, DevBuf &nm) {
    const uint64_t n = sec->ks->n_reps;
    if (n == 0) return QS3_OK;
    hipLaunchKernelGGL((k_pg_classify<K, RT>), dim3(blocks_for(n, 256)), dim3(256), 0, 0, pg_args(sec),
                       sec->bt->dev.as<RT>(), sec->ks->reps.as<uint64_t>(), sec->ks->stab.as<uint16_t>(),
                       sec->ks->nt_of.as<int32_t>(), nt_ok.as<uint8_t>(), n, cs.as<int32_t>(),
                       nm.as<int32_t>());
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

template <int K, typename RT>
int ell_K(qs3_pg_sector *sec) {
    if (sec->dim == 0) return QS3_OK;
    auto kern = sec->packed ? k_pg_ell<K, RT, true> : k_pg_ell<K, RT, false>;
    hipLaunchKernelGGL(kern, dim3(blocks_for(sec->dim, 128)), dim3(128), 0, 0, pg_args(sec), lat_args(sec->lat),
                       sec->bt->dev.as<RT>(), sec->reps.as<uint64_t>(), sec->rnorm.as<double>(), sec->dim,
                       sec->width, sec->col.as<uint32_t>(), sec->val.as<double>(), sec->scale.as<double>(),
                       sec->diag.as<double>());
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

template <int K>
int dispatch_rt(qs3_pg_sector *sec, bool ell, const DevBuf *nt_ok, DevBuf *cs, DevBuf *nm) {
    if (sec->bt->wide)
        return ell ? ell_K<K, uint64_t>(sec) : classify_K<K, uint64_t>(sec, *nt_ok, *cs, *nm);
    return ell ? ell_K<K, uint32_t>(sec) : classify_K<K, uint32_t>(sec, *nt_ok, *cs, *nm);
}

struct ExpandArgs {
    const double *x;
    const qs3_sector *msec;
    double2 *out;
    hipStream_t s;
};

template <int K, typename RT>
int expand_K(qs3_pg_sector *sec, const ExpandArgs &E) {
    const KStructure &ks = *E.msec->bat->ks;
    const double n_t = (double)sec->lat->lx * sec->lat->ly * sec->lat->lz;
    hipLaunchKernelGGL((k_pg_expand<K, RT>), dim3(blocks_for(sec->dim, 128)), dim3(128), 0, E.s, pg_args(sec),
                       sec->bt->dev.as<RT>(), sec->reps.as<uint64_t>(), sec->rnorm.as<double>(), sec->dim, E.x,
                       ks.reps.as<uint64_t>(), ks.stab.as<uint16_t>(), E.msec->comp2u.as<int64_t>(), E.msec->dim,
                       n_t, E.out);
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

int dispatch_expand(qs3_pg_sector *sec, const ExpandArgs &E) {
    const bool w = sec->bt->wide;
    switch (sec->K) {
        case 1: return w ? expand_K<1, uint64_t>(sec, E) : expand_K<1, uint32_t>(sec, E);
        case 2: return w ? expand_K<2, uint64_t>(sec, E) : expand_K<2, uint32_t>(sec, E);
        case 3: return w ? expand_K<3, uint64_t>(sec, E) : expand_K<3, uint32_t>(sec, E);
        case 4: return w ? expand_K<4, uint64_t>(sec, E) : expand_K<4, uint32_t>(sec, E);
        case 5: return w ? expand_K<5, uint64_t>(sec, E) : expand_K<5, uint32_t>(sec, E);
        case 6: return w ? expand_K<6, uint64_t>(sec, E) : expand_K<6, uint32_t>(sec, E);
        default: set_error("n_down out of range"); return QS3_EINVAL;
    }
}

int dispatch(qs3_pg_sector *sec, bool ell, const DevBuf *nt_ok = nullptr, DevBuf *cs = nullptr,
             DevBuf *nm = nullptr) {
    switch (sec->K) {
        case 1: return dispatch_rt<1>(sec, ell, nt_ok, cs, nm);
        case 2: return dispatch_rt<2>(sec, ell, nt_ok, cs, nm);
        case 3: return dispatch_rt<3>(sec, ell, nt_ok, cs, nm);
        case 4: return dispatch_rt<4>(sec, ell, nt_ok, cs, nm);
        case 5: return dispatch_rt<5>(sec, ell, nt_ok, cs, nm);
        case 6: return dispatch_rt<6>(sec, ell, nt_ok, cs, nm);
        default: set_error("n_down out of range"); return QS3_EINVAL;
    }
}

// ---- host checks of the group (every one an error, never a kernel fault)

// Site r = s + ns * cell moved by the cell translation t (place s kept).
int shifted_site(const qs3_lattice *lat, int r, const int *t) {
    const int ns = lat->ns, lx = lat->lx, ly = lat->ly, lz = lat->lz;
    const int sub = r % ns, c = r / ns;
    const int x = c % lx, y = (c / lx) % ly, z = c / (lx * ly);
    return sub + ns * ((x + t[0]) % lx + lx * (((y + t[1]) % ly) + ly * ((z + t[2]) % lz)));
}

// The cell translation t whose site map equals f, or -1.
int translation_of(const qs3_lattice *lat, const std::vector<int> &f, int *t) {
    const int N = lat->N, ns = lat->ns, lx = lat->lx, ly = lat->ly;
    if (f[0] % ns != 0) return -1;  // place 0 of cell 0 must stay a place 0
    const int c0 = f[0] / ns;
    const int tt[3] = {c0 % lx, (c0 / lx) % ly, c0 / (lx * ly)};
    for (int r = 0; r < N; ++r)
        if (f[r] != shifted_site(lat, r, tt)) return -1;
    t[0] = tt[0];
    t[1] = tt[1];
    t[2] = tt[2];
    return 0;
}

int kchar_host(const int *kv, const int *t) {
    int s = 0;
    for (int d = 0; d < 3; ++d) s ^= (kv[d] != 0 ? 1 : 0) & t[d];
    return (s & 1) ? -1 : 1;
}

int validate_group(const qs3_lattice *lat, const int *kv, int n_ops, const int32_t *perms,
                   const int32_t *chars) {
    const int N = lat->N;
    std::vector<std::vector<int>> P(n_ops, std::vector<int>(N)), Pinv(n_ops, std::vector<int>(N));
    for (int p = 0; p < n_ops; ++p) {
        QS3_REQUIRE(chars[p] == 1 || chars[p] == -1, QS3_EINVAL, "characters must be +1 or -1");
        std::vector<char> hit(N, 0);
        for (int r = 0; r < N; ++r) {
            const int v = perms[(size_t)p * N + r];
            QS3_REQUIRE(v >= 0 && v < N && !hit[v], QS3_EINVAL, "a point operation is not a permutation of the sites");
            hit[v] = 1;
            P[p][r] = v;
            Pinv[p][v] = r;
        }
    }
    for (int r = 0; r < N; ++r)
        QS3_REQUIRE(P[0][r] == r, QS3_EINVAL, "operation 0 must be the identity");
    QS3_REQUIRE(chars[0] == 1, QS3_EINVAL, "the identity's character must be +1");
    // the couplings are invariant: (i, j) -> (P i, P j) maps the bond sums onto themselves
    std::map<std::pair<int, int>, std::pair<double, double>> bonds;
    double scale = 0;
    for (int i = 0; i < N; ++i)
        for (int e = lat->h_ptr[i]; e < lat->h_ptr[i + 1]; ++e) {
            auto &b = bonds[{i, (int)lat->h_nbr[e]}];
            b.first += lat->h_jxy_h[e];
            b.second += lat->h_jz_h[e];
            scale = std::max(scale, std::max(std::fabs(lat->h_jxy_h[e]), std::fabs(lat->h_jz_h[e])));
        }
    const double tol = 1e-12 * std::max(scale, 1.0);
    for (int p = 1; p < n_ops; ++p)
        for (const auto &b : bonds) {
            auto it = bonds.find({P[p][b.first.first], P[p][b.first.second]});
            QS3_REQUIRE(it != bonds.end() && std::fabs(it->second.first - b.second.first) <= tol &&
                            std::fabs(it->second.second - b.second.second) <= tol,
                        QS3_EINVAL, "a point operation does not leave the couplings invariant");
        }
    // P_p T P_p^{-1} is a translation with the same character (k is invariant)
    const int L[3] = {lat->lx, lat->ly, lat->lz};
    std::vector<int> f(N);
    for (int p = 1; p < n_ops; ++p)
        for (int d = 0; d < 3; ++d) {
            if (L[d] == 1) continue;
            int u[3] = {0, 0, 0};
            u[d] = 1;
            for (int r = 0; r < N; ++r) f[r] = P[p][shifted_site(lat, Pinv[p][r], u)];
            int t[3];
            QS3_REQUIRE(translation_of(lat, f, t) == 0, QS3_EINVAL,
                        "a point operation does not map translations to translations");
            QS3_REQUIRE(kchar_host(kv, t) == kchar_host(kv, u), QS3_EINVAL,
                        "the momentum is not invariant under the point operations");
        }
    // closure: P_p P_q = T^s P_o for exactly one o, and chi(p) chi(q) = chi(o) e^{i k.s}
    for (int p = 0; p < n_ops; ++p)
        for (int q = 0; q < n_ops; ++q) {
            int found = 0;
            for (int o = 0; o < n_ops; ++o) {
                for (int r = 0; r < N; ++r) f[r] = P[p][P[q][Pinv[o][r]]];
                int t[3];
                if (translation_of(lat, f, t) != 0) continue;
                ++found;
                QS3_REQUIRE(chars[p] * chars[q] == chars[o] * kchar_host(kv, t), QS3_EINVAL,
                            "the characters are not a representation of the group");
            }
            QS3_REQUIRE(found == 1, QS3_EINVAL,
                        "the point operations are not closed, or two differ by a translation");
        }
    return QS3_OK;
}

int pg_build(qs3_pg_sector *sec) {
    qs3_lattice *lat = sec->lat;
    qs3_ctx *ctx = lat->ctx;
    QS3_TRY(get_kstruct(lat, sec->K, &sec->ks, 0));
    QS3_TRY(get_binom(lat, sec->K, &sec->bt));
    const KStructure &ks = *sec->ks;
    // translation stabilisers compatible with k
    std::vector<uint8_t> ok(std::max<size_t>(ks.nt_u.size(), 1), 1);
    for (size_t q = 0; q < ks.nt_u.size(); ++q)
        for (int tp : ks.nt_trans[q]) {
            const int t[3] = {tp & 1023, (tp >> 10) & 1023, (tp >> 20) & 1023};
            if (kchar_host(sec->kv, t) != 1) ok[q] = 0;
        }
    DevBuf nt_ok, cs, nm;
    const uint64_t n = ks.n_reps;
    QS3_TRY(nt_ok.alloc(ctx, ok.size()));
    QS3_HIP(hipMemcpy(nt_ok.ptr, ok.data(), ok.size(), hipMemcpyHostToDevice));
    QS3_TRY(cs.alloc(ctx, sizeof(int32_t) * std::max<uint64_t>(n, 1)));
    QS3_TRY(nm.alloc(ctx, sizeof(int32_t) * std::max<uint64_t>(n, 1)));
    QS3_TRY(dispatch(sec, false, &nt_ok, &cs, &nm));
    std::vector<int32_t> hcs(n), hnm(n);
    if (n) {
        QS3_HIP(hipMemcpy(hcs.data(), cs.ptr, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
        QS3_HIP(hipMemcpy(hnm.data(), nm.ptr, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    }
    const double order = (double)sec->n_ops * lat->lx * lat->ly * lat->lz;
    for (uint64_t u = 0; u < n; ++u) {
        if (hcs[u] == 0) continue;
        // cs and nc over G are the stabiliser's size times the point-operation sums
        const double st = ks.h_stab[u];
        sec->h_reps.push_back(ks.h_reps[u]);
        sec->h_norm.push_back(st * (double)hcs[u] * hcs[u] * order / hnm[u]);
    }
    sec->dim = sec->h_reps.size();
    sec->width = sec->K * lat->max_degree;
    QS3_REQUIRE(sec->dim < (1ull << 31), QS3_ENOMEM, "point-group sector too large for 32-bit columns");
    const uint64_t d1 = std::max<uint64_t>(sec->dim, 1);
    QS3_TRY(sec->reps.alloc(ctx, sizeof(uint64_t) * d1));
    QS3_TRY(sec->rnorm.alloc(ctx, sizeof(double) * d1));
    QS3_TRY(sec->diag.alloc(ctx, sizeof(double) * d1));
    sec->packed = lat->uniform;
    QS3_TRY(sec->col.alloc(ctx, sizeof(uint32_t) * d1 * std::max(sec->width, 1)));
    if (sec->packed) {
        QS3_TRY(sec->scale.alloc(ctx, sizeof(double) * d1));
        QS3_TRY(sec->xr.alloc(ctx, sizeof(double) * d1));
        QS3_TRY(sec->xr32.alloc(ctx, sizeof(float) * d1));
    }
    else QS3_TRY(sec->val.alloc(ctx, sizeof(double) * d1 * std::max(sec->width, 1)));
    if (sec->dim) {
        std::vector<double> rn(sec->dim);
        for (uint64_t a = 0; a < sec->dim; ++a) rn[a] = std::sqrt(sec->h_norm[a]);
        QS3_HIP(hipMemcpy(sec->reps.ptr, sec->h_reps.data(), sizeof(uint64_t) * sec->dim, hipMemcpyHostToDevice));
        QS3_HIP(hipMemcpy(sec->rnorm.ptr, rn.data(), sizeof(double) * sec->dim, hipMemcpyHostToDevice));
    }
    QS3_TRY(dispatch(sec, true));
    QS3_HIP(hipDeviceSynchronize());
    return QS3_OK;
}

// the all-slots kernel for widths up to 36 (false: the caller takes the chunked one)
template <typename XT, typename AT>
bool packed_w(qs3_pg_sector *sec, const XT *xr, const XT *x, double *y, hipStream_t s) {
    const dim3 g(blocks_for(sec->dim, 256)), b(256);
    const uint32_t *col = sec->col.as<uint32_t>();
    const double *sc = sec->scale.as<double>(), *dg = sec->diag.as<double>();
    const int w = sec->width;
    if (w <= 8) hipLaunchKernelGGL((k_pg_spmv_packed_w<XT, AT, 8>), g, b, 0, s, col, xr, sc, dg, sec->dim, w, x, y);
    else if (w <= 12) hipLaunchKernelGGL((k_pg_spmv_packed_w<XT, AT, 12>), g, b, 0, s, col, xr, sc, dg, sec->dim, w, x, y);
    else if (w <= 16) hipLaunchKernelGGL((k_pg_spmv_packed_w<XT, AT, 16>), g, b, 0, s, col, xr, sc, dg, sec->dim, w, x, y);
    else if (w <= 24) hipLaunchKernelGGL((k_pg_spmv_packed_w<XT, AT, 24>), g, b, 0, s, col, xr, sc, dg, sec->dim, w, x, y);
    else if (w <= 36) hipLaunchKernelGGL((k_pg_spmv_packed_w<XT, AT, 36>), g, b, 0, s, col, xr, sc, dg, sec->dim, w, x, y);
    else return false;
    return true;
}

int pg_apply(qs3_pg_sector *sec, const double *x, double *y, hipStream_t s) {
    if (sec->dim == 0) return QS3_OK;
    if (sec->packed) {
        hipLaunchKernelGGL(k_pg_prescale, dim3(blocks_for(sec->dim, 256)), dim3(256), 0, s, sec->rnorm.as<double>(),
                           sec->dim, x, sec->xr.as<double>());
        if (!packed_w<double, double>(sec, sec->xr.as<double>(), x, y, s))
            hipLaunchKernelGGL(k_pg_spmv_packed, dim3(blocks_for(sec->dim, 256)), dim3(256), 0, s,
                               sec->col.as<uint32_t>(), sec->xr.as<double>(), sec->scale.as<double>(),
                               sec->diag.as<double>(), sec->dim, sec->width, x, y);
    } else
        hipLaunchKernelGGL(k_pg_spmv, dim3(blocks_for(sec->dim, 256)), dim3(256), 0, s, sec->col.as<uint32_t>(),
                           sec->val.as<double>(), sec->diag.as<double>(), sec->dim, sec->width, x, y);
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

int pg_apply_f32(qs3_pg_sector *sec, const float *x, double *y, hipStream_t s) {
    if (sec->dim == 0) return QS3_OK;
    if (sec->packed) {
        hipLaunchKernelGGL(k_pg_prescale_f32, dim3(blocks_for(sec->dim, 256)), dim3(256), 0, s,
                           sec->rnorm.as<double>(), sec->dim, x, sec->xr32.as<float>());
        if (!packed_w<float, float>(sec, sec->xr32.as<float>(), x, y, s))
            hipLaunchKernelGGL(k_pg_spmv_packed_f32, dim3(blocks_for(sec->dim, 256)), dim3(256), 0, s,
                               sec->col.as<uint32_t>(), sec->xr32.as<float>(), sec->scale.as<double>(),
                               sec->diag.as<double>(), sec->dim, sec->width, x, y);
    } else {
        hipLaunchKernelGGL(k_pg_spmv_f32, dim3(blocks_for(sec->dim, 256)), dim3(256), 0, s, sec->col.as<uint32_t>(),
                           sec->val.as<double>(), sec->diag.as<double>(), sec->dim, sec->width, x, y);
    }
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

struct PGOp : Operator {
    qs3_pg_sector *sec;
    explicit PGOp(qs3_pg_sector *s) : sec(s) {}
    uint64_t rows() const override { return sec->dim; }
    int cols() const override { return 1; }
    bool is_complex() const override { return false; }
    int apply(const double *x, double *y, hipStream_t s) override { return pg_apply(sec, x, y, s); }
    int apply_f32in(const float *x, double *y, hipStream_t s) override { return pg_apply_f32(sec, x, y, s); }
};

}  // namespace

extern "C" {

int qs3_pg_sector_create(qs3_lattice *lat, int n_down, const int32_t *kvec, int n_ops, const int32_t *perms,
                         const int32_t *chars, qs3_pg_sector **out) {
    QS3_REQUIRE(lat && kvec && perms && chars && out, QS3_EINVAL, "NULL argument");
    QS3_REQUIRE(lat->translation_invariant, QS3_EINVAL, "the lattice is not translation invariant");
    QS3_REQUIRE(n_down >= 1 && n_down <= std::min(lat->N, MAX_K_MOM), QS3_EINVAL,
                "point-group sectors need 1 <= n_down <= min(N, 6)");
    QS3_REQUIRE(n_ops >= 1 && n_ops <= 48, QS3_EINVAL, "1 <= n_ops <= 48");
    const int L[3] = {lat->lx, lat->ly, lat->lz};
    for (int d = 0; d < 3; ++d)
        QS3_REQUIRE(kvec[d] >= 0 && kvec[d] < L[d] && (kvec[d] == 0 || 2 * kvec[d] == L[d]), QS3_EINVAL,
                    "point-group sectors need every momentum component 0 or pi");
    (void)hipSetDevice(lat->ctx->device);
    int kv[3] = {kvec[0], kvec[1], kvec[2]};
    QS3_TRY(validate_group(lat, kv, n_ops, perms, chars));
    auto sec = std::make_unique<qs3_pg_sector>();
    sec->lat = lat;
    sec->K = n_down;
    sec->n_ops = n_ops;
    for (int d = 0; d < 3; ++d) sec->kv[d] = kv[d];
    qs3_ctx *ctx = lat->ctx;
    std::vector<uint16_t> p16((size_t)n_ops * lat->N);
    for (size_t i = 0; i < p16.size(); ++i) p16[i] = (uint16_t)perms[i];
    QS3_TRY(sec->perm.alloc(ctx, sizeof(uint16_t) * p16.size()));
    QS3_TRY(sec->chi.alloc(ctx, sizeof(int32_t) * n_ops));
    QS3_HIP(hipMemcpy(sec->perm.ptr, p16.data(), sizeof(uint16_t) * p16.size(), hipMemcpyHostToDevice));
    QS3_HIP(hipMemcpy(sec->chi.ptr, chars, sizeof(int32_t) * n_ops, hipMemcpyHostToDevice));
    QS3_TRY(pg_build(sec.get()));
    *out = sec.release();
    return QS3_OK;
}

int qs3_pg_sector_destroy(qs3_pg_sector *sec) {
    if (sec) {
        (void)hipSetDevice(sec->lat->ctx->device);
        delete sec;
    }
    return QS3_OK;
}

int qs3_pg_sector_dim(const qs3_pg_sector *sec, uint64_t *dim) {
    QS3_REQUIRE(sec && dim, QS3_EINVAL, "NULL argument");
    *dim = sec->dim;
    return QS3_OK;
}

int qs3_pg_sector_basis(const qs3_pg_sector *sec, uint64_t *ranks, double *norms) {
    QS3_REQUIRE(sec, QS3_EINVAL, "NULL argument");
    for (uint64_t a = 0; a < sec->dim; ++a) {
        if (ranks) ranks[a] = sec->h_reps[a];
        if (norms) norms[a] = sec->h_norm[a];
    }
    return QS3_OK;
}

int qs3_pg_start_vector(qs3_pg_sector *sec, uint64_t seed, double *v, void *stream) {
    QS3_REQUIRE(sec && v, QS3_EINVAL, "NULL argument");
    (void)hipSetDevice(sec->lat->ctx->device);
    if (sec->dim == 0) return QS3_OK;
    hipLaunchKernelGGL(k_pg_start, dim3(blocks_for(sec->dim, 256)), dim3(256), 0, (hipStream_t)stream,
                       sec->reps.as<uint64_t>(), sec->dim, seed, v);
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

int qs3_pg_matvec(qs3_pg_sector *sec, const double *v, double *w, void *stream) {
    QS3_REQUIRE(sec && v && w, QS3_EINVAL, "NULL argument");
    QS3_REQUIRE(v != w, QS3_EINVAL, "v and w must not alias");
    (void)hipSetDevice(sec->lat->ctx->device);
    return pg_apply(sec, v, w, (hipStream_t)stream);
}

int qs3_pg_to_momentum(qs3_pg_sector *sec, const double *v, qs3_sector *msec, void *out, void *stream) {
    QS3_REQUIRE(sec && v && msec && out, QS3_EINVAL, "NULL argument");
    QS3_REQUIRE(msec->has_k && msec->lat == sec->lat && msec->K == sec->K && msec->kv[0] == sec->kv[0] &&
                    msec->kv[1] == sec->kv[1] && msec->kv[2] == sec->kv[2],
                QS3_EINVAL, "msec must be the momentum sector of the same lattice, n_down and k");
    (void)hipSetDevice(sec->lat->ctx->device);
    hipStream_t s = (hipStream_t)stream;
    if (msec->dim)
        hipLaunchKernelGGL(k_pg_zero2, dim3(blocks_for(msec->dim, 256)), dim3(256), 0, s, msec->dim, (double2 *)out);
    QS3_HIP(hipGetLastError());
    if (sec->dim == 0 || msec->dim == 0) return QS3_OK;
    return dispatch_expand(sec, ExpandArgs{v, msec, (double2 *)out, s});
}

int qs3_pg_eigs(qs3_pg_sector *sec, const qs3_eigs_opts *opts, double *evals, double *evecs,
                qs3_eigs_info *info, void *stream) {
    QS3_REQUIRE(sec && opts && evals, QS3_EINVAL, "NULL argument");
    QS3_REQUIRE(sec->dim > 0, QS3_EINVAL, "empty sector");
    QS3_REQUIRE(opts->precision == QS3_PREC_F64 || opts->precision == QS3_PREC_F32MV, QS3_EINVAL,
                "unknown precision");
    (void)hipSetDevice(sec->lat->ctx->device);
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = (hipStream_t)stream;
    qs3_eigs_opts o = *opts;
    QS3_TRY(fill_opts(o, sec->dim));
    qs3_ctx *ctx = sec->lat->ctx;
    PGOp op(sec);
    DevBuf v0, vo;
    QS3_TRY(v0.alloc(ctx, sizeof(double) * sec->dim));
    QS3_TRY(qs3_pg_start_vector(sec, o.seed, v0.as<double>(), s));
    if (evecs) QS3_TRY(vo.alloc(ctx, sizeof(double) * sec->dim * o.nev));
    std::vector<double> ev;
    std::vector<qs3_eigs_info> infs;
    QS3_TRY(solve_blocking(ctx, &op, o, v0.as<double>(), s, ev, infs, evecs ? vo.as<double>() : nullptr));
    if (evecs)
        QS3_HIP(hipMemcpyAsync(evecs, vo.ptr, sizeof(double) * sec->dim * o.nev, hipMemcpyDeviceToDevice, s));
    QS3_HIP(hipStreamSynchronize(s));
    qs3_eigs_info inf = infs[0];
    for (int y = 0; y < opts->nev; ++y) evals[y] = ev[y];
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return inf.converged ? QS3_OK : QS3_ENOCONV;
}

}  // extern "C"
