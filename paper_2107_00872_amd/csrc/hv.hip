// Host-side dispatch of the H.v kernels (Sec. 3.5, Alg. 9) over N_down: each
// N_down's template instances live in their own translation unit
// (hv_inst.hip built with QS3_INST_K = 0..8).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "qs3_hv.h"
#include "qs3_impl.h"

namespace qs3 {

LatArgs lat_args(const qs3_lattice *lat) {
    LatArgs L;
    L.N = lat->N;
    L.lx = lat->lx;
    L.ly = lat->ly;
    L.lz = lat->lz;
    L.ptr = lat->d_ptr.as<int>();
    L.nbr = lat->d_nbr.as<uint16_t>();
    L.jxy_h = lat->d_jxy_h.as<double>();
    L.jz_h = lat->d_jz_h.as<double>();
    L.jxy_hf = lat->d_jxy_hf.as<float>();
    L.jz_hf = lat->d_jz_hf.as<float>();
    L.jp_h = lat->d_jp_h.as<double2>();
    L.jp_hf = lat->d_jp_hf.as<float2>();
    L.n_edges = (int)lat->h_nbr.size();
    L.uniform = lat->uniform ? 1 : 0;
    L.u_jxy_h = lat->u_jxy_h;
    L.u_jz_h = lat->u_jz_h;
    L.ez4 = lat->ez4;
    L.coords = lat->d_coords.as<uint32_t>();
    L.ns = lat->ns;
    L.sqrt_tab = lat->d_sqrt.as<double>();
    return L;
}

BatchArgs batch_args(qs3_batch *bat) {
    BatchArgs A;
    A.L = lat_args(bat->lat);
    A.n_reps = bat->ks->n_reps;
    A.reps = bat->ks->reps.as<uint64_t>();
    A.stab = bat->ks->stab.as<uint16_t>();
    A.nt_of = bat->ks->nt_of.as<int32_t>();
    A.compat_nt = bat->compat_nt.as<uint8_t>();
    A.table = bat->ks->table.as<uint64_t>();
    A.hops = bat->ks->hops.as<uint64_t>();
    A.hmax = bat->ks->hmax;
    A.dir = bat->ks->dir.as<uint32_t>();
    A.dir_shift = bat->ks->dir_shift;
    A.B = bat->B;
    A.ld = bat->B;
    A.G = 1;
    while (A.G < bat->B && A.G < 64) A.G <<= 1;
    A.kmul = bat->kmul.as<int32_t>();
    A.M = bat->M;
    A.invM = 1.0 / bat->M;
    A.phase = bat->phase.as<double2>();
    A.active = bat->active_dev;
    A.ph_lds_off = -1;
    A.tP = bat->tP.as<uint16_t>();
    A.gcls = bat->gcls.as<uint8_t>();
    return A;
}

int grid_for(qs3_ctx *ctx, uint64_t tiles) {
    uint64_t want = (uint64_t)ctx->n_cu * 8;
    uint64_t g = std::min<uint64_t>(tiles, want);
    if (g >= 8) g &= ~uint64_t(7);
    return (int)std::max<uint64_t>(g, 1);
}

int grid_cover(qs3_ctx *ctx, uint64_t tiles) {
    // one tile per block while the tiles fill at most 8 blocks per CU (the
    // count rounded up to whole XCD rounds: no block takes two tiles while
    // others idle), else 8 blocks per CU
    const uint64_t want = (uint64_t)ctx->n_cu * 8;
    if (tiles >= want) return (int)want;
    return (int)std::max<uint64_t>((tiles + 7) / 8 * 8, 1);
}

#define QS3_SWITCH_K(K, MAXK, CALL)                     \
    switch (K) {                                       \
        case 0: return CALL(0);                        \
        case 1: return CALL(1);                        \
        case 2: return CALL(2);                        \
        case 3: return CALL(3);                        \
        case 4: return CALL(4);                        \
        case 5: return CALL(5);                        \
        case 6: return CALL(6);                        \
        default: break;                                \
    }                                                  \
    if (MAXK > 6) {                                    \
        if (K == 7) return CALL##_HI(7);               \
        if (K == 8) return CALL##_HI(8);               \
    }                                                  \
    set_error("N_down out of range");                  \
    return QS3_EINVAL;

#define QS3_HV_U1(k) hv_u1_K<k>(sec, v, vtype, w, wtype, s)
#define QS3_HV_U1_HI QS3_HV_U1
int hv_u1(qs3_sector *sec, const void *v, int vtype, void *w, int wtype, hipStream_t s) {
    if (sec->dim == 0) return QS3_OK;
    QS3_SWITCH_K(sec->K, 8, QS3_HV_U1)
}

#define QS3_ROW_U1(k) row_u1_K<k>(sec, row, cap, cols, vals, diag, nnz)
#define QS3_ROW_U1_HI QS3_ROW_U1
int row_u1(qs3_sector *sec, uint64_t row, int cap, int64_t *cols, double *vals, double *diag,
           int *nnz) {
    QS3_REQUIRE(row < sec->dim, QS3_EINVAL, "row out of range");
    QS3_SWITCH_K(sec->K, 8, QS3_ROW_U1)
}

#define QS3_HV_B(k) hv_batch_K<k>(bat, v, vtype, w, wtype, s)
#define QS3_HV_B_HI(k) QS3_EINVAL
static int hv_batch_raw(qs3_batch *bat, const void *v, int vtype, void *w, int wtype,
                        hipStream_t s) {
    QS3_SWITCH_K(bat->K, 6, QS3_HV_B)
}

__global__ void k_c128_to_c64(uint64_t nd, const double *__restrict__ in, float *__restrict__ out) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nd) out[i] = (float)in[i];
}

int hv_batch(qs3_batch *bat, const void *v, int vtype, void *w, int wtype, hipStream_t s) {
    if (bat->ks->n_reps == 0) return QS3_OK;
    if (vtype == QS3_C64 && wtype == QS3_C64) {
        // float32 rows, float32 result: the kernel stores float64 copies of the
        // float32 row sums, converted here
        const uint64_t nd = 2 * bat->ks->n_reps * (uint64_t)bat->B;
        DevBuf tmp;
        QS3_TRY(tmp.alloc(bat->lat->ctx, sizeof(double) * nd));
        QS3_TRY(hv_batch_raw(bat, v, QS3_C64, tmp.ptr, QS3_C128, s));
        hipLaunchKernelGGL(k_c128_to_c64, dim3((unsigned)((nd + 255) / 256)), dim3(256), 0, s, nd,
                           tmp.as<double>(), (float *)w);
        QS3_HIP(hipGetLastError());
        QS3_HIP(hipStreamSynchronize(s));
        return QS3_OK;
    }
    return hv_batch_raw(bat, v, vtype, w, wtype, s);
}

#define QS3_ROW_K(k) row_k_K<k>(sec, (uint64_t)u, cap, cols, vals, diag, nnz)
#define QS3_ROW_K_HI(k) QS3_EINVAL
static int row_k_raw(qs3_sector *sec, int64_t u, int cap, int64_t *cols, double *vals,
                     double *diag, int *nnz) {
    QS3_SWITCH_K(sec->K, 6, QS3_ROW_K)
}

int row_k(qs3_sector *sec, uint64_t row, int cap, int64_t *cols, double *vals, double *diag,
          int *nnz) {
    QS3_REQUIRE(row < sec->dim, QS3_EINVAL, "row out of range");
    std::vector<int64_t> c2u(sec->dim);
    QS3_HIP(hipMemcpy(c2u.data(), sec->comp2u.ptr, sizeof(int64_t) * sec->dim, hipMemcpyDeviceToHost));
    QS3_TRY(row_k_raw(sec, c2u[row], cap, cols, vals, diag, nnz));
    // union indices -> basis indices of the sector
    int m = std::min(*nnz, cap);
    for (int i = 0; i < m; ++i) {
        auto it = std::lower_bound(c2u.begin(), c2u.end(), cols[i]);
        cols[i] = (it != c2u.end() && *it == cols[i]) ? (int64_t)(it - c2u.begin()) : -1;
    }
    return QS3_OK;
}

#define QS3_SMALL(k) lanczos_small_K<k>(lat, bt, bat, S, s)
#define QS3_SMALL_HI QS3_SMALL
int lanczos_small(qs3_lattice *lat, int K, const BinomTable *bt, qs3_batch *bat, const SmallArgs &S,
                  hipStream_t s) {
    if (S.slots + 2 > 520 || S.n > 65536) return 1;
    QS3_SWITCH_K(K, 8, QS3_SMALL)
}

#define QS3_BUILD(k) build_kstruct_K<k>(lat, *bt, ks, s)
#define QS3_BUILD_HI(k) QS3_EINVAL
int build_kstruct(qs3_lattice *lat, int K, KStructure *ks, hipStream_t s) {
    std::shared_ptr<BinomTable> bt;
    QS3_TRY(get_binom(lat, K, &bt));
    ks->K = K;
    QS3_SWITCH_K(K, 6, QS3_BUILD)
}

}  // namespace qs3
