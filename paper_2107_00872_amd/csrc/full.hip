// Full diagonalisation of a sector and thermal averages (Sec. 3.4 "Full
// diagonalization", Eq. (ens)).  The dense block is formed on the device by
// the hop kernels (one row per thread, column major); its eigenpairs come
// from the ROCm library's dense Hermitian eigensolver (divide and conquer),
// as the paper delegates them to LAPACK (divide and conquer for eigenvalues,
// the QR iteration when eigenvectors are wanted).
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "qs3_hv.h"
#include "qs3_impl.h"

namespace qs3 {

#define QS3_SWK(K, CALL)          \
    switch (K) {                  \
        case 0: return CALL(0);   \
        case 1: return CALL(1);   \
        case 2: return CALL(2);   \
        case 3: return CALL(3);   \
        case 4: return CALL(4);   \
        case 5: return CALL(5);   \
        case 6: return CALL(6);   \
        case 7: return CALL(7);   \
        case 8: return CALL(8);   \
        default: break;           \
    }                             \
    set_error("N_down out of range"); \
    return QS3_EINVAL;

static int dense_u1(qs3_sector *sec, double *A, hipStream_t s) {
#define QS3_DU(k) dense_u1_K<k>(sec, A, s)
    QS3_SWK(sec->K, QS3_DU)
#undef QS3_DU
}

static int dense_k(qs3_sector *sec, const int64_t *u2c, double *A, hipStream_t s) {
#define QS3_DK(k) dense_k_K<(k > 6 ? 6 : k)>(sec, u2c, A, s)
    QS3_REQUIRE(sec->K <= 6, QS3_EINVAL, "momentum sectors need N_down <= 6");
    QS3_SWK(sec->K, QS3_DK)
#undef QS3_DK
}

// H of the sector into A (device, dim x dim column major, zeroed here)
static int build_dense(qs3_sector *sec, void *A, hipStream_t s) {
    const uint64_t d = sec->dim;
    const size_t elem = sec->has_k ? 16 : 8;
    QS3_HIP(hipMemsetAsync(A, 0, elem * d * d, s));
    if (!sec->has_k) return dense_u1(sec, (double *)A, s);
    // union row -> basis index of the sector
    const uint64_t n = sec->bat->ks->n_reps;
    std::vector<int64_t> c2u(d), u2c(std::max<uint64_t>(n, 1), -1);
    if (d) QS3_HIP(hipMemcpy(c2u.data(), sec->comp2u.ptr, sizeof(int64_t) * d, hipMemcpyDeviceToHost));
    for (uint64_t i = 0; i < d; ++i) u2c[c2u[i]] = (int64_t)i;
    DevBuf du;
    QS3_TRY(du.alloc(sec->lat->ctx, sizeof(int64_t) * u2c.size()));
    QS3_HIP(hipMemcpyAsync(du.ptr, u2c.data(), sizeof(int64_t) * u2c.size(), hipMemcpyHostToDevice, s));
    QS3_TRY(dense_k(sec, du.as<int64_t>(), (double *)A, s));
    QS3_HIP(hipStreamSynchronize(s));  // du is released on return
    return QS3_OK;
}

void *blas_on(qs3_ctx *ctx, hipStream_t s) {
    if (!ctx->blas) {
        rocblas_handle h = nullptr;
        if (rocblas_create_handle(&h) != rocblas_status_success) return nullptr;
        ctx->blas = h;
    }
    rocblas_set_stream((rocblas_handle)ctx->blas, s);
    return ctx->blas;
}

void blas_release(qs3_ctx *ctx) {
    if (ctx->blas) {
        hipSetDevice(ctx->device);
        rocblas_destroy_handle((rocblas_handle)ctx->blas);
        ctx->blas = nullptr;
    }
}

}  // namespace qs3

using namespace qs3;

extern "C" {

int qs3_dense(qs3_sector *sec, void *H, void *stream) {
    QS3_REQUIRE(sec && H, QS3_EINVAL, "NULL argument");
    QS3_REQUIRE(sec->dim <= 46340, QS3_EINVAL, "dense blocks need dim <= 46340");
    hipSetDevice(sec->lat->ctx->device);
    hipStream_t s = (hipStream_t)stream;
    QS3_TRY(build_dense(sec, H, s));
    QS3_HIP(hipStreamSynchronize(s));
    return QS3_OK;
}

int qs3_full_diag(qs3_sector *sec, double *evals, void *evecs, void *stream) {
    QS3_REQUIRE(sec && evals, QS3_EINVAL, "NULL argument");
    QS3_REQUIRE(sec->dim <= 46340, QS3_EINVAL, "full diagonalisation needs dim <= 46340");
    hipSetDevice(sec->lat->ctx->device);
    hipStream_t s = (hipStream_t)stream;
    const uint64_t d = sec->dim;
    if (d == 0) return QS3_OK;
    const size_t elem = sec->has_k ? 16 : 8;
    DevBuf work, dvals, dE, dinfo;
    void *A = evecs;
    if (!A) {
        QS3_TRY(work.alloc(sec->lat->ctx, elem * d * d));
        A = work.ptr;
    }
    QS3_TRY(dvals.alloc(sec->lat->ctx, sizeof(double) * d));
    QS3_TRY(dE.alloc(sec->lat->ctx, sizeof(double) * d));
    QS3_TRY(dinfo.alloc(sec->lat->ctx, sizeof(rocblas_int)));
    QS3_TRY(build_dense(sec, A, s));
    std::lock_guard<std::mutex> lock(sec->lat->ctx->blas_mu);
    rocblas_handle h = (rocblas_handle)blas_on(sec->lat->ctx, s);
    QS3_REQUIRE(h, QS3_EDEVICE, "rocblas handle");
    // eigenvalues only: divide and conquer; with eigenvectors: the QR
    // iteration, which keeps degenerate eigenspaces finite
    rocblas_status st;
    if (!evecs) {
        if (sec->has_k)
            st = rocsolver_zheevd(h, rocblas_evect_none, rocblas_fill_upper, (rocblas_int)d,
                                  (rocblas_double_complex *)A, (rocblas_int)d, dvals.as<double>(), dE.as<double>(),
                                  dinfo.as<rocblas_int>());
        else
            st = rocsolver_dsyevd(h, rocblas_evect_none, rocblas_fill_upper, (rocblas_int)d, (double *)A,
                                  (rocblas_int)d, dvals.as<double>(), dE.as<double>(), dinfo.as<rocblas_int>());
    } else if (sec->has_k) {
        st = rocsolver_zheev(h, rocblas_evect_original, rocblas_fill_upper, (rocblas_int)d,
                             (rocblas_double_complex *)A, (rocblas_int)d, dvals.as<double>(), dE.as<double>(),
                             dinfo.as<rocblas_int>());
    } else {
        st = rocsolver_dsyev(h, rocblas_evect_original, rocblas_fill_upper, (rocblas_int)d, (double *)A,
                             (rocblas_int)d, dvals.as<double>(), dE.as<double>(), dinfo.as<rocblas_int>());
    }
    rocblas_int info = 0;
    hipError_t e1 = hipMemcpyAsync(evals, dvals.ptr, sizeof(double) * d, hipMemcpyDeviceToHost, s);
    hipError_t e2 = hipMemcpyAsync(&info, dinfo.ptr, sizeof(rocblas_int), hipMemcpyDeviceToHost, s);
    hipError_t e3 = hipStreamSynchronize(s);
    QS3_REQUIRE(st == rocblas_status_success, QS3_EDEVICE, "dense eigensolver failed to launch");
    QS3_HIP(e1);
    QS3_HIP(e2);
    QS3_HIP(e3);
    QS3_REQUIRE(info == 0, QS3_ENUMERIC, "dense eigensolver did not converge");
    return QS3_OK;
}

int qs3_thermal(uint64_t n, const double *E, const double *Sz, double h, int n_beta, const double *beta,
                double *lnZ, double *energy, double *heat, double *mag, double *chi) {
    QS3_REQUIRE(n > 0 && E && Sz && n_beta >= 0 && (n_beta == 0 || beta), QS3_EINVAL, "bad argument");
    double e0 = INFINITY;
    for (uint64_t i = 0; i < n; ++i) e0 = std::min(e0, E[i] - h * Sz[i]);
    for (int t = 0; t < n_beta; ++t) {
        const double b = beta[t];
        QS3_REQUIRE(b >= 0 && std::isfinite(b), QS3_EINVAL, "beta must be finite and >= 0");
        double Z = 0, s1 = 0, s2 = 0, m1 = 0, m2 = 0;
        for (uint64_t i = 0; i < n; ++i) {
            const double eh = E[i] - h * Sz[i];
            const double w = std::exp(-b * (eh - e0));
            Z += w;
            s1 += w * eh;
            s2 += w * eh * eh;
            m1 += w * Sz[i];
            m2 += w * Sz[i] * Sz[i];
        }
        const double em = s1 / Z, mm = m1 / Z;
        if (lnZ) lnZ[t] = std::log(Z) - b * e0;
        if (energy) energy[t] = em;
        if (heat) heat[t] = b * b * (s2 / Z - em * em);
        if (mag) mag[t] = mm;
        if (chi) chi[t] = b * (m2 / Z - mm * mm);
    }
    return QS3_OK;
}

}  // extern "C"
