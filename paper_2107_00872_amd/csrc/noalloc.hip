// The allocation-free variant of qs3_matvec (for callers that cannot
// allocate device memory: code under HIP graph capture, tight serving loops).
//
// A momentum sector whose compact basis is smaller than the union of
// representatives (some representatives are incompatible with its k) is
// multiplied in the union layout: scatter into a union vector, the batched
// H.v, gather back.  qs3_matvec allocates those two union vectors on the
// sector's first call; this variant takes them from one file-scope device
// array instead, whose address is looked up once per device when a context is
// created.  Every call on a device shares that device's array (it keeps the
// last call's contents; everything a call reads from it is written by the
// same call first), so calls that overlap on one GPU race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "qs3_impl.h"
#include "qs3_krylov.h"

namespace qs3 {

constexpr uint64_t NOALLOC_SCRATCH_BYTES = 64ull << 20;

// the two union vectors of the largest admitted sector: 2 x 16 B x n_reps
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
static void *g_scratch_dev[NOALLOC_MAX_DEVICES] = {};
static std::mutex g_scratch_mu;

// Called by qs3_ctx_create with `device` current: the device address of this
// device's copy of the array (in host code `scratch` names a host-side
// stand-in, not device memory).
int noalloc_init(int device) {
    QS3_REQUIRE(device >= 0 && device < NOALLOC_MAX_DEVICES, QS3_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_dev[device]) return QS3_OK;
    void *p = nullptr;
    QS3_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    QS3_REQUIRE(p != nullptr, QS3_EDEVICE, "no device address for the scratch array");
    g_scratch_dev[device] = p;
    return QS3_OK;
}

static __global__ void k_gather_to_f32(uint64_t d, const int64_t *__restrict__ c2u,
                                       const double2 *__restrict__ src, float2 *__restrict__ dst) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d) return;
    const double2 x = c2u ? src[c2u[i]] : src[i];
    dst[i] = make_float2((float)x.x, (float)x.y);
}

}  // namespace qs3

using namespace qs3;

extern "C" int qs3_matvec_noalloc(qs3_sector *sec, const void *v, void *w, int dtype, void *stream) {
    QS3_REQUIRE(sec && v && w, QS3_EINVAL, "NULL argument");
    QS3_REQUIRE(v != w, QS3_EINVAL, "v and w must not alias");
    const int dev = sec->lat->ctx->device;
    QS3_HIP(hipSetDevice(dev));
    hipStream_t s = (hipStream_t)stream;
    if (!sec->has_k) {
        // the fixed-N_down product needs no scratch
        QS3_REQUIRE(dtype == QS3_F64 || dtype == QS3_F32, QS3_EINVAL,
                    "fixed-N_down vectors are QS3_F64 or QS3_F32");
        return hv_u1(sec, v, dtype, w, dtype, s);
    }
    QS3_REQUIRE(dtype == QS3_C128 || dtype == QS3_C64, QS3_EINVAL,
                "momentum vectors are QS3_C128 or QS3_C64");
    const uint64_t n = sec->bat->ks->n_reps;
    if (sec->dim == n && dtype == QS3_C128) return hv_batch(sec->bat, v, dtype, w, dtype, s);
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        base = dev >= 0 && dev < NOALLOC_MAX_DEVICES ? g_scratch_dev[dev] : nullptr;
    }
    QS3_REQUIRE(base, QS3_EINVAL, "no context was created on this device");
    QS3_REQUIRE(2 * 16 * n <= NOALLOC_SCRATCH_BYTES, QS3_EINVAL,
                "sector too large for qs3_matvec_noalloc (at most 2,097,152 representatives)");
    double *ua = (double *)base;                              // union input
    double *ub = (double *)((char *)base + 16 * n);           // union output (complex128)
    const uint64_t nb = (sec->dim + 255) / 256;
    if (dtype == QS3_C128) {
        QS3_TRY(scatter_compact(sec, (const double *)v, ua, s));
        QS3_TRY(hv_batch(sec->bat, ua, QS3_C128, ub, QS3_C128, s));
        return gather_compact(sec, ub, (double *)w, s);
    }
    // complex64 in and out: float32 products, float32 result converted from
    // the kernel's float64 copies of its float32 row sums
    const float *vin = (const float *)v;
    if (sec->dim != n) {
        QS3_TRY(scatter_compact_f32(sec, (const float *)v, (float *)ua, s));
        vin = (const float *)ua;
    }
    QS3_TRY(hv_batch(sec->bat, vin, QS3_C64, ub, QS3_C128, s));
    if (sec->dim)
        hipLaunchKernelGGL(k_gather_to_f32, dim3((unsigned)nb), dim3(256), 0, s, sec->dim,
                           sec->dim != n ? sec->comp2u.as<int64_t>() : nullptr, (const double2 *)ub,
                           (float2 *)w);
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}
