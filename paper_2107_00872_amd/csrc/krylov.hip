// Lanczos and thick-restart Lanczos (Sec. 3.7, Alg. 10) on the device.
//
// Vectors are "multi-vectors" of n rows x B columns in the layout [row][col]
// (B = 1 for a single sector, B = number of momentum sectors for a batch),
// real (fixed-N_down) or complex (momentum).  Every column is an independent
// Lanczos run: its alpha, beta and reorthogonalisation coefficients are
// per-column device scalars, so one launch of each kernel advances all
// columns and the host only reads alpha/beta once per restart cycle.
//
// Column reductions are deterministic: fixed row chunks, a fixed in-block
// tree, and a fixed-order sum over chunks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <limits>
#include <thread>
#include <vector>

#include "qs3_device.h"
#include "qs3_impl.h"
#include "qs3_hv.h"
#include "qs3_krylov.h"

namespace qs3 {

// ------------------------------------------------------------------ geometry of reductions
static RedGeom red_geom(uint64_t n, int B) {
    // about 1024 blocks per reduction launch (4 per CU); chunk rows are a
    // multiple of the block's row count
    RedGeom g;
    g.n = n;
    g.B = B;
    g.TC = 1;
    while (g.TC < B && g.TC < 64) g.TC <<= 1;
    g.TR = 256 / g.TC;
    g.ncoltile = (B + g.TC - 1) / g.TC;
    const uint64_t want = std::max<uint64_t>(1, 1024 / g.ncoltile);
    uint64_t rc = std::max<uint64_t>((uint64_t)g.TR, (n + want - 1) / want);
    rc = (rc + g.TR - 1) / g.TR * g.TR;
    g.RC = rc;
    g.nchunk = (int)std::max<uint64_t>(1, (n + rc - 1) / rc);
    return g;
}

template <bool CPLX>
struct Elem;
template <>
struct Elem<false> {
    using T = double;
    __device__ static double re(T a) { return a; }
};
template <>
struct Elem<true> {
    using T = double2;
};

// conj(x) * y accumulated as (re, im)
__device__ __forceinline__ void cdot_acc(double x, double y, double &sr, double &si) { sr += x * y; }
__device__ __forceinline__ void cdot_acc(double2 x, double2 y, double &sr, double &si) {
    sr += x.x * y.x + x.y * y.y;
    si += x.x * y.y - x.y * y.x;
}

// ------------------------------------------------------------------ kernels
// The three-term part of a Lanczos step, applied on the fly (never stored):
// Y - alpha_b P0 - beta_b P1 per column, in the order a separate update pass
// would use.  P0 == null: Y unchanged; P1 == null: no beta term.  i0 / i1:
// the slot indices of P0 / P1 among the basis vectors X_j of the same pass
// (-1 if they are not among them), so that a kernel holding P0 and P1 in
// registers does not read those slots a second time.
struct ThreeTerm {
    const double *P0 = nullptr, *P1 = nullptr;
    const double2 *alpha = nullptr;
    const double *beta = nullptr;
    int i0 = -1, i1 = -1;
};

__device__ __forceinline__ double three_term(double w, uint64_t e, const ThreeTerm &f, double a, double be) {
    w -= a * f.P0[e];
    if (f.P1) w -= be * f.P1[e];
    return w;
}
__device__ __forceinline__ double2 three_term(double2 w, uint64_t e, const ThreeTerm &f, double a, double be) {
    const double2 p0 = ((const double2 *)f.P0)[e];
    w.x -= a * p0.x;
    w.y -= a * p0.y;
    if (f.P1) {
        const double2 p1 = ((const double2 *)f.P1)[e];
        w.x -= be * p1.x;
        w.y -= be * p1.y;
    }
    return w;
}

// The three-term part on values already loaded (the arithmetic of three_term).
__device__ __forceinline__ double sub_three(double w, double p0, double p1, bool has1, double a, double be) {
    w -= a * p0;
    if (has1) w -= be * p1;
    return w;
}
__device__ __forceinline__ double2 sub_three(double2 w, double2 p0, double2 p1, bool has1, double a, double be) {
    w.x -= a * p0.x;
    w.y -= a * p0.y;
    if (has1) {
        w.x -= be * p1.x;
        w.y -= be * p1.y;
    }
    return w;
}

// partial[(chunk * JO + j) * B + b] (re, im) = sum over the chunk's rows of
// conj(X_j[r, b]) * Y'[r, b] for j < J (X_j = X + j * stride) and, when
// selfdot, |Y'[r, b]|^2 at j = J (JO = J + selfdot outputs), with Y' = Y
// after the three-term part f.  Blocks along z take groups of JM outputs
// (Y is read once per group).
// Columns with mask[b] == 0 are skipped (their partials are written as zero).
template <bool CPLX, int JM>
__global__ __launch_bounds__(256) void k_multidot(RedGeom g, const double *__restrict__ X,
                                                  uint64_t stride, int J, int selfdot,
                                                  const double *__restrict__ Y, ThreeTerm f,
                                                  const uint8_t *__restrict__ mask,
                                                  double2 *__restrict__ partial) {
    using T = typename Elem<CPLX>::T;
    const int tc = threadIdx.x % g.TC, tr = threadIdx.x / g.TC;
    const int b = blockIdx.y * g.TC + tc;
    const uint64_t r0 = (uint64_t)blockIdx.x * g.RC;
    const uint64_t r1 = min(g.n, r0 + g.RC);
    const int JO = J + selfdot;
    const bool on = b < g.B && (!mask || mask[b]);
    const double fa = (on && f.P0) ? f.alpha[b].x : 0.0;
    const double fb = (on && f.P0 && f.P1) ? f.beta[b] : 0.0;
    __shared__ double2 red[256][4];
    const T *Yt = (const T *)Y;
    for (int j0 = blockIdx.z * JM; j0 < JO; j0 += JM * gridDim.z) {
        double sr[JM], si[JM];
#pragma unroll
        for (int q = 0; q < JM; ++q) sr[q] = si[q] = 0.0;
        if (on) {
            // two rows (r, r + TR) per pass, each output summed in row order
            for (uint64_t r = r0 + tr; r < r1; r += 2 * (uint64_t)g.TR) {
                const uint64_t e = r * g.B + b, e2 = (r + g.TR) * g.B + b;
                const bool two = r + g.TR < r1;
                T y = Yt[e], y2 = two ? Yt[e2] : T{};
                if (f.P0) {
                    y = three_term(y, e, f, fa, fb);
                    if (two) y2 = three_term(y2, e2, f, fa, fb);
                }
#pragma unroll
                for (int q = 0; q < JM; ++q) {
                    const int jj = j0 + q;
                    if (jj < J) {
                        const T *xj = (const T *)(X + (size_t)jj * stride);
                        const T x = xj[e], x2 = two ? xj[e2] : T{};
                        cdot_acc(x, y, sr[q], si[q]);
                        if (two) cdot_acc(x2, y2, sr[q], si[q]);
                    } else if (jj == J && selfdot) {
                        cdot_acc(y, y, sr[q], si[q]);
                        if (two) cdot_acc(y2, y2, sr[q], si[q]);
                    }
                }
            }
        }
#pragma unroll
        for (int q0 = 0; q0 < JM; q0 += 4) {
            if (j0 + q0 >= JO) break;
#pragma unroll
            for (int q = 0; q < 4; ++q) red[threadIdx.x][q] = make_double2(sr[q0 + q], si[q0 + q]);
            __syncthreads();
            for (int s = g.TR / 2; s > 0; s >>= 1) {
                if (tr < s) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        double2 a = red[threadIdx.x][q], c = red[threadIdx.x + s * g.TC][q];
                        red[threadIdx.x][q] = make_double2(a.x + c.x, a.y + c.y);
                    }
                }
                __syncthreads();
            }
            if (tr == 0 && b < g.B) {
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (j0 + q0 + q < JO)
                        partial[((size_t)blockIdx.x * JO + j0 + q0 + q) * g.B + b] = red[threadIdx.x][q];
            }
            __syncthreads();
        }
    }
}

// The same multi-dot for many outputs with Y' read from memory once per G *
// JPL outputs instead of once per 4: G thread groups cover the same (row,
// column) elements, group gi taking outputs j0 + gi * JPL .. + JPL - 1.
// With TC * G <= 64 the groups sit in one wavefront, so their loads of Y, P0
// and P1 are the same addresses in the same instructions (one request per
// cache line); with TC * G > 64 they are spread over the waves of the block,
// which read the same lines within a short time.  The slots that
// are P0 or P1 come from the registers that formed Y'.  Threads are (column
// c < TC, group gi < G, row lane rr < TR) with c fastest; each thread sums
// its rows in row order, then a fixed tree over rr.  Partials as in
// k_multidot.
template <bool CPLX, int G, int JPL>
__global__ __launch_bounds__(256) void k_multidot_g(RedGeom g, const double *__restrict__ X,
                                                    uint64_t stride, int J, int selfdot,
                                                    const double *__restrict__ Y, ThreeTerm f,
                                                    const uint8_t *__restrict__ mask,
                                                    double2 *__restrict__ partial) {
    using T = typename Elem<CPLX>::T;
    const int c = threadIdx.x % g.TC, gi = (threadIdx.x / g.TC) % G, rr = threadIdx.x / (g.TC * G);
    const int b = blockIdx.y * g.TC + c;
    const uint64_t r0 = (uint64_t)blockIdx.x * g.RC;
    const uint64_t r1 = min(g.n, r0 + g.RC);
    const int JO = J + selfdot;
    const bool on = b < g.B && (!mask || mask[b]);
    const double fa = (on && f.P0) ? f.alpha[b].x : 0.0;
    const double fb = (on && f.P0 && f.P1) ? f.beta[b] : 0.0;
    __shared__ double2 red[256][JPL];
    const T *Yt = (const T *)Y;
    for (int j0 = blockIdx.z * G * JPL; j0 < JO; j0 += G * JPL * gridDim.z) {
        const int jb = j0 + gi * JPL;  // this group's first output
        double sr[JPL], si[JPL];
#pragma unroll
        for (int q = 0; q < JPL; ++q) sr[q] = si[q] = 0.0;
        if (on) {
            for (uint64_t r = r0 + rr; r < r1; r += (uint64_t)g.TR) {
                const uint64_t e = r * g.B + b;
                T y = Yt[e], p0{}, p1{};
                if (f.P0) {
                    p0 = ((const T *)f.P0)[e];
                    if (f.P1) p1 = ((const T *)f.P1)[e];
                    y = sub_three(y, p0, p1, f.P1 != nullptr, fa, fb);
                }
                T xv[JPL];
#pragma unroll
                for (int q = 0; q < JPL; ++q) {
                    const int jj = jb + q;
                    if (jj == f.i0) xv[q] = p0;
                    else if (jj == f.i1) xv[q] = p1;
                    else if (jj < J) xv[q] = ((const T *)(X + (size_t)jj * stride))[e];
                    else xv[q] = y;  // the self-dot (jj == J) or unused
                }
#pragma unroll
                for (int q = 0; q < JPL; ++q) {
                    const int jj = jb + q;
                    if (jj < J || (jj == J && selfdot)) cdot_acc(xv[q], y, sr[q], si[q]);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < JPL; ++q) red[threadIdx.x][q] = make_double2(sr[q], si[q]);
        __syncthreads();
        for (int s2 = g.TR / 2; s2 > 0; s2 >>= 1) {
            if (rr < s2) {
#pragma unroll
                for (int q = 0; q < JPL; ++q) {
                    const double2 a = red[threadIdx.x][q], o = red[threadIdx.x + s2 * g.TC * G][q];
                    red[threadIdx.x][q] = make_double2(a.x + o.x, a.y + o.y);
                }
            }
            __syncthreads();
        }
        if (rr == 0 && b < g.B) {
#pragma unroll
            for (int q = 0; q < JPL; ++q)
                if (jb + q < JO) partial[((size_t)blockIdx.x * JO + jb + q) * g.B + b] = red[threadIdx.x][q];
        }
        __syncthreads();
    }
}

// W := W' - sum_{j<J} X_j h[j * B + b] on the columns with mask[b] != 0 (all
// when mask is null), W' = W after the three-term part f, and
// partial[chunk * B + b] = sum over the chunk's rows of |W|^2 after the
// update (the norm for beta, fused into the same pass).
template <bool CPLX>
__global__ __launch_bounds__(256) void k_cgs_update_norm(RedGeom g, double *__restrict__ W,
                                                         const double *__restrict__ X, uint64_t stride,
                                                         int J, const double2 *__restrict__ h, ThreeTerm f,
                                                         const uint8_t *__restrict__ mask,
                                                         double2 *__restrict__ partial) {
    const int tc = threadIdx.x % g.TC, tr = threadIdx.x / g.TC;
    const int b = blockIdx.y * g.TC + tc;
    const uint64_t r0 = (uint64_t)blockIdx.x * g.RC;
    const uint64_t r1 = min(g.n, r0 + g.RC);
    const bool on = b < g.B && (!mask || mask[b]);
    const double fa = (on && f.P0) ? f.alpha[b].x : 0.0;
    const double fb = (on && f.P0 && f.P1) ? f.beta[b] : 0.0;
    double acc = 0.0;
    if (on) {
        // two rows per pass, so each coefficient load serves both
        for (uint64_t r = r0 + tr; CPLX && r < r1; r += 2 * (uint64_t)g.TR) {
            const uint64_t e = r * g.B + b, e2 = (r + g.TR) * g.B + b;
            const bool two = r + g.TR < r1;
            const double2 z2 = make_double2(0.0, 0.0);
            double2 w = ((double2 *)W)[e];
            double2 w2 = two ? ((double2 *)W)[e2] : z2;
            double2 p0 = z2, p0b = z2, p1 = z2, p1b = z2;
            if (f.P0) {
                p0 = ((const double2 *)f.P0)[e];
                if (two) p0b = ((const double2 *)f.P0)[e2];
                if (f.P1) {
                    p1 = ((const double2 *)f.P1)[e];
                    if (two) p1b = ((const double2 *)f.P1)[e2];
                }
                // the three-term part, in the order of three_term()
                w.x -= fa * p0.x;
                w.y -= fa * p0.y;
                w2.x -= fa * p0b.x;
                w2.y -= fa * p0b.y;
                if (f.P1) {
                    w.x -= fb * p1.x;
                    w.y -= fb * p1.y;
                    w2.x -= fb * p1b.x;
                    w2.y -= fb * p1b.y;
                }
            }
            for (int jj = 0; jj < J; ++jj) {
                const double2 *xj = (const double2 *)(X + (size_t)jj * stride);
                const double2 c = h[(size_t)jj * g.B + b];
                double2 x, x2;
                if (jj == f.i0) {
                    x = p0;
                    x2 = p0b;
                } else if (jj == f.i1) {
                    x = p1;
                    x2 = p1b;
                } else {
                    x = xj[e];
                    x2 = two ? xj[e2] : z2;
                }
                w.x -= x.x * c.x - x.y * c.y;
                w.y -= x.x * c.y + x.y * c.x;
                w2.x -= x2.x * c.x - x2.y * c.y;
                w2.y -= x2.x * c.y + x2.y * c.x;
            }
            ((double2 *)W)[e] = w;
            acc += w.x * w.x + w.y * w.y;
            if (two) {
                ((double2 *)W)[e2] = w2;
                acc += w2.x * w2.x + w2.y * w2.y;
            }
        }
        for (uint64_t r = r0 + tr; !CPLX && r < r1; r += 2 * (uint64_t)g.TR) {
            const uint64_t e = r * g.B + b, e2 = (r + g.TR) * g.B + b;
            const bool two = r + g.TR < r1;
            double w = W[e], w2 = two ? W[e2] : 0.0;
            double p0 = 0.0, p0b = 0.0, p1 = 0.0, p1b = 0.0;
            if (f.P0) {
                p0 = f.P0[e];
                if (two) p0b = f.P0[e2];
                if (f.P1) {
                    p1 = f.P1[e];
                    if (two) p1b = f.P1[e2];
                }
                w -= fa * p0;
                w2 -= fa * p0b;
                if (f.P1) {
                    w -= fb * p1;
                    w2 -= fb * p1b;
                }
            }
            for (int jj = 0; jj < J; ++jj) {
                const double c = h[(size_t)jj * g.B + b].x;
                const double *xj = X + (size_t)jj * stride;
                double x, x2;
                if (jj == f.i0) {
                    x = p0;
                    x2 = p0b;
                } else if (jj == f.i1) {
                    x = p1;
                    x2 = p1b;
                } else {
                    x = xj[e];
                    x2 = two ? xj[e2] : 0.0;
                }
                w -= x * c;
                if (two) w2 -= x2 * c;
            }
            W[e] = w;
            acc += w * w;
            if (two) {
                W[e2] = w2;
                acc += w2 * w2;
            }
        }
    }
    __shared__ double red[256];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = g.TR / 2; s > 0; s >>= 1) {
        if (tr < s) red[threadIdx.x] += red[threadIdx.x + s * g.TC];
        __syncthreads();
    }
    if (tr == 0 && b < g.B) partial[(size_t)blockIdx.x * g.B + b] = make_double2(red[threadIdx.x], 0.0);
}

// Partial reorthogonalisation: Simon's recurrence for the overlaps
// w_{j,k} ~ <psi_j, psi_k> of plain Lanczos, one thread per column.  om holds
// two rows per column ([parity][k][B], row j at parity j & 1, w_{j,j} = 1);
// ab: alpha at [k * B + b], beta_k (the coupling of psi_k and psi_{k+1}) at
// [(slots + k) * B + b]; nrm2: |W|^2 after the three-term update of step x, so
// beta_x = |W|.  Writes row x + 1:
//   beta_x w_{x+1,k} = beta_k w_{x,k+1} + (alpha_k - alpha_x) w_{x,k}
//                      + beta_{k-1} w_{x,k-1} - beta_{x-1} w_{x-1,k}  (k < x)
// plus a rounding term eps1 (beta_k + beta_x) of the sign of the sum,
// w_{x+1,x} = eps1, w_{x+1,x+1} = 1.  Where some |w_{x+1,k}| exceeds sqrt(eps)
// the column is flagged for a Gram-Schmidt pass against psi_0..psi_x now and
// at the next step, and its row is reset to eps1.
__global__ void k_omega(int B, int x, const double *__restrict__ ab, int slots, const double2 *__restrict__ nrm2,
                        double *__restrict__ om, int ostride, const uint8_t *__restrict__ mask,
                        uint8_t *__restrict__ force, uint8_t *__restrict__ flag, double eps1) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double *cur = om + ((size_t)(x & 1) * ostride) * B + b;
    double *nxt = om + ((size_t)((x + 1) & 1) * ostride) * B + b;
    if (x == 0) cur[0] = 1.0;
    if (mask && !mask[b]) {
        flag[b] = 0;
        return;
    }
    const double bx = sqrt(fmax(nrm2[b].x, 0.0));
    const double ax = ab[(size_t)x * B + b];
    const double bxm = x > 0 ? ab[(size_t)(slots + x - 1) * B + b] : 0.0;
    double worst = 0.0;
    double prev_cur = 0.0;  // w_{x,k-1}
    for (int k = 0; k < x; ++k) {
        const double ck = cur[(size_t)k * B], ck1 = cur[(size_t)(k + 1) * B];
        const double bk = ab[(size_t)(slots + k) * B + b];
        const double bkm = k > 0 ? ab[(size_t)(slots + k - 1) * B + b] : 0.0;
        double t = bk * ck1 + (ab[(size_t)k * B + b] - ax) * ck + bkm * prev_cur - bxm * nxt[(size_t)k * B];
        t += copysign(eps1 * (bk + bx), t);
        const double w = bx > 0.0 ? t / bx : INFINITY;
        prev_cur = ck;
        nxt[(size_t)k * B] = w;
        worst = fmax(worst, fabs(w));
    }
    const bool over = !(worst <= 1.4901161193847656e-8);  // sqrt(eps); NaN/inf count as over
    const bool fl = over || force[b];
    force[b] = over && !force[b];
    if (fl)
        for (int k = 0; k < x; ++k) nxt[(size_t)k * B] = eps1;
    nxt[(size_t)x * B] = eps1;
    nxt[(size_t)(x + 1) * B] = 1.0;
    flag[b] = fl;
}

// |W|^2 of the flagged columns from their second pass, then beta = |W|
__global__ void k_merge_sqrt(int B, const uint8_t *__restrict__ flag, const double2 *__restrict__ n2,
                             double2 *__restrict__ n1, double *__restrict__ beta) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double2 v = n1[b];
    if (flag[b]) {
        v = n2[b];
        n1[b] = v;
    }
    beta[b] = sqrt(fmax(v.x, 0.0));
}

// out[j * B + b] = sum_chunk partial[(chunk * J + j) * B + b]: one wavefront
// per output, lanes take chunks lane, lane+64, ... in order, then a fixed
// shuffle tree -- deterministic for a given chunking.  re_out (optional)
// receives the real parts as well.
__global__ __launch_bounds__(256) void k_reduce_chunks(const double2 *__restrict__ partial, int nchunk,
                                                       int JB, double2 *__restrict__ out,
                                                       double *__restrict__ re_out) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= JB) return;
    double sr = 0, si = 0;
    for (int c = lane; c < nchunk; c += 64) {
        double2 p = partial[(size_t)c * JB + i];
        sr += p.x;
        si += p.y;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        sr += __shfl_down(sr, off, 64);
        si += __shfl_down(si, off, 64);
    }
    if (lane == 0) {
        out[i] = make_double2(sr, si);
        if (re_out) re_out[i] = sr;
    }
}

// k_reduce_chunks for the norms of a first Gram-Schmidt pass (one output per
// column) that also sets the second-pass flags: the pass cancelled more than
// half of |W|^2 (Daniel-Gragg-Kaufman-Stewart criterion, eta^2 = 1/2).
__global__ __launch_bounds__(256) void k_reduce_norm_dgks(const double2 *__restrict__ partial, int nchunk, int B,
                                                          double2 *__restrict__ out,
                                                          const double2 *__restrict__ before,
                                                          const uint8_t *__restrict__ mask,
                                                          uint8_t *__restrict__ flag) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= B) return;
    double sr = 0, si = 0;
    for (int c = lane; c < nchunk; c += 64) {
        double2 p = partial[(size_t)c * B + i];
        sr += p.x;
        si += p.y;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        sr += __shfl_down(sr, off, 64);
        si += __shfl_down(si, off, 64);
    }
    if (lane == 0) {
        out[i] = make_double2(sr, si);
        flag[i] = (sr < 0.5 * before[i].x && (!mask || mask[i])) ? 1 : 0;
    }
}

// W -= alpha[b] * P0 (+ beta[b] * P1 when P1 != null); alpha, beta real per column.
template <bool CPLX>
__global__ __launch_bounds__(256) void k_lanczos_update(uint64_t ne, int B, double *__restrict__ W,
                                                        const double *__restrict__ P0,
                                                        const double *__restrict__ P1,
                                                        const double2 *__restrict__ alpha,
                                                        const double *__restrict__ beta,
                                                        const uint8_t *__restrict__ mask) {
    uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const int b = (int)(e % (uint64_t)B);
    if (mask && !mask[b]) return;
    const double a = alpha[b].x;
    const double be = P1 ? beta[b] : 0.0;
    if (CPLX) {
        double2 w = ((double2 *)W)[e], p0 = ((const double2 *)P0)[e];
        w.x -= a * p0.x;
        w.y -= a * p0.y;
        if (P1) {
            double2 p1 = ((const double2 *)P1)[e];
            w.x -= be * p1.x;
            w.y -= be * p1.y;
        }
        ((double2 *)W)[e] = w;
    } else {
        double w = W[e] - a * P0[e];
        if (P1) w -= be * P1[e];
        W[e] = w;
    }
}

// W -= sum_{j<J} X_j * h[j * B + b]
template <bool CPLX>
__global__ __launch_bounds__(256) void k_cgs_update(uint64_t ne, int B, double *__restrict__ W,
                                                    const double *__restrict__ X, uint64_t stride,
                                                    int J, const double2 *__restrict__ h) {
    uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const int b = (int)(e % (uint64_t)B);
    if (CPLX) {
        double2 w = ((double2 *)W)[e];
        for (int j = 0; j < J; ++j) {
            const double2 x = ((const double2 *)(X + (size_t)j * stride))[e];
            const double2 c = h[(size_t)j * B + b];
            w.x -= x.x * c.x - x.y * c.y;
            w.y -= x.x * c.y + x.y * c.x;
        }
        ((double2 *)W)[e] = w;
    } else {
        double w = W[e];
        for (int j = 0; j < J; ++j) w -= X[(size_t)j * stride + e] * h[(size_t)j * B + b].x;
        W[e] = w;
    }
}

// beta[b] = sqrt(nrm2[b].x); P = W / beta (0 if beta == 0)
template <bool CPLX>
__global__ __launch_bounds__(256) void k_scale_out(uint64_t ne, int B, const double *__restrict__ W,
                                                   double *__restrict__ P,
                                                   const double2 *__restrict__ nrm2,
                                                   const uint8_t *__restrict__ mask) {
    uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const int b = (int)(e % (uint64_t)B);
    if (mask && !mask[b]) return;
    const double nb = sqrt(fmax(nrm2[b].x, 0.0));
    const double s = nb > 0.0 ? 1.0 / nb : 0.0;
    if (CPLX) {
        double2 w = ((const double2 *)W)[e];
        ((double2 *)P)[e] = make_double2(w.x * s, w.y * s);
    } else {
        P[e] = W[e] * s;
    }
}

__global__ void k_sqrt_to(int B, const double2 *__restrict__ nrm2, double *__restrict__ out) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < B) out[b] = sqrt(fmax(nrm2[b].x, 0.0));
}

// Out_y = sum_{x < NX} X_x * C[x][y][b] for y < NY (C real, per column, the
// column index fastest so a wavefront's coefficient loads are contiguous),
// masked by active[b].  Each thread takes RPT elements of one column, RPT
// equal row blocks apart, so that every coefficient it loads serves RPT rows.
template <bool CPLX, int NYT, int RPT>
// Out may be X itself when NY <= NYT: a thread then reads every input of its
// elements before it writes any output, and no other thread touches them.
__global__ __launch_bounds__(256) void k_rotate(uint64_t ne, int B, const double *X,
                                                uint64_t stride, int NX, const double *__restrict__ Cm,
                                                int NY, double *Out,
                                                const uint8_t *__restrict__ active) {
    const uint64_t rows = ne / (uint64_t)B;
    const uint64_t part = (rows + RPT - 1) / RPT * (uint64_t)B;  // elements per row block
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= part) return;
    const int b = (int)(e % (uint64_t)B);
    if (active && !active[b]) return;
    uint64_t ei[RPT];
    bool ok[RPT];
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
        ei[k] = e + (uint64_t)k * part;
        ok[k] = ei[k] < ne;
    }
    const double *Cb = Cm + b;
    const size_t cs = (size_t)B;  // stride between consecutive (x, y) coefficients
    for (int y0 = 0; y0 < NY; y0 += NYT) {
        double ar[RPT][NYT], ai[RPT][NYT];
#pragma unroll
        for (int k = 0; k < RPT; ++k)
#pragma unroll
            for (int q = 0; q < NYT; ++q) ar[k][q] = ai[k][q] = 0.0;
        for (int x = 0; x < NX; ++x) {
            double vr[RPT], vi[RPT];
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                vr[k] = vi[k] = 0.0;
                if (ok[k]) {
                    if (CPLX) {
                        const double2 v = ((const double2 *)(X + (size_t)x * stride))[ei[k]];
                        vr[k] = v.x;
                        vi[k] = v.y;
                    } else {
                        vr[k] = X[(size_t)x * stride + ei[k]];
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < NYT; ++q) {
                if (y0 + q < NY) {
                    const double c = Cb[((size_t)x * NY + y0 + q) * cs];
#pragma unroll
                    for (int k = 0; k < RPT; ++k) {
                        ar[k][q] += vr[k] * c;
                        if (CPLX) ai[k][q] += vi[k] * c;
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < NYT; ++q) {
            if (y0 + q >= NY) break;
#pragma unroll
            for (int k = 0; k < RPT; ++k) {
                if (!ok[k]) continue;
                if (CPLX)
                    ((double2 *)(Out + (size_t)(y0 + q) * stride))[ei[k]] = make_double2(ar[k][q], ai[k][q]);
                else
                    Out[(size_t)(y0 + q) * stride + ei[k]] = ar[k][q];
            }
        }
    }
}

// Dst = Src for active columns (doubles per element = dpe)
__global__ void k_masked_copy(uint64_t ne, int B, int dpe, const double *__restrict__ Src,
                              double *__restrict__ Dst, const uint8_t *__restrict__ active) {
    uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const int b = (int)(e % (uint64_t)B);
    if (active && !active[b]) return;
    for (int q = 0; q < dpe; ++q) Dst[e * dpe + q] = Src[e * dpe + q];
}

// Dst[r, j] = Src[r, idx[j]] (rows n, Bs source and Bd destination columns,
// dpe doubles per element)
__global__ void k_gather_cols(uint64_t n, int Bs, int Bd, int dpe, const double *__restrict__ Src,
                              double *__restrict__ Dst, const int32_t *__restrict__ idx) {
    uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * (uint64_t)Bd) return;
    const uint64_t r = e / (uint64_t)Bd;
    const int j = (int)(e - r * (uint64_t)Bd);
    const uint64_t se = r * (uint64_t)Bs + (uint64_t)idx[j];
    for (int q = 0; q < dpe; ++q) Dst[e * dpe + q] = Src[se * dpe + q];
}

__global__ void k_to_f32(uint64_t nd, const double *__restrict__ in, float *__restrict__ out) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nd) out[i] = (float)in[i];
}

__global__ void k_fill0(uint64_t nd, double *__restrict__ p) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nd) p[i] = 0.0;
}

// ------------------------------------------------------------------ start vectors
__global__ void k_start_u1(uint64_t D, uint64_t seed, double *__restrict__ v) {
    uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < D) v[r] = u01_pm1(splitmix64(seed, r));
}
__global__ void k_start_u1_f32(uint64_t D, uint64_t seed, float *__restrict__ v) {
    uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < D) v[r] = (float)u01_pm1(splitmix64(seed, r));
}

// union layout [u][b]; zero where the representative is incompatible with b
__global__ void k_start_batch(uint64_t n, int B, const uint64_t *__restrict__ reps,
                              const uint16_t *__restrict__ stab, const int32_t *__restrict__ nt_of,
                              const uint8_t *__restrict__ compat_nt,
                              const uint64_t *__restrict__ seeds, double2 *__restrict__ v) {
    uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * (uint64_t)B) return;
    const uint64_t u = e / B;
    const int b = (int)(e % B);
    bool ok = true;
    if (stab[u] > 1) ok = compat_nt[(size_t)nt_of[u] * B + b] != 0;
    double2 o = make_double2(0.0, 0.0);
    if (ok) {
        const uint64_t r = reps[u];
        o.x = u01_pm1(splitmix64(seeds[b], 2 * r));
        o.y = u01_pm1(splitmix64(seeds[b], 2 * r + 1));
    }
    v[e] = o;
}

__global__ void k_scatter(uint64_t d, const int64_t *__restrict__ c2u, const double2 *__restrict__ src,
                          double2 *__restrict__ dst) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d) dst[c2u[i]] = src[i];
}
__global__ void k_gather(uint64_t d, const int64_t *__restrict__ c2u, const double2 *__restrict__ src,
                         double2 *__restrict__ dst) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d) dst[i] = src[c2u[i]];
}
__global__ void k_scatter_f(uint64_t d, const int64_t *__restrict__ c2u, const float2 *__restrict__ src,
                            float2 *__restrict__ dst) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d) dst[c2u[i]] = src[i];
}
__global__ void k_gather_f(uint64_t d, const int64_t *__restrict__ c2u, const float2 *__restrict__ src,
                           float2 *__restrict__ dst) {
    uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < d) dst[i] = src[c2u[i]];
}

static inline dim3 grid1(uint64_t n, int bs = 256) { return dim3((unsigned)((n + bs - 1) / bs)); }

int start_vector_u1(qs3_sector *sec, uint64_t seed, void *v, int dtype, hipStream_t s) {
    if (sec->dim == 0) return QS3_OK;
    if (dtype == QS3_F64)
        hipLaunchKernelGGL(k_start_u1, grid1(sec->dim), dim3(256), 0, s, sec->dim, seed, (double *)v);
    else if (dtype == QS3_F32)
        hipLaunchKernelGGL(k_start_u1_f32, grid1(sec->dim), dim3(256), 0, s, sec->dim, seed, (float *)v);
    else {
        set_error("dtype of a fixed-N_down sector is QS3_F64 or QS3_F32");
        return QS3_EINVAL;
    }
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

int start_vector_batch(qs3_batch *bat, const uint64_t *seeds_dev, double *v, hipStream_t s) {
    uint64_t n = bat->ks->n_reps;
    if (n == 0) return QS3_OK;
    hipLaunchKernelGGL(k_start_batch, grid1(n * bat->B), dim3(256), 0, s, n, bat->B,
                       bat->ks->reps.as<uint64_t>(), bat->ks->stab.as<uint16_t>(),
                       bat->ks->nt_of.as<int32_t>(), bat->compat_nt.as<uint8_t>(), seeds_dev,
                       (double2 *)v);
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

int scatter_compact(qs3_sector *sec, const double *src, double *dst_union, hipStream_t s) {
    uint64_t n = sec->bat->ks->n_reps;
    hipLaunchKernelGGL(k_fill0, grid1(2 * n), dim3(256), 0, s, 2 * n, dst_union);
    if (sec->dim)
        hipLaunchKernelGGL(k_scatter, grid1(sec->dim), dim3(256), 0, s, sec->dim,
                           sec->comp2u.as<int64_t>(), (const double2 *)src, (double2 *)dst_union);
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

int gather_compact(qs3_sector *sec, const double *src_union, double *dst, hipStream_t s) {
    if (sec->dim)
        hipLaunchKernelGGL(k_gather, grid1(sec->dim), dim3(256), 0, s, sec->dim,
                           sec->comp2u.as<int64_t>(), (const double2 *)src_union, (double2 *)dst);
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

int scatter_compact_f32(qs3_sector *sec, const float *src, float *dst_union, hipStream_t s) {
    uint64_t n = sec->bat->ks->n_reps;
    hipLaunchKernelGGL(k_fill0, grid1(n), dim3(256), 0, s, n, (double *)dst_union);  // 2n floats
    if (sec->dim)
        hipLaunchKernelGGL(k_scatter_f, grid1(sec->dim), dim3(256), 0, s, sec->dim,
                           sec->comp2u.as<int64_t>(), (const float2 *)src, (float2 *)dst_union);
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

int gather_compact_f32(qs3_sector *sec, const float *src_union, float *dst, hipStream_t s) {
    if (sec->dim)
        hipLaunchKernelGGL(k_gather_f, grid1(sec->dim), dim3(256), 0, s, sec->dim,
                           sec->comp2u.as<int64_t>(), (const float2 *)src_union, (float2 *)dst);
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

// ------------------------------------------------------------------ host eigensolver
// Eigen-decomposition of a real symmetric n x n matrix A (row-major; A is
// overwritten): Householder reduction to tridiagonal form with the
// transformation accumulated, then implicit QL with Wilkinson shifts applied
// to the columns of that transformation.  e ascending, V[i * n + k] = row i
// of eigenvector k.
void sym_eig(int n, std::vector<double> &A, std::vector<double> &e, std::vector<double> &V) {
    auto a = [&](int i, int j) -> double & { return A[(size_t)i * n + j]; };
    // Z holds the transformation column-major (column j at Z + j * n), so
    // that both updates below run along contiguous columns
    std::vector<double> Z((size_t)n * n, 0.0);
    for (int i = 0; i < n; ++i) Z[(size_t)i * n + i] = 1.0;
    std::vector<double> v(n), p(n);
    for (int k = 0; k + 2 < n; ++k) {
        // reflector H = I - c v v^T on rows/columns k+1.. that zeroes a(k+2.., k)
        double tail = 0;
        for (int i = k + 2; i < n; ++i) tail += a(i, k) * a(i, k);
        if (tail == 0.0) continue;  // the column is already tridiagonal
        const double xn = std::sqrt(tail + a(k + 1, k) * a(k + 1, k));
        const double alpha = a(k + 1, k) > 0 ? -xn : xn;
        double vn = 0;
        for (int i = k + 1; i < n; ++i) {
            v[i] = a(i, k) - (i == k + 1 ? alpha : 0.0);
            vn += v[i] * v[i];
        }
        if (vn == 0.0) continue;
        const double c = 2.0 / vn;
        // trailing block: A <- A - v w^T - w v^T, p = c A v, w = p - (c v.p / 2) v
        double vp = 0;
        for (int i = k + 1; i < n; ++i) {
            double s = 0;
            for (int j = k + 1; j < n; ++j) s += a(i, j) * v[j];
            p[i] = c * s;
            vp += v[i] * p[i];
        }
        const double K2 = 0.5 * c * vp;
        for (int i = k + 1; i < n; ++i) p[i] -= K2 * v[i];
        for (int i = k + 1; i < n; ++i)
            for (int j = k + 1; j < n; ++j) a(i, j) -= v[i] * p[j] + p[i] * v[j];
        a(k + 1, k) = a(k, k + 1) = alpha;
        for (int i = k + 2; i < n; ++i) a(i, k) = a(k, i) = 0.0;
        // Z <- Z H: every row r loses c (Z_r . v) v
        std::fill(p.begin(), p.end(), 0.0);
        for (int j = k + 1; j < n; ++j) {
            const double *zj = &Z[(size_t)j * n];
            for (int r = 0; r < n; ++r) p[r] += zj[r] * v[j];
        }
        for (int j = k + 1; j < n; ++j) {
            double *zj = &Z[(size_t)j * n];
            const double cv = c * v[j];
            for (int r = 0; r < n; ++r) zj[r] -= cv * p[r];
        }
    }
    std::vector<double> d(n), sub(n, 0.0);
    for (int i = 0; i < n; ++i) d[i] = a(i, i);
    for (int i = 0; i + 1 < n; ++i) sub[i] = a(i + 1, i);
    const double eps = std::numeric_limits<double>::epsilon();
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        for (;;) {
            int m = l;
            for (; m + 1 < n; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(sub[m]) <= eps * dd) break;
            }
            if (m == l || iter++ > 90) break;
            double g = (d[l + 1] - d[l]) / (2.0 * sub[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + sub[l] / (g + std::copysign(r, g));
            double sn = 1.0, cs = 1.0, pp = 0.0;
            bool underflow = false;
            for (int i = m - 1; i >= l; --i) {
                const double f = sn * sub[i], bb = cs * sub[i];
                r = std::sqrt(f * f + g * g);
                sub[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= pp;
                    sub[m] = 0.0;
                    underflow = true;
                    break;
                }
                sn = f / r;
                cs = g / r;
                g = d[i + 1] - pp;
                r = (d[i] - g) * sn + 2.0 * cs * bb;
                pp = sn * r;
                d[i + 1] = g + pp;
                g = cs * r - bb;
                double *zi = &Z[(size_t)i * n], *zi1 = &Z[(size_t)(i + 1) * n];
                for (int k = 0; k < n; ++k) {  // the same rotation on columns i, i+1
                    const double t = zi1[k];
                    zi1[k] = sn * zi[k] + cs * t;
                    zi[k] = cs * zi[k] - sn * t;
                }
            }
            if (underflow) continue;
            d[l] -= pp;
            sub[l] = g;
            sub[m] = 0.0;
        }
    }
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] < d[y]; });
    e.resize(n);
    V.assign((size_t)n * n, 0.0);
    for (int k = 0; k < n; ++k) {
        e[k] = d[idx[k]];
        const double *zk = &Z[(size_t)idx[k] * n];
        for (int i = 0; i < n; ++i) V[(size_t)i * n + k] = zk[i];
    }
}

// ------------------------------------------------------------------ engine
Engine::~Engine() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
}

int Engine::init(qs3_ctx *c, Operator *o, int slots_, int precision_, int reorth_, hipStream_t s) {
    ctx = c;
    op = o;
    st = s;
    n = op->rows();
    B = op->cols();
    cplx = op->is_complex();
    dpe = cplx ? 2 : 1;
    ne = n * (uint64_t)B;
    stride = ne * dpe;
    slots = slots_;
    precision = precision_;
    reorth = reorth_;
    rg = red_geom(n, B);
    QS3_TRY(Psi.alloc(ctx, sizeof(double) * stride * slots));
    QS3_TRY(W.alloc(ctx, sizeof(double) * stride));
    if (precision == QS3_PREC_F32MV) QS3_TRY(X32.alloc(ctx, sizeof(float) * stride));
    const int maxJ = slots;
    QS3_TRY(partial.alloc(ctx, sizeof(double2) * (size_t)rg.nchunk * (maxJ + 1) * B));
    QS3_TRY(hvec.alloc(ctx, sizeof(double2) * (size_t)(maxJ + 1) * B));
    QS3_TRY(alpha.alloc(ctx, sizeof(double2) * (size_t)B));
    QS3_TRY(nrm2.alloc(ctx, sizeof(double2) * (size_t)B));
    QS3_TRY(ab_hist.alloc(ctx, sizeof(double) * 2 * (size_t)slots * B));
    QS3_TRY(act.alloc(ctx, 3 * (size_t)B + 16));
    if (reorth == 3) {
        QS3_TRY(om.alloc(ctx, sizeof(double) * 2 * (size_t)(slots + 1) * B));
        QS3_HIP(hipMemsetAsync(act.ptr, 0, 3 * (size_t)B + 16, st));
    }
    return QS3_OK;
}

double *Engine::slot(int j) { return Psi.as<double>() + (size_t)j * stride; }

int Engine::apply(const double *x, double *y) {
    if (precision == QS3_PREC_F32MV) {
        hipLaunchKernelGGL(k_to_f32, grid1(stride), dim3(256), 0, st, stride, x, X32.as<float>());
        QS3_HIP(hipGetLastError());
        op->set_mask(colmask);
        return op->apply_f32in(X32.as<float>(), y, st);
    }
    op->set_mask(colmask);
    return op->apply(x, y, st);
}

// Row chunking of one multi-dot launch: blocks over (row chunk, column tile,
// group of 4 outputs), about 1024 blocks in all but at least 64 row chunks
// (never more chunks than the engine's partial buffer holds).
static RedGeom dot_geom(const RedGeom &rg, int JO) {
    RedGeom g = rg;
    const int nz = (JO + 3) / 4;
    const uint64_t want = std::max<uint64_t>(64, (1024 + (uint64_t)rg.ncoltile * nz - 1) / ((uint64_t)rg.ncoltile * nz));
    uint64_t rc = std::max<uint64_t>((uint64_t)g.TR, (g.n + want - 1) / want);
    rc = (rc + g.TR - 1) / g.TR * g.TR;
    if (rc < rg.RC) rc = rg.RC;
    g.RC = rc;
    g.nchunk = (int)std::max<uint64_t>(1, (g.n + rc - 1) / rc);
    return g;
}

// Geometry of k_multidot_g with G groups of JPL outputs: TC columns (a power
// of two) x G groups x TR row lanes per block, about 2048 blocks, and chunks
// no shorter than the engine's own (so the chunk count fits its partial
// buffer).  in_lanes: TC * G <= 64, so the groups share each wavefront's
// loads of Y, P0 and P1; otherwise TC <= 64 and the groups are the waves of
// a block, which read the same lines within a short time (through L1/L2),
// with longer contiguous runs per vector.
static RedGeom dot_geom_g(const RedGeom &rg, int JO, int G, int JPL, bool in_lanes) {
    RedGeom g = rg;
    g.TC = 1;
    while (g.TC < rg.B && g.TC < 64 && (!in_lanes || g.TC * G < 64)) g.TC <<= 1;
    g.TR = 256 / (g.TC * G);
    g.ncoltile = (rg.B + g.TC - 1) / g.TC;
    const int nz = (JO + G * JPL - 1) / (G * JPL);
    const uint64_t want = std::max<uint64_t>(1, (2048 + (uint64_t)g.ncoltile * nz - 1) / ((uint64_t)g.ncoltile * nz));
    uint64_t rc = std::max<uint64_t>((uint64_t)g.TR, (g.n + want - 1) / want);
    rc = std::max<uint64_t>(rc, rg.RC);
    rc = (rc + g.TR - 1) / g.TR * g.TR;
    g.RC = rc;
    g.nchunk = (int)std::max<uint64_t>(1, (g.n + rc - 1) / rc);
    return g;
}

template <bool CPLX>
static RedGeom launch_multidot(const RedGeom &rg, hipStream_t st, const double *X, uint64_t stride, int J,
                               int selfdot, const double *Y, const ThreeTerm &f, const uint8_t *mask,
                               double2 *partial, bool dense) {
    const int JO = J + selfdot;
    constexpr int JPL = 8;
    // Few outputs, vectors small enough for the caches to serve the
    // per-group re-reads of Y, or a mask that may leave only a few columns
    // (a second or partial Gram-Schmidt pass, where short row chunks keep
    // the few active threads' loops short): groups of 4 outputs, each block
    // group re-reading Y.  Otherwise vectors beyond the last-level cache
    // (256 MB) share loads inside a wavefront, smaller ones across the
    // waves of a block.
    const uint64_t elems = rg.n * (uint64_t)rg.B;
    if (JO <= 4 || elems < (1ull << 20) || !dense) {
        const RedGeom g = dot_geom(rg, JO);
        dim3 grid(g.nchunk, g.ncoltile, (JO + 3) / 4);
        hipLaunchKernelGGL((k_multidot<CPLX, 4>), grid, dim3(256), 0, st, g, X, stride, J, selfdot, Y, f, mask,
                           partial);
        return g;
    }
    const int G = JO <= JPL ? 1 : (JO <= 2 * JPL ? 2 : 4);
    const bool in_lanes = elems * (CPLX ? 16 : 8) > (256ull << 20);
    const RedGeom g = dot_geom_g(rg, JO, G, JPL, in_lanes);
    dim3 grid(g.nchunk, g.ncoltile, (JO + G * JPL - 1) / (G * JPL));
    if (G == 1)
        hipLaunchKernelGGL((k_multidot_g<CPLX, 1, JPL>), grid, dim3(256), 0, st, g, X, stride, J, selfdot, Y, f,
                           mask, partial);
    else if (G == 2)
        hipLaunchKernelGGL((k_multidot_g<CPLX, 2, JPL>), grid, dim3(256), 0, st, g, X, stride, J, selfdot, Y, f,
                           mask, partial);
    else
        hipLaunchKernelGGL((k_multidot_g<CPLX, 4, JPL>), grid, dim3(256), 0, st, g, X, stride, J, selfdot, Y, f,
                           mask, partial);
    return g;
}

int Engine::multidot(const double *X, int J, const double *Y, double2 *out, int selfdot,
                     const uint8_t *mask, const ThreeTerm *f, double *re_out) {
    const ThreeTerm none{};
    // the first pass of a step (the one with the three-term part) takes
    // every column still iterating
    const bool dense = f != nullptr;
    const RedGeom g = cplx ? launch_multidot<true>(rg, st, X, stride, J, selfdot, Y, f ? *f : none, mask,
                                                   partial.as<double2>(), dense)
                           : launch_multidot<false>(rg, st, X, stride, J, selfdot, Y, f ? *f : none, mask,
                                                    partial.as<double2>(), dense);
    QS3_HIP(hipGetLastError());
    const int JB = (J + selfdot) * B;
    hipLaunchKernelGGL(k_reduce_chunks, dim3((JB + 3) / 4), dim3(256), 0, st, partial.as<double2>(),
                       g.nchunk, JB, out, re_out);
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

int Engine::cgs_update_norm(int J, const double2 *h, const uint8_t *mask, double2 *nrm_out,
                            const ThreeTerm *f, const double2 *dgks_before, uint8_t *dgks_flag) {
    dim3 grid(rg.nchunk, rg.ncoltile);
    const ThreeTerm none{};
    if (cplx)
        hipLaunchKernelGGL((k_cgs_update_norm<true>), grid, dim3(256), 0, st, rg, W.as<double>(), slot(0),
                           stride, J, h, f ? *f : none, mask, partial.as<double2>());
    else
        hipLaunchKernelGGL((k_cgs_update_norm<false>), grid, dim3(256), 0, st, rg, W.as<double>(), slot(0),
                           stride, J, h, f ? *f : none, mask, partial.as<double2>());
    QS3_HIP(hipGetLastError());
    if (dgks_flag)
        hipLaunchKernelGGL(k_reduce_norm_dgks, dim3((B + 3) / 4), dim3(256), 0, st, partial.as<double2>(),
                           rg.nchunk, B, nrm_out, dgks_before, mask, dgks_flag);
    else
        hipLaunchKernelGGL(k_reduce_chunks, dim3((B + 3) / 4), dim3(256), 0, st, partial.as<double2>(), rg.nchunk,
                           B, nrm_out, (double *)nullptr);
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

// One Lanczos step: slot x holds psi_x (normalised); writes alpha_x, beta_x and
// psi_{x+1} into slot x+1.  prev: slot of psi_{x-1} or -1.  Full
// reorthogonalisation against slots 0..x by classical Gram-Schmidt, with a
// second pass only for the columns whose first pass cancelled more than half
// of |W|^2; the norm is fused into the update.
int Engine::step(int x, int prev) {
    QS3_TRY(apply(slot(x), W.as<double>()));
    // alpha_x, its real part also into the coefficient history
    QS3_TRY(multidot(slot(x), 1, W.as<double>(), alpha.as<double2>(), 0, colmask, nullptr,
                     ab_hist.as<double>() + (size_t)x * B));
    double *betap = ab_hist.as<double>() + (size_t)slots * B + (size_t)(prev < 0 ? 0 : prev) * B;
    double *beta_x = ab_hist.as<double>() + (size_t)slots * B + (size_t)x * B;
    bool have_beta = false;  // beta_x written by a merge below
    double2 *h = hvec.as<double2>();
    double2 *n_before = h + (size_t)(x + 1) * B;  // the self-dot output of the first pass
    if (reorth == 1 || reorth == 2) {
        // W' = W - alpha psi_x - beta psi_prev is formed on the fly inside
        // the first Gram-Schmidt pass (dots) and its update (stored there)
        ThreeTerm f;
        f.P0 = slot(x);
        f.P1 = prev >= 0 ? slot(prev) : nullptr;
        f.alpha = alpha.as<double2>();
        f.beta = betap;
        f.i0 = x;  // P0 and P1 are slots x and prev of the basis the passes read
        f.i1 = prev;
        QS3_TRY(multidot(slot(0), x + 1, W.as<double>(), h, 1, colmask, &f));
        uint8_t *flag = act.as<uint8_t>() + 8 + B;
        // the norm's reduction also sets the second-pass flags
        QS3_TRY(cgs_update_norm(x + 1, h, colmask, nrm2.as<double2>(), &f, n_before, reorth > 1 ? flag : nullptr));
        if (reorth > 1) {
            QS3_TRY(multidot(slot(0), x + 1, W.as<double>(), h, 0, flag));
            double2 *n2 = h + (size_t)(x + 1) * B;
            QS3_TRY(cgs_update_norm(x + 1, h, flag, n2));
            hipLaunchKernelGGL(k_merge_sqrt, grid1(B), dim3(256), 0, st, B, flag, n2, nrm2.as<double2>(), beta_x);
            QS3_HIP(hipGetLastError());
            have_beta = true;
        }
    } else {
        // three-term recurrence (and with reorth == 3 the partial
        // reorthogonalisation below)
        if (cplx)
            hipLaunchKernelGGL(k_lanczos_update<true>, grid1(ne), dim3(256), 0, st, ne, B,
                               W.as<double>(), slot(x), prev >= 0 ? slot(prev) : nullptr,
                               alpha.as<double2>(), betap, colmask);
        else
            hipLaunchKernelGGL(k_lanczos_update<false>, grid1(ne), dim3(256), 0, st, ne, B,
                               W.as<double>(), slot(x), prev >= 0 ? slot(prev) : nullptr,
                               alpha.as<double2>(), betap, colmask);
        QS3_HIP(hipGetLastError());
        QS3_TRY(multidot(W.as<double>(), 1, W.as<double>(), nrm2.as<double2>(), 0, colmask));
        if (reorth == 3) {
            uint8_t *flag = act.as<uint8_t>() + 8 + B, *force = act.as<uint8_t>() + 8 + 2 * B;
            const double eps1 = 2.220446049250313e-16 * std::sqrt((double)n);
            hipLaunchKernelGGL(k_omega, grid1(B), dim3(256), 0, st, B, x, ab_hist.as<double>(), slots,
                               nrm2.as<double2>(), om.as<double>(), slots + 1, colmask, force, flag, eps1);
            QS3_HIP(hipGetLastError());
            double2 *h = hvec.as<double2>();
            QS3_TRY(multidot(slot(0), x + 1, W.as<double>(), h, 0, flag));
            double2 *n2 = h + (size_t)(x + 1) * B;
            QS3_TRY(cgs_update_norm(x + 1, h, flag, n2));
            hipLaunchKernelGGL(k_merge_sqrt, grid1(B), dim3(256), 0, st, B, flag, n2, nrm2.as<double2>(), beta_x);
            QS3_HIP(hipGetLastError());
            have_beta = true;
        }
    }
    if (!have_beta)
        hipLaunchKernelGGL(k_sqrt_to, grid1(B), dim3(256), 0, st, B, nrm2.as<double2>(), beta_x);
    if (cplx)
        hipLaunchKernelGGL(k_scale_out<true>, grid1(ne), dim3(256), 0, st, ne, B, W.as<double>(),
                           slot(x + 1), nrm2.as<double2>(), colmask);
    else
        hipLaunchKernelGGL(k_scale_out<false>, grid1(ne), dim3(256), 0, st, ne, B, W.as<double>(),
                           slot(x + 1), nrm2.as<double2>(), colmask);
    QS3_HIP(hipGetLastError());
    ++n_matvec;
    return QS3_OK;
}

// Small single-column sectors run a whole cycle in one workgroup (one launch
// instead of ~15 per step) while their Krylov basis fits comfortably in L2.
int Engine::cycle(int x0, int x1, int prev_first) {
    const size_t basis_bytes = sizeof(double) * stride * (size_t)slots;
    if (B == 1 && precision == QS3_PREC_F64 && basis_bytes <= (2u << 20)) {
        const int rc = op->small_cycle(*this, x0, x1, prev_first);
        if (rc != 1) {
            if (rc == QS3_OK) n_matvec += x1 - x0;
            return rc;
        }
    }
    for (int x = x0; x < x1; ++x) QS3_TRY(step(x, x == x0 ? prev_first : x - 1));
    return QS3_OK;
}

static SmallArgs small_args(Engine &E, int x0, int x1, int prev_first) {
    SmallArgs S;
    S.n = E.n;
    S.x0 = x0;
    S.x1 = x1;
    S.prev_first = prev_first;
    S.Psi = E.Psi.as<double>();
    S.stride = E.stride;
    S.W = E.W.as<double>();
    S.ab = E.ab_hist.as<double>();
    S.slots = E.slots;
    S.reorth = E.reorth;
    return S;
}

int small_cycle_u1(qs3_sector *sec, Engine &E, int x0, int x1, int prev_first) {
    return lanczos_small(sec->lat, sec->K, sec->bt.get(), nullptr, small_args(E, x0, x1, prev_first), E.st);
}

int small_cycle_batch(qs3_batch *bat, Engine &E, int x0, int x1, int prev_first) {
    return lanczos_small(bat->lat, bat->K, bat->bt.get(), bat, small_args(E, x0, x1, prev_first), E.st);
}

// slot 0 := v0 / |v0|; norms0[b] = |v0|
int Engine::normalize_into_slot0(const double *v0, std::vector<double> *norms0) {
    QS3_TRY(multidot(v0, 1, v0, nrm2.as<double2>(), 0, nullptr));
    if (cplx)
        hipLaunchKernelGGL(k_scale_out<true>, grid1(ne), dim3(256), 0, st, ne, B, v0, slot(0),
                           nrm2.as<double2>(), nullptr);
    else
        hipLaunchKernelGGL(k_scale_out<false>, grid1(ne), dim3(256), 0, st, ne, B, v0, slot(0),
                           nrm2.as<double2>(), nullptr);
    QS3_HIP(hipGetLastError());
    if (norms0) {
        std::vector<double2> h(B);
        QS3_HIP(hipMemcpyAsync(h.data(), nrm2.ptr, sizeof(double2) * B, hipMemcpyDeviceToHost, st));
        QS3_HIP(hipStreamSynchronize(st));
        norms0->resize(B);
        for (int b = 0; b < B; ++b) (*norms0)[b] = std::sqrt(std::max(h[b].x, 0.0));
    }
    return QS3_OK;
}

int Engine::read_ab(int x0, int x1, std::vector<double> &a, std::vector<double> &bb) {
    // a[x * B + b], bb[x * B + b] for x in [x0, x1)
    int cnt = x1 - x0;
    a.resize((size_t)slots * B);
    bb.resize((size_t)slots * B);
    if (cnt <= 0) return QS3_OK;
    QS3_HIP(hipMemcpyAsync(a.data() + (size_t)x0 * B, ab_hist.as<double>() + (size_t)x0 * B,
                           sizeof(double) * cnt * B, hipMemcpyDeviceToHost, st));
    QS3_HIP(hipMemcpyAsync(bb.data() + (size_t)x0 * B,
                           ab_hist.as<double>() + (size_t)slots * B + (size_t)x0 * B,
                           sizeof(double) * cnt * B, hipMemcpyDeviceToHost, st));
    QS3_HIP(hipStreamSynchronize(st));
    return QS3_OK;
}

template <int NYT>
static void launch_rotate(bool cplx, dim3 grid, hipStream_t st, uint64_t ne, int B, const double *X, uint64_t stride,
                          int NX, const double *dC, int NY, double *out, const uint8_t *act) {
    if (cplx)
        hipLaunchKernelGGL((k_rotate<true, NYT, 2>), grid, dim3(256), 0, st, ne, B, X, stride, NX, dC, NY, out, act);
    else
        hipLaunchKernelGGL((k_rotate<false, NYT, 2>), grid, dim3(256), 0, st, ne, B, X, stride, NX, dC, NY, out, act);
}

int Engine::rotate_dev(int from_slot, int NX, const double *dC, int NY, int to_slot, const uint8_t *act_dev) {
    // two rows per thread; the accumulator tile is the smallest of 8, 12, 16
    // outputs that holds NY (fewer registers, more waves in flight)
    const uint64_t part = (n + 1) / 2 * (uint64_t)B;
    const dim3 grid = grid1(part);
    if (NY <= 8)
        launch_rotate<8>(cplx, grid, st, ne, B, slot(from_slot), stride, NX, dC, NY, slot(to_slot), act_dev);
    else if (NY <= 12)
        launch_rotate<12>(cplx, grid, st, ne, B, slot(from_slot), stride, NX, dC, NY, slot(to_slot), act_dev);
    else
        launch_rotate<16>(cplx, grid, st, ne, B, slot(from_slot), stride, NX, dC, NY, slot(to_slot), act_dev);
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

int Engine::copy_slot_dev(int from, int to, const uint8_t *act_dev) {
    hipLaunchKernelGGL(k_masked_copy, grid1(ne), dim3(256), 0, st, ne, B, dpe, slot(from), slot(to), act_dev);
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

int Engine::gather_columns_into(Engine &dst, int from_slot, int to_slot, const int32_t *idx_dev) {
    const uint64_t cnt = n * (uint64_t)dst.B;
    hipLaunchKernelGGL(k_gather_cols, grid1(cnt), dim3(256), 0, st, n, B, dst.B, dpe, slot(from_slot),
                       dst.slot(to_slot), idx_dev);
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

void Engine::release() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
    for (DevBuf *b : {&Psi, &W, &X32, &partial, &hvec, &alpha, &nrm2, &ab_hist, &act, &om}) b->release();
}

int Engine::cycle_replay(int x0, int x1, int prev_first) {
    if (!ctx->use_graphs || st == nullptr) return cycle(x0, x1, prev_first);
    if (gexec && g_x0 == x0 && g_x1 == x1 && g_pf == prev_first && g_mask == colmask) {
        QS3_HIP(hipGraphLaunch(gexec, st));
        n_matvec += x1 - x0;
        ++graph_launches;
        return QS3_OK;
    }
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
    // capture records the launches without running them (and counts the
    // steps once); the graph then runs them
    QS3_HIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    const int rc = cycle(x0, x1, prev_first);
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(st, &graph);
    if (rc != QS3_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    QS3_HIP(ec);
    const hipError_t ei = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    QS3_HIP(ei);
    g_x0 = x0;
    g_x1 = x1;
    g_pf = prev_first;
    g_mask = colmask;
    QS3_HIP(hipGraphLaunch(gexec, st));
    ++graph_launches;
    return QS3_OK;
}

// ------------------------------------------------------------------ host-side solver logic
static void build_tri(int m, const double *a, const double *b, std::vector<double> &T) {
    T.assign((size_t)m * m, 0.0);
    for (int i = 0; i < m; ++i) {
        T[(size_t)i * m + i] = a[i];
        if (i + 1 < m) T[(size_t)i * m + i + 1] = T[(size_t)(i + 1) * m + i] = b[i];
    }
}

// The lowest `nev` distinct levels (indices into the ascending e).  A Ritz
// value has converged when its residual |beta_m c_{m,i}| is at most
// tol * min(max(1, |e_i|), max(1, spread)), spread = the width of the Ritz
// spectrum: the scale does not grow with a constant offset of H (the Ising
// energy of the ferromagnet dominates |e| near saturation), so a level cannot
// pass while its Ritz vector still mixes with a partner split by more than
// about tol * spread.  Ritz values within cluster * max(1, |e|) of the
// previous level belong to it (partner copies of a degenerate level, which
// rounding lets emerge, are ignored whether or not they have converged):
// 1e-10 for float64 products, 1e-6 for float32 ones (whose rounding splits a
// degenerate level by about 1e-8).
// require_conv (fixed-step Lanczos, which cannot iterate further):
// unconverged values are skipped.
static std::vector<int> pick_levels(const std::vector<double> &e, const std::vector<double> &res,
                                    int nev, double tol, double spread, double cluster,
                                    bool require_conv, bool *all_conv) {
    std::vector<int> out;
    *all_conv = true;
    double last = 0.0;
    const double ssc = std::max(1.0, spread);
    for (size_t i = 0; i < e.size() && (int)out.size() < nev; ++i) {
        const double sc = std::max(1.0, std::fabs(e[i]));
        const bool conv = res[i] <= tol * std::min(sc, ssc);
        if (require_conv && !conv) continue;
        if (!out.empty() && std::fabs(e[i] - last) <= cluster * sc) continue;
        out.push_back((int)i);
        last = e[i];
        if (!conv) *all_conv = false;
    }
    if ((int)out.size() < nev) *all_conv = false;
    return out;
}

static double cluster_rel(const qs3_eigs_opts &o) { return o.precision == QS3_PREC_F32MV ? 1e-6 : 1e-10; }

// Eigenvalues of the symmetric tridiagonal matrix (diagonal d, off-diagonal
// e[i] coupling i and i+1) by the implicit QL algorithm with Wilkinson-type
// shifts (Bowdler, Martin, Reinsch and Wilkinson 1968), tracking rows
// `first` and `last` of the eigenvector matrix through the plane rotations.
// Outputs ascending eigenvalues w and the matching components z0 (row 0) and
// zl (row n-1).
static void tridiag_ql(int n, const double *d_in, const double *e_in, std::vector<double> &w,
                       std::vector<double> &z0, std::vector<double> &zl) {
    std::vector<double> d(d_in, d_in + n), e(n, 0.0), a(n, 0.0), b(n, 0.0);
    for (int i = 0; i + 1 < n; ++i) e[i] = e_in[i];
    a[0] = 1.0;
    b[n - 1] = 1.0;
    const double eps = std::numeric_limits<double>::epsilon();
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        for (;;) {
            int m = l;
            for (; m + 1 < n; ++m) {
                const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
                if (std::fabs(e[m]) <= eps * dd) break;
            }
            if (m == l || iter++ > 90) break;
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = std::hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
            double sn = 1.0, cs = 1.0, p = 0.0;
            int i = m - 1;
            bool underflow = false;
            for (; i >= l; --i) {
                const double f = sn * e[i], bb = cs * e[i];
                // f and g are bounded by the norm of T (Lanczos coefficients):
                // their squares cannot overflow, and the plain square root
                // avoids hypot's scaling (a third of the routine's time)
                r = std::sqrt(f * f + g * g);
                e[i + 1] = r;
                if (r == 0.0) {
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    underflow = true;
                    break;
                }
                sn = f / r;
                cs = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * sn + 2.0 * cs * bb;
                p = sn * r;
                d[i + 1] = g + p;
                g = cs * r - bb;
                // the same rotation on the tracked rows of the eigenvector matrix
                double t = a[i + 1];
                a[i + 1] = sn * a[i] + cs * t;
                a[i] = cs * a[i] - sn * t;
                t = b[i + 1];
                b[i + 1] = sn * b[i] + cs * t;
                b[i] = cs * b[i] - sn * t;
            }
            if (underflow) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
    }
    std::vector<int> idx(n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int x, int y) { return d[x] < d[y]; });
    w.resize(n);
    z0.resize(n);
    zl.resize(n);
    for (int k = 0; k < n; ++k) {
        w[k] = d[idx[k]];
        z0[k] = a[idx[k]];
        zl[k] = b[idx[k]];
    }
}

// Eigenvector of the tridiagonal matrix for the eigenvalue lam by two steps
// of inverse iteration (LU with partial pivoting of T - (lam + delta) I).
static void tridiag_vector(int n, const double *d, const double *e, double lam, double *x) {
    double nrm = 0;
    for (int i = 0; i < n; ++i) nrm = std::max(nrm, std::fabs(d[i]) + (i + 1 < n ? std::fabs(e[i]) : 0.0) +
                                                   (i > 0 ? std::fabs(e[i - 1]) : 0.0));
    const double shift = lam + 1e-13 * std::max(nrm, 1.0);
    std::vector<double> a(n), bu(n), c2(n), l(n);  // U: diag a, super bu, super-super c2
    std::vector<int> piv(n, 0);
    std::vector<double> sub(n), dia(n), sup(n);
    for (int i = 0; i < n; ++i) {
        dia[i] = d[i] - shift;
        sup[i] = i + 1 < n ? e[i] : 0.0;
        sub[i] = i + 1 < n ? e[i] : 0.0;  // sub[i] = T[i+1][i]
    }
    // Gaussian elimination with row interchanges on the band
    for (int i = 0; i < n; ++i) {
        a[i] = dia[i];
        bu[i] = sup[i];
        c2[i] = 0.0;
    }
    for (int i = 0; i + 1 < n; ++i) {
        // rows i and i+1: row i = (a[i], bu[i], c2[i]) at cols (i, i+1, i+2); row i+1 = (sub[i], dia, sup)
        double r0 = a[i], r1 = bu[i], r2 = c2[i];
        double s0 = sub[i], s1 = a[i + 1], s2 = bu[i + 1];
        if (std::fabs(s0) > std::fabs(r0)) {
            std::swap(r0, s0);
            std::swap(r1, s1);
            std::swap(r2, s2);
            piv[i] = 1;
        }
        const double m = r0 != 0.0 ? s0 / r0 : 0.0;
        l[i] = m;
        a[i] = r0;
        bu[i] = r1;
        c2[i] = r2;
        a[i + 1] = s1 - m * r1;
        bu[i + 1] = s2 - m * r2;
    }
    for (int i = 0; i < n; ++i)
        if (a[i] == 0.0) a[i] = 1e-300;
    for (int i = 0; i < n; ++i) x[i] = 1.0;
    for (int it = 0; it < 3; ++it) {
        for (int i = 0; i + 1 < n; ++i) {  // forward: apply the row interchanges and multipliers
            if (piv[i]) std::swap(x[i], x[i + 1]);
            x[i + 1] -= l[i] * x[i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = x[i];
            if (i + 1 < n) s -= bu[i] * x[i + 1];
            if (i + 2 < n) s -= c2[i] * x[i + 2];
            x[i] = s / a[i];
        }
        double nn = 0;
        for (int i = 0; i < n; ++i) nn += x[i] * x[i];
        nn = std::sqrt(nn);
        for (int i = 0; i < n; ++i) x[i] /= nn;
    }
}

// Run f(c) for c in [0, n) on a few host threads (the per-column host work of
// a batch: eigensolves of small tridiagonal / arrowhead matrices).
template <typename F>
static void parallel_columns(int n, F &&f) {
    // about 25 us of host work per column (a 20 x 20 restart eigenproblem):
    // one thread per 16 columns keeps the thread start-up below the work
    const int nt = std::min(16, std::max(1, n / 16));
    if (nt <= 1) {
        for (int c = 0; c < n; ++c) f(c);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
            for (int c = t; c < n; c += nt) f(c);
        });
    for (auto &x : th) x.join();
}

int run_lanczos(Engine &E, const double *v0, int steps, std::vector<double> &a_out,
                std::vector<double> &b_out, std::vector<double> &norm0, std::vector<int> &done) {
    const int B = E.B;
    QS3_TRY(E.normalize_into_slot0(v0, &norm0));
    QS3_TRY(E.cycle(0, steps, -1));
    std::vector<double> a, b;
    QS3_TRY(E.read_ab(0, steps, a, b));
    a_out.assign((size_t)B * steps, 0.0);
    b_out.assign((size_t)B * steps, 0.0);
    done.assign(B, steps);
    for (int c = 0; c < B; ++c) {
        for (int x = 0; x < steps; ++x) {
            a_out[(size_t)c * steps + x] = a[(size_t)x * B + c];
            b_out[(size_t)c * steps + x] = b[(size_t)x * B + c];
        }
        for (int x = 0; x < steps; ++x) {
            const double sc = std::max(1.0, std::fabs(a_out[(size_t)c * steps + x]));
            if (b_out[(size_t)c * steps + x] <= 1e-14 * sc) {
                done[c] = x + 1;
                break;
            }
        }
    }
    return QS3_OK;
}

// ------------------------------------------------------------------ resumable solver
template <typename T>
static int pinned(qs3_ctx *c, T **p, size_t n, size_t *cap) {
    void *q = nullptr;
    QS3_TRY(pinned_get(c, sizeof(T) * n, &q, cap));
    *p = (T *)q;
    return QS3_OK;
}

SolveRun::~SolveRun() {
    if (ev) (void)hipEventDestroy(ev);
    // no copy through the host buffers may still be queued when they go
    // back to the pool (an error can end a run mid-cycle)
    if (pctx) {
        (void)hipStreamSynchronize(root.st);
        pinned_put(pctx, hab, cap_hab);
        pinned_put(pctx, hC, cap_hC);
        pinned_put(pctx, hact, cap_hact);
        pinned_put(pctx, hidx, cap_hidx);
    }
}

int SolveRun::slots_for(const qs3_eigs_opts &o) {
    // thick restart: N_M + 1 basis vectors, plus N_K staging slots for the
    // rotation only when it cannot run in place (N_K > 16)
    return o.alg == QS3_ALG_TRL ? o.nm + 1 + (o.nk > 16 ? o.nk : 0) : o.steps + 1 + o.nev;
}

int SolveRun::init(qs3_ctx *ctx, Operator *op, const qs3_eigs_opts &opts, hipStream_t s) {
    o = opts;
    QS3_TRY(root.init(ctx, op, slots_for(o), o.precision, engine_reorth(o.reorth, o.alg == QS3_ALG_TRL), s));
    B = root.B;
    const int NX = o.alg == QS3_ALG_TRL ? o.nm : o.steps;
    const int NY = o.alg == QS3_ALG_TRL ? o.nk : o.nev;
    pctx = ctx;
    QS3_TRY(pinned(ctx, &hab, 2 * (size_t)root.slots * B, &cap_hab));
    QS3_TRY(pinned(ctx, &hC, (size_t)B * NX * NY, &cap_hC));
    QS3_TRY(pinned(ctx, &hact, 2 * (size_t)B, &cap_hact));
    QS3_TRY(pinned(ctx, &hidx, (size_t)B, &cap_hidx));
    QS3_TRY(dC.alloc(ctx, sizeof(double) * (size_t)B * NX * NY));
    QS3_TRY(dact.alloc(ctx, 2 * (size_t)B));
    QS3_TRY(didx.alloc(ctx, sizeof(int32_t) * (size_t)B));
    QS3_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    evals.assign((size_t)B * o.nev, std::numeric_limits<double>::quiet_NaN());
    info.assign(B, qs3_eigs_info{});
    active.assign(B, 1);
    final_lv.assign(B, {});
    return QS3_OK;
}

// alpha/beta of steps x0..x1-1 of the current engine into hab ([x][column],
// the current engine's column count), then the event
int SolveRun::enqueue_ab_copy(int x0, int x1) {
    Engine &E = eng();
    const int Bc = E.B;
    const int cnt = x1 - x0;
    if (cnt > 0) {
        QS3_HIP(hipMemcpyAsync(hab + (size_t)x0 * Bc, E.ab_hist.as<double>() + (size_t)x0 * Bc,
                               sizeof(double) * cnt * Bc, hipMemcpyDeviceToHost, E.st));
        QS3_HIP(hipMemcpyAsync(hab + (size_t)E.slots * Bc + (size_t)x0 * Bc,
                               E.ab_hist.as<double>() + (size_t)E.slots * Bc + (size_t)x0 * Bc,
                               sizeof(double) * cnt * Bc, hipMemcpyDeviceToHost, E.st));
    }
    QS3_HIP(hipEventRecord(ev, E.st));
    return QS3_OK;
}

bool SolveRun::ready() const { return hipEventQuery(ev) == hipSuccess; }

int SolveRun::wait() {
    QS3_HIP(hipEventSynchronize(ev));
    return QS3_OK;
}

int SolveRun::begin(const double *v0) {
    QS3_TRY(root.normalize_into_slot0(v0, nullptr));
    const int steps = o.alg == QS3_ALG_TRL ? o.nm : o.steps;
    QS3_TRY(root.cycle(0, steps, -1));
    QS3_TRY(enqueue_ab_copy(0, steps));
    phase = 1;
    if (o.alg == QS3_ALG_TRL) {
        al.assign(B, std::vector<double>(o.nm));
        be.assign(B, std::vector<double>(o.nm));
        coup.assign(B, std::vector<double>(o.nk, 0.0));
    }
    return QS3_OK;
}

// Moves the columns with keep[j] != 0 into a new engine over the operator
// restricted to them: the kept Ritz vectors (slots 0..NK-1) and the residual
// (slot NM) become slots 0..NK of the new engine.  *compacted = false when
// the operator has no restriction (the run then goes on with masks).
int SolveRun::compact(const uint8_t *keep, bool *compacted) {
    *compacted = false;
    Engine &E = eng();
    std::vector<int> sel;
    for (int j = 0; j < E.B; ++j)
        if (keep[j]) sel.push_back(j);
    if (sel.empty()) return QS3_OK;
    std::unique_ptr<Operator> nop;
    const int rc = E.op->subset(sel, &nop);
    if (rc == 1 || !nop) return QS3_OK;
    QS3_TRY(rc);
    auto ne = std::make_unique<Engine>();
    QS3_TRY(ne->init(E.ctx, nop.get(), E.slots, E.precision, E.reorth, E.st));
    ne->n_matvec = E.n_matvec;
    const int nb = (int)sel.size();
    for (int j = 0; j < nb; ++j) hidx[j] = sel[j];
    QS3_HIP(hipMemcpyAsync(didx.ptr, hidx, sizeof(int32_t) * nb, hipMemcpyHostToDevice, E.st));
    const int NK = o.nk, NM = o.nm;
    for (int y = 0; y < NK; ++y) QS3_TRY(E.gather_columns_into(*ne, y, y, didx.as<int32_t>()));
    QS3_TRY(E.gather_columns_into(*ne, NM, NK, didx.as<int32_t>()));
    std::vector<int> nmap(nb);
    for (int j = 0; j < nb; ++j) nmap[j] = col(sel[j]);
    // the previous engine's memory is released below: let the copies finish
    QS3_HIP(hipStreamSynchronize(E.st));
    graph_prev += E.graph_launches;
    if (!narrow) root.release();
    narrow = std::move(ne);
    narrow_op = std::move(nop);
    cmap = std::move(nmap);
    *compacted = true;
    return QS3_OK;
}

int SolveRun::advance(bool *done) {
    *done = false;
    if (phase == 4) {
        *done = true;
        return QS3_OK;
    }
    Engine &E = eng();
    const int Bc = E.B;
    const double *ha = hab, *hb = hab + (size_t)E.slots * Bc;
    if (o.alg == QS3_ALG_LANCZOS) {
        if (phase == 3) {
            phase = 4;
            *done = true;
            return QS3_OK;
        }
        const int S = o.steps, nev = o.nev;
        std::fill(hC, hC + (size_t)B * S * nev, 0.0);
        parallel_columns(B, [&](int c) {
            int m = S;
            for (int x = 0; x < S; ++x)
                if (hb[(size_t)x * B + c] <= 1e-14 * std::max(1.0, std::fabs(ha[(size_t)x * B + c]))) {
                    m = x + 1;
                    break;
                }
            std::vector<double> a(m), b(m), e, z0, zl;
            for (int x = 0; x < m; ++x) {
                a[x] = ha[(size_t)x * B + c];
                b[x] = hb[(size_t)x * B + c];
            }
            tridiag_ql(m, a.data(), b.data(), e, z0, zl);
            std::vector<double> res(m);
            for (int i = 0; i < m; ++i) res[i] = std::fabs(b[m - 1] * zl[i]);
            bool allc;
            auto lv = pick_levels(e, res, nev, o.tol, e.back() - e.front(), cluster_rel(o), true, &allc);
            // a Krylov space that closed (breakdown) or spans every row holds
            // all the levels the start vector reaches: fewer than nev is final
            const bool exhausted = m < S || (uint64_t)S >= E.n;
            if (exhausted && !lv.empty()) allc = true;
            double mr = 0;
            std::vector<double> vec(m);
            for (size_t y = 0; y < lv.size(); ++y) {
                evals[(size_t)c * nev + y] = e[lv[y]];
                mr = std::max(mr, res[lv[y]]);
                if (want_vecs) {
                    tridiag_vector(m, a.data(), b.data(), e[lv[y]], vec.data());
                    for (int x = 0; x < m; ++x) hC[((size_t)x * nev + y) * B + c] = vec[x];
                }
            }
            info[c].converged = allc ? 1 : 0;
            info[c].n_found = (int)lv.size();
            info[c].max_residual = mr;
            info[c].n_matvec = E.n_matvec;
            info[c].width = B;
        });
        if (want_vecs) {
            QS3_HIP(hipMemcpyAsync(dC.ptr, hC, sizeof(double) * (size_t)B * S * nev, hipMemcpyHostToDevice, E.st));
            QS3_TRY(E.rotate_dev(0, S, dC.as<double>(), nev, S + 1, nullptr));
            QS3_HIP(hipEventRecord(ev, E.st));
            phase = 3;
            return QS3_OK;
        }
        phase = 4;
        *done = true;
        return QS3_OK;
    }
    // ---- thick restart (Alg. 10); j indexes the current engine's columns,
    // c = col(j) the sector
    const int NK = o.nk, NM = o.nm, nev = o.nev;
    const int x0 = first ? 0 : NK;
    for (int j = 0; j < Bc; ++j) {
        const int c = col(j);
        for (int x = x0; x < NM; ++x) {
            al[c][x] = ha[(size_t)x * Bc + j];
            be[c][x] = hb[(size_t)x * Bc + j];
        }
    }
    uint8_t *act_rot = hact, *act_next = hact + Bc;
    for (int j = 0; j < Bc; ++j) act_rot[j] = active[col(j)];
    parallel_columns(Bc, [&](int j) {
        const int c = col(j);
        if (!active[c]) return;
        std::vector<double> T((size_t)NM * NM, 0.0), e, V;
        for (int x = 0; x < NM; ++x) T[(size_t)x * NM + x] = al[c][x];
        if (first) {
            for (int x = 0; x + 1 < NM; ++x) T[(size_t)x * NM + x + 1] = T[(size_t)(x + 1) * NM + x] = be[c][x];
        } else {
            for (int y = 0; y < NK; ++y) T[(size_t)y * NM + NK] = T[(size_t)NK * NM + y] = coup[c][y];
            for (int z = NK; z + 1 < NM; ++z) T[(size_t)z * NM + z + 1] = T[(size_t)(z + 1) * NM + z] = be[c][z];
        }
        sym_eig(NM, T, e, V);
        const double bm = be[c][NM - 1];
        std::vector<double> res(NM);
        for (int i = 0; i < NM; ++i) res[i] = std::fabs(bm * V[(size_t)(NM - 1) * NM + i]);
        bool allc;
        auto lv = pick_levels(std::vector<double>(e.begin(), e.begin() + NK),
                              std::vector<double>(res.begin(), res.begin() + NK), nev, o.tol,
                              e.back() - e.front(), cluster_rel(o), false, &allc);
        for (int x = 0; x < NM; ++x)
            for (int y = 0; y < NK; ++y) hC[((size_t)x * NK + y) * Bc + j] = V[(size_t)x * NM + y];
        for (int y = 0; y < NK; ++y) {
            coup[c][y] = bm * V[(size_t)(NM - 1) * NM + y];
            al[c][y] = e[y];
        }
        double mr = 0;
        for (size_t y = 0; y < lv.size(); ++y) {
            evals[(size_t)c * nev + y] = e[lv[y]];
            mr = std::max(mr, res[lv[y]]);
        }
        info[c].n_found = (int)lv.size();
        info[c].max_residual = mr;
        info[c].n_restarts = restarts;
        info[c].n_matvec = E.n_matvec;
        info[c].width = Bc;
        info[c].graph_cycles = graph_prev + E.graph_launches;
        final_lv[c] = lv;
        if (allc) info[c].converged = 1;
    });
    bool any_active = false;
    int n_next = 0;
    for (int j = 0; j < Bc; ++j) {
        const int c = col(j);
        if (info[c].converged) active[c] = 0;
        act_next[j] = active[c];
        if (active[c]) {
            any_active = true;
            ++n_next;
        }
    }
    // Ritz vectors into slots 0..NK-1 (rotated columns; through slots NM+1..
    // when NK needs more than one accumulator tile)
    QS3_HIP(hipMemcpyAsync(dC.ptr, hC, sizeof(double) * (size_t)Bc * NM * NK, hipMemcpyHostToDevice, E.st));
    QS3_HIP(hipMemcpyAsync(dact.ptr, hact, 2 * (size_t)Bc, hipMemcpyHostToDevice, E.st));
    const uint8_t *d_rot = dact.as<uint8_t>(), *d_next = dact.as<uint8_t>() + Bc;
    if (NK <= 16) {
        // one accumulator tile: the rotation can overwrite slots 0..NK-1 in place
        QS3_TRY(E.rotate_dev(0, NM, dC.as<double>(), NK, 0, d_rot));
    } else {
        QS3_TRY(E.rotate_dev(0, NM, dC.as<double>(), NK, NM + 1, d_rot));
        for (int y = 0; y < NK; ++y) QS3_TRY(E.copy_slot_dev(NM + 1 + y, y, d_rot));
    }
    if (!any_active || restarts >= o.max_restarts) {
        QS3_HIP(hipEventRecord(ev, E.st));
        phase = 4;
        *done = true;
        return QS3_OK;
    }
    // from here on the kernels skip the columns that have converged, or the
    // columns still iterating move into a narrower engine
    bool compacted = false;
    if (Bc > 1 && !want_vecs && 4 * n_next <= 3 * Bc) QS3_TRY(compact(act_next, &compacted));
    Engine &En = eng();
    if (compacted) {
        En.colmask = nullptr;
    } else {
        // restart cycle: the residual becomes psi_{NK+1}
        En.colmask = Bc > 1 ? d_next : nullptr;
        QS3_TRY(En.copy_slot_dev(NM, NK, d_next));
    }
    // the first step has no three-term partner (the couplings to the kept
    // Ritz vectors are removed by the full reorthogonalisation), then
    // x = NK+1..NM-1
    QS3_TRY(En.cycle_replay(NK, NM, -1));
    QS3_TRY(enqueue_ab_copy(NK, NM));
    first = false;
    ++restarts;
    phase = 2;
    return QS3_OK;
}

int SolveRun::vec_slot(int col, int y) const {
    if (o.alg == QS3_ALG_TRL) return y < (int)final_lv[col].size() ? final_lv[col][y] : -1;
    return o.steps + 1 + y;
}

static int run_blocking(SolveRun &R, const double *v0) {
    QS3_TRY(R.begin(v0));
    bool done = false;
    while (!done) {
        QS3_TRY(R.wait());
        QS3_TRY(R.advance(&done));
    }
    QS3_TRY(R.wait());
    return QS3_OK;
}

int solve_blocking(qs3_ctx *ctx, Operator *op, const qs3_eigs_opts &o, const double *v0, hipStream_t s,
                   std::vector<double> &evals, std::vector<qs3_eigs_info> &info, double *vec_out) {
    SolveRun R;
    R.want_vecs = vec_out != nullptr;
    QS3_TRY(R.init(ctx, op, o, s));
    QS3_TRY(run_blocking(R, v0));
    evals = R.evals;
    info = R.info;
    if (vec_out) {
        for (int y = 0; y < o.nev; ++y) {
            const int sl = R.vec_slot(0, y);
            if (sl < 0) continue;
            QS3_HIP(hipMemcpyAsync(vec_out + (size_t)y * R.eng().stride, R.eng().slot(sl), sizeof(double) * R.eng().stride,
                                   hipMemcpyDeviceToDevice, s));
        }
        QS3_HIP(hipStreamSynchronize(s));
    }
    return QS3_OK;
}

}  // namespace qs3
