// Launchers of the H.v, debug-row and structure-build kernels for one N_down
// (QS3_INST_K, set by the build), so that the template instances of every
// N_down compile in parallel translation units.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "hv_kernels.h"
#include "obs_kernels.h"

#ifndef QS3_INST_K
#error "QS3_INST_K must be defined"
#endif

namespace qs3 {

constexpr int KI = QS3_INST_K;
// a rank type wider than 32 bits is only ever needed from N_down = 3 on
constexpr bool WIDE_OK = KI >= 3;

template <typename RT>
static size_t lds_need(const qs3_lattice *lat, int K) {
    size_t ntab = K >= 2 ? (size_t)(K - 1) << binom_shift(lat->N) : 0;
    return ((ntab * sizeof(RT) + 15) & ~size_t(15)) + sizeof(int) * (lat->N + 1) +
           sizeof(uint16_t) * lat->h_nbr.size() + 16;
}

// ------------------------------------------------------------------ U(1)
template <typename RT, typename VT, typename OT, int ZM, int UM>
static int launch_u1_z(qs3_sector *sec, const void *v, void *w, hipStream_t s) {
    qs3_lattice *lat = sec->lat;
    LatArgs L = lat_args(lat);
    size_t sh = lds_need<RT>(lat, KI);
    QS3_REQUIRE(sh <= 160 * 1024, QS3_EINVAL, "lattice tables exceed LDS");
    uint64_t tiles = (sec->dim + 255) / 256;
    int grid = grid_for(lat->ctx, tiles);
    hipLaunchKernelGGL((k_hv_u1<KI, RT, VT, OT, ZM, UM>), dim3(grid), dim3(256), sh, s, L,
                       sec->bt->dev.as<RT>(), (RT)sec->dim, (const VT *)v, (OT *)w);
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

// the unrolled all-hops-in-flight row on lattices where every site has 2, 4
// or 6 neighbours (chains, square and cubic lattices, with any couplings)
// while K * degree stays within the registers; the plain loop otherwise
template <typename RT, typename VT, typename OT>
static int launch_u1(qs3_sector *sec, const void *v, void *w, hipStream_t s) {
    const qs3_lattice *lat = sec->lat;
    const int z = lat->regular ? lat->max_degree : 0;
    if (lat->uniform) {
        if (z == 2 && KI * 2 <= 24) return launch_u1_z<RT, VT, OT, 2, 1>(sec, v, w, s);
        if (z == 4 && KI * 4 <= 24) return launch_u1_z<RT, VT, OT, 4, 1>(sec, v, w, s);
        if (z == 6 && KI * 6 <= 24) return launch_u1_z<RT, VT, OT, 6, 1>(sec, v, w, s);
    } else {
        if (z == 2 && KI * 2 <= 24) return launch_u1_z<RT, VT, OT, 2, 2>(sec, v, w, s);
        if (z == 4 && KI * 4 <= 24) return launch_u1_z<RT, VT, OT, 4, 2>(sec, v, w, s);
        if (z == 6 && KI * 6 <= 24) return launch_u1_z<RT, VT, OT, 6, 2>(sec, v, w, s);
    }
    return launch_u1_z<RT, VT, OT, 0, 0>(sec, v, w, s);
}

template <typename RT>
static int u1_types(qs3_sector *sec, const void *v, int vtype, void *w, int wtype, hipStream_t s) {
    if (vtype == QS3_F64 && wtype == QS3_F64) return launch_u1<RT, double, double>(sec, v, w, s);
    if (vtype == QS3_F32 && wtype == QS3_F32) return launch_u1<RT, float, float>(sec, v, w, s);
    if (vtype == QS3_F32 && wtype == QS3_F64) return launch_u1<RT, float, double>(sec, v, w, s);
    set_error("unsupported dtype pair for a fixed-N_down matvec");
    return QS3_EINVAL;
}

template <>
int hv_u1_K<KI>(qs3_sector *sec, const void *v, int vtype, void *w, int wtype, hipStream_t s) {
    if constexpr (WIDE_OK) {
        if (sec->bt->wide) return u1_types<uint64_t>(sec, v, vtype, w, wtype, s);
    }
    QS3_REQUIRE(!sec->bt->wide, QS3_EINVAL, "internal: wide ranks at small N_down");
    return u1_types<uint32_t>(sec, v, vtype, w, wtype, s);
}

template <typename RT>
static int row_u1_t(qs3_sector *sec, uint64_t row, int cap, int64_t *cols, double *vals,
                    double *diag, int *nnz) {
    qs3_ctx *ctx = sec->lat->ctx;
    DevBuf buf;
    size_t capb = std::max(cap, 1);
    QS3_TRY(buf.alloc(ctx, capb * 16 + 64));
    int64_t *dc = (int64_t *)buf.ptr;
    double *dv = (double *)(dc + capb);
    double *dd = dv + capb;
    int *dn = (int *)(dd + 1);
    hipLaunchKernelGGL((k_row_u1<KI, RT>), dim3(1), dim3(1), 0, 0, lat_args(sec->lat),
                       sec->bt->dev.as<RT>(), (RT)row, cap, dc, dv, dd, dn);
    QS3_HIP(hipGetLastError());
    QS3_HIP(hipDeviceSynchronize());
    int n = 0;
    QS3_HIP(hipMemcpy(&n, dn, sizeof(int), hipMemcpyDeviceToHost));
    QS3_HIP(hipMemcpy(diag, dd, sizeof(double), hipMemcpyDeviceToHost));
    int m = std::min(n, cap);
    if (m > 0) {
        QS3_HIP(hipMemcpy(cols, dc, sizeof(int64_t) * m, hipMemcpyDeviceToHost));
        QS3_HIP(hipMemcpy(vals, dv, sizeof(double) * m, hipMemcpyDeviceToHost));
    }
    *nnz = n;
    return QS3_OK;
}

template <>
int row_u1_K<KI>(qs3_sector *sec, uint64_t row, int cap, int64_t *cols, double *vals,
                 double *diag, int *nnz) {
    if constexpr (WIDE_OK) {
        if (sec->bt->wide) return row_u1_t<uint64_t>(sec, row, cap, cols, vals, diag, nnz);
    }
    return row_u1_t<uint32_t>(sec, row, cap, cols, vals, diag, nnz);
}


// ------------------------------------------------------------------ observables (fixed N_down)
// All pair sums pm_ij at once as the Gram matrix of the factor of k_pm_rows
// (chunks of at most 256 MB of factor; per chunk, split-row tile partials and
// their ordered sum, added to G on the host), then read out for the requested
// pairs (hpi < hpj, host).
template <typename RT>
static int pm_gram(qs3_sector *sec, const double *phi, int npairs, const int32_t *hpi, const int32_t *hpj,
                   std::vector<double> &pm, hipStream_t s) {
    constexpr int K = KI;
    qs3_ctx *ctx = sec->lat->ctx;
    const int N = sec->lat->N;
    const BinomTable &bt = *sec->bt;
    const uint64_t nb = bt.C(N, K - 1);
    const uint64_t nc = std::max<uint64_t>(1, std::min<uint64_t>(nb, (32ull << 20) / (uint64_t)N));
    const int nt = (N + 63) / 64;
    std::vector<int2> tiles;
    for (int a = 0; a < nt; ++a)
        for (int b = a; b < nt; ++b) tiles.push_back(make_int2(a, b));
    const int ntp = (int)tiles.size();
    // about four blocks per CU for the tile kernel; the chunk partials are
    // summed in order in groups of GS chunks, then the group sums
    const int max_chunks = std::max(1, 4 * ctx->n_cu / ntp);
    constexpr int GS = 16;
    const int max_groups = (max_chunks + GS - 1) / GS;
    DevBuf U, G, P, P2, T;
    QS3_TRY(U.alloc(ctx, sizeof(double) * nc * N));
    QS3_TRY(G.alloc(ctx, sizeof(double) * (size_t)N * N));
    QS3_TRY(P.alloc(ctx, sizeof(double) * 4096 * (size_t)ntp * max_chunks));
    QS3_TRY(P2.alloc(ctx, sizeof(double) * 4096 * (size_t)ntp * max_groups));
    QS3_TRY(T.alloc(ctx, sizeof(int2) * (size_t)ntp));
    QS3_HIP(hipMemcpyAsync(T.ptr, tiles.data(), sizeof(int2) * ntp, hipMemcpyHostToDevice, s));
    std::vector<double> acc((size_t)N * N, 0.0), hG((size_t)N * N);
    for (uint64_t b0 = 0; b0 < nb; b0 += nc) {
        const uint64_t m = std::min(nc, nb - b0);
        hipLaunchKernelGGL((k_pm_rows<K, RT>), dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, N,
                           sec->bt->dev.as<RT>(), b0, m, phi, U.as<double>());
        QS3_HIP(hipGetLastError());
        // rows per chunk: a multiple of 16, at most max_chunks chunks
        uint64_t rc = std::max<uint64_t>(16, (m + max_chunks - 1) / max_chunks);
        rc = (rc + 15) / 16 * 16;
        const int nchunk = (int)((m + rc - 1) / rc);
        hipLaunchKernelGGL(k_gram_tiles<64>, dim3(nchunk, ntp), dim3(256), 0, s, U.as<double>(), m, N, rc,
                           T.as<int2>(), ntp, P.as<double>());
        QS3_HIP(hipGetLastError());
        const unsigned eb = (unsigned)(((uint64_t)ntp * 4096 + 255) / 256);
        const int ngroup = (nchunk + GS - 1) / GS;
        hipLaunchKernelGGL(k_gram_group<64>, dim3(eb, ngroup), dim3(256), 0, s, P.as<double>(), nchunk, ntp, GS,
                           P2.as<double>());
        QS3_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_gram_reduce<64>, dim3(eb), dim3(256), 0, s, P2.as<double>(), ngroup, T.as<int2>(), ntp, N,
                           G.as<double>());
        QS3_HIP(hipGetLastError());
        QS3_HIP(hipMemcpyAsync(hG.data(), G.ptr, sizeof(double) * hG.size(), hipMemcpyDeviceToHost, s));
        QS3_HIP(hipStreamSynchronize(s));
        for (size_t e = 0; e < hG.size(); ++e) acc[e] += hG[e];
    }
    for (int t = 0; t < npairs; ++t) pm[t] = acc[(size_t)hpi[t] + (size_t)hpj[t] * N];
    return QS3_OK;
}

template <typename RT>
static int obs_u1_t(qs3_sector *sec, const double *phi, int npairs, const int32_t *pi,
                    const int32_t *pj, std::vector<double> &p_site, std::vector<double> &q,
                    std::vector<double> &pm, hipStream_t s, const int32_t *hpi, const int32_t *hpj) {
    constexpr int K = KI;
    qs3_lattice *lat = sec->lat;
    const int N = lat->N;
    LatArgs L = lat_args(lat);
    const RT *tab = sec->bt->dev.as<RT>();
    const BinomTable &bt = *sec->bt;
    p_site.assign(N, 0.0);
    q.assign(npairs, 0.0);
    pm.assign(npairs, 0.0);
    if (K == 0) return QS3_OK;
    {
        const uint64_t cnt = bt.C(N - 1, K - 1);
        const int nchunk = (int)std::max<uint64_t>(1, std::min<uint64_t>((cnt + 4095) / 4096, (2048 + N - 1) / N));
        DevBuf part;
        QS3_TRY(part.alloc(lat->ctx, sizeof(double2) * (size_t)N * nchunk));
        hipLaunchKernelGGL((k_site_prob<K, RT>), dim3(N, nchunk), dim3(256), 0, s, L, tab, cnt, nchunk,
                           phi, part.as<double2>());
        QS3_HIP(hipGetLastError());
        std::vector<double2> h((size_t)N * nchunk);
        QS3_HIP(hipMemcpyAsync(h.data(), part.ptr, sizeof(double2) * h.size(), hipMemcpyDeviceToHost, s));
        QS3_HIP(hipStreamSynchronize(s));
        for (int i = 0; i < N; ++i)
            for (int c = 0; c < nchunk; ++c) p_site[i] += h[(size_t)i * nchunk + c].x;
    }
    if (npairs > 0) {
        // many pairs (host pairs given): the S^+S^- sums come from one Gram
        // matrix over all sites instead of one subset loop per pair
        const bool gram = hpi && hpj && npairs >= N;
        const uint64_t cq = K >= 2 ? bt.C(N - 2, K - 2) : 0, cpm = gram ? 0 : bt.C(N - 2, K - 1);
        const uint64_t cmax = std::max(cq, cpm);
        const int nchunk = (int)std::max<uint64_t>(1, std::min<uint64_t>((cmax + 4095) / 4096,
                                                                          (4096 + npairs - 1) / npairs));
        DevBuf part;
        QS3_TRY(part.alloc(lat->ctx, sizeof(double2) * (size_t)npairs * nchunk));
        hipLaunchKernelGGL((k_pair_u1<K, RT>), dim3(npairs, nchunk), dim3(256), 0, s, L, tab, pi, pj, cq,
                           cpm, nchunk, phi, part.as<double2>());
        QS3_HIP(hipGetLastError());
        std::vector<double2> h((size_t)npairs * nchunk);
        QS3_HIP(hipMemcpyAsync(h.data(), part.ptr, sizeof(double2) * h.size(), hipMemcpyDeviceToHost, s));
        QS3_HIP(hipStreamSynchronize(s));
        for (int p = 0; p < npairs; ++p)
            for (int c = 0; c < nchunk; ++c) {
                q[p] += h[(size_t)p * nchunk + c].x;
                pm[p] += h[(size_t)p * nchunk + c].y;
            }
        if (gram) QS3_TRY(pm_gram<RT>(sec, phi, npairs, hpi, hpj, pm, s));
    }
    return QS3_OK;
}

template <>
int obs_u1_K<KI>(qs3_sector *sec, const double *phi, int npairs, const int32_t *pi,
                 const int32_t *pj, std::vector<double> &p_site, std::vector<double> &q,
                 std::vector<double> &pm, hipStream_t s, const int32_t *hpi, const int32_t *hpj) {
    if constexpr (WIDE_OK) {
        if (sec->bt->wide) return obs_u1_t<uint64_t>(sec, phi, npairs, pi, pj, p_site, q, pm, s, hpi, hpj);
    }
    return obs_u1_t<uint32_t>(sec, phi, npairs, pi, pj, p_site, q, pm, s, hpi, hpj);
}

// ------------------------------------------------------------------ small sectors
template <typename RT, bool CPLX, bool TABLE>
static int small_t(qs3_lattice *lat, const BinomTable *bt, qs3_batch *bat, const SmallArgs &S, hipStream_t s) {
    BatchArgs A{};
    if (bat) A = batch_args(bat);
    else A.L = lat_args(lat);
    const size_t sh = lds_need<RT>(lat, KI);
    QS3_REQUIRE(sh <= 64 * 1024, QS3_EINVAL, "lattice tables exceed LDS");
    // fixed N_down on a regular lattice: the unrolled row
    const int z = lat->regular ? lat->max_degree : 0;
    if constexpr (!CPLX) {
        if (z == 2 && KI * 2 <= 24)
            hipLaunchKernelGGL((k_lanczos_small<KI, RT, CPLX, TABLE, 2>), dim3(1), dim3(1024), sh, s, S, A,
                               bt->dev.as<RT>());
        else if (z == 4 && KI * 4 <= 24)
            hipLaunchKernelGGL((k_lanczos_small<KI, RT, CPLX, TABLE, 4>), dim3(1), dim3(1024), sh, s, S, A,
                               bt->dev.as<RT>());
        else if (z == 6 && KI * 6 <= 24)
            hipLaunchKernelGGL((k_lanczos_small<KI, RT, CPLX, TABLE, 6>), dim3(1), dim3(1024), sh, s, S, A,
                               bt->dev.as<RT>());
        else
            hipLaunchKernelGGL((k_lanczos_small<KI, RT, CPLX, TABLE, 0>), dim3(1), dim3(1024), sh, s, S, A,
                               bt->dev.as<RT>());
    } else {
        (void)z;
        hipLaunchKernelGGL((k_lanczos_small<KI, RT, CPLX, TABLE, 0>), dim3(1), dim3(1024), sh, s, S, A,
                           bt->dev.as<RT>());
    }
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

template <>
int lanczos_small_K<KI>(qs3_lattice *lat, const BinomTable *bt, qs3_batch *bat, const SmallArgs &S, hipStream_t s) {
    if (bt->wide) return 1;  // small sectors never need 64-bit ranks
    if (!bat) return small_t<uint32_t, false, false>(lat, bt, bat, S, s);
#if QS3_INST_K <= 6
    if (bat->ks->has_table) return small_t<uint32_t, true, true>(lat, bt, bat, S, s);
    return small_t<uint32_t, true, false>(lat, bt, bat, S, s);
#else
    return 1;
#endif
}

#if QS3_INST_K <= 6
// ------------------------------------------------------------------ momentum batches
// One launch of the batched kernel with G lanes per row and `bpc` blocks
// per CU (at most 8 sectors per lane and pass, several passes beyond that).
template <typename RT, typename CT, typename OT, int MODE>
static int launch_batch_g(qs3_batch *bat, BatchArgs A, int G, int bpc, const void *v, void *w,
                          hipStream_t s) {
    A.G = G;
    size_t sh = lds_need<RT>(bat->lat, KI);
    // the phase table after the lattice tables, when it fits
    const size_t ph_off = (sh + 15) & ~size_t(15);
    if (A.M <= 4096 && ph_off + 16 * (size_t)A.M <= 64 * 1024) {
        A.ph_lds_off = (int)ph_off;
        sh = ph_off + 16 * (size_t)A.M;
    }
    QS3_REQUIRE(sh <= 160 * 1024, QS3_EINVAL, "lattice tables exceed LDS");
    const int per = (A.B + A.G - 1) / A.G;
    const uint64_t rows_per_tile = 256 / A.G;
    const uint64_t tiles = (A.n_reps + rows_per_tile - 1) / rows_per_tile;
    uint64_t g = std::min<uint64_t>(tiles, (uint64_t)bat->lat->ctx->n_cu * bpc);
    if (g >= 8) g &= ~uint64_t(7);
    const int grid = (int)std::max<uint64_t>(g, 1);
    const RT *tab = bat->bt->dev.as<RT>();
    using C2 = typename Cplx<CT>::type;
    using O2 = typename Cplx<OT>::type;
#define QS3_LB(BPL, NP)                                                                             \
    hipLaunchKernelGGL((k_hv_batch<KI, RT, CT, OT, MODE, BPL, NP>), dim3(grid), dim3(256), sh, s, A, \
                       tab, (const C2 *)v, (O2 *)w)
    bat->last_G = G;
    bat->last_bpc = bpc;
    if (per <= 1) QS3_LB(1, 1);
    else if (per <= 2) QS3_LB(2, 1);
    else if (per <= 4) QS3_LB(4, 1);
    else if (per <= 8) QS3_LB(8, 1);
    else if (per <= 16) QS3_LB(8, 2);
    else if (per <= 32) QS3_LB(8, 4);
    else {
        set_error("batch larger than 2048 sectors");
        return QS3_EINVAL;
    }
#undef QS3_LB
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

// Times the candidate schedules on the caller's vectors (every launch writes
// the same w) and returns the fastest: first G in {8, 16, 32, 64} (at most 32
// sectors per lane) at 8 blocks per CU, then 4, 8 and 16 blocks per CU.
template <typename RT, typename CT, typename OT, int MODE>
static int tune_batch(qs3_batch *bat, const BatchArgs &A, const void *v, void *w, hipStream_t s, int *G_out,
                      int *bpc_out) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    QS3_HIP(hipEventCreate(&e0));
    QS3_HIP(hipEventCreate(&e1));
    auto timed = [&](int G, int bpc, float *ms) -> int {
        QS3_TRY((launch_batch_g<RT, CT, OT, MODE>(bat, A, G, bpc, v, w, s)));  // warm-up
        QS3_HIP(hipEventRecord(e0, s));
        for (int r = 0; r < 2; ++r) QS3_TRY((launch_batch_g<RT, CT, OT, MODE>(bat, A, G, bpc, v, w, s)));
        QS3_HIP(hipEventRecord(e1, s));
        QS3_HIP(hipEventSynchronize(e1));
        QS3_HIP(hipEventElapsedTime(ms, e0, e1));
        return QS3_OK;
    };
    int rc = QS3_OK, bestG = 0, bestB = 8;
    float best = 0;
    for (int G = 8; G <= 64 && rc == QS3_OK; G <<= 1) {
        if ((A.B + G - 1) / G > 32) continue;
        float ms = 0;
        rc = timed(G, 8, &ms);
        if (rc == QS3_OK && (bestG == 0 || ms < best)) {
            best = ms;
            bestG = G;
        }
    }
    for (int bpc : {4, 16}) {
        if (rc != QS3_OK) break;
        float ms = 0;
        rc = timed(bestG, bpc, &ms);
        if (rc == QS3_OK && ms < best) {
            best = ms;
            bestB = bpc;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != QS3_OK) return rc;
    *G_out = bestG;
    *bpc_out = bestB;
    return QS3_OK;
}

template <typename RT, typename CT, typename OT, int MODE>
static int launch_batch(qs3_batch *bat, const void *v, void *w, hipStream_t s) {
    BatchArgs A = batch_args(bat);
    if (A.B == 1) {
        bat->last_groups = bat->last_group_width = 1;
        // a single sector: one or two lanes per row, all of its hops in flight together
        using C2 = typename Cplx<CT>::type;
        using O2 = typename Cplx<OT>::type;
        // LDS of the hop-list kernel: per cell translation t, (J_xy/2) e^{ik.t}
        // and its phase index; the phase table
        const int ntr = bat->lat->lx * bat->lat->ly * bat->lat->lz;
        const size_t lds1 = ((sizeof(C2) * (size_t)ntr + 15) & ~size_t(15)) + sizeof(double2) * (size_t)A.M +
                            sizeof(double) * 16 + sizeof(uint16_t) * (size_t)ntr;
        const bool factors = bat->ks->nt_u.empty() || A.gcls;
        if (MODE == HOP_LISTS && A.tP && factors && A.L.uniform && A.hmax <= 24 && lds1 <= 64 * 1024) {
            // hop lists with one exchange constant: the entries give every term
            // two lanes per row while the sector is small enough for its rows
            // to be resident at once; one lane per row (more registers per
            // lane, fewer instructions per row) for larger ones
            const bool two = A.n_reps <= (2ull << 20);
            const int g1 = grid_cover(bat->lat->ctx, (A.n_reps + 255) / 256);
            const int g2 = grid_cover(bat->lat->ctx, (A.n_reps + 127) / 128);
#define QS3_L1(HM)                                                                                           \
    do {                                                                                                     \
        if (two)                                                                                             \
            hipLaunchKernelGGL((k_hv_one_lists<CT, OT, HM, 2>), dim3(g2), dim3(256), lds1, s, A, (const C2 *)v, \
                               (O2 *)w);                                                                     \
        else                                                                                                 \
            hipLaunchKernelGGL((k_hv_one_lists<CT, OT, HM, 1>), dim3(g1), dim3(256), lds1, s, A, (const C2 *)v, \
                               (O2 *)w);                                                                     \
    } while (0)
            if (A.hmax <= 6) QS3_L1(6);
            else if (A.hmax <= 8) QS3_L1(8);
            else if (A.hmax <= 12) QS3_L1(12);
            else if (A.hmax <= 16) QS3_L1(16);
            else if (A.hmax <= 18) QS3_L1(18);
            else QS3_L1(24);
#undef QS3_L1
            QS3_HIP(hipGetLastError());
            return QS3_OK;
        }
        size_t sh1 = lds_need<RT>(bat->lat, KI);
        QS3_REQUIRE(sh1 <= 160 * 1024, QS3_EINVAL, "lattice tables exceed LDS");
        const int grid1 = grid_cover(bat->lat->ctx, (A.n_reps + 255) / 256);
        hipLaunchKernelGGL((k_hv_one<KI, RT, CT, OT, MODE>), dim3(grid1), dim3(256), sh1, s, A,
                           bat->bt->dev.as<RT>(), (const C2 *)v, (O2 *)w);
        QS3_HIP(hipGetLastError());
        return QS3_OK;
    }
    // Schedule: G lanes per row (a power of two, 8..64) and blocks per CU.
    // The rule: G = the smallest power of two >= B (at least 8, at most 64),
    // so a narrow batch (the few sectors a solve has left) still resolves 8
    // hops at a time with 8 gathers in flight, and 8 blocks per CU.  With
    // autotuning on, the first launch of each width class (B rounded up to a
    // power of two), element type and hop store times every G with at most
    // 32 sectors per lane, then 4, 8 and 16 blocks per CU at the best G, and
    // keeps the fastest in the structure's cache.  Every schedule sums each
    // sector's hops in hop order, so the choice does not change results.
    //
    // A wide batch of long vectors runs as consecutive launches over groups
    // of at most 256 sectors (same row stride, the group's columns): a group's
    // share of v is gathered from a smaller footprint, which the caches serve
    // better (10^3 cube, N_down = 3: 6.7 us per sector at 256 sectors a
    // launch, 8.4 us at 1000).  Each sector's sum is unchanged.
    using C2g = typename Cplx<CT>::type;
    using O2g = typename Cplx<OT>::type;
    int ng = 1;
    if (A.B > 256 && A.n_reps * (uint64_t)A.B * sizeof(C2g) > (512ull << 20)) ng = (A.B + 255) / 256;
    const int Bg = (A.B + ng - 1) / ng;
    auto group = [&](int gi) {
        BatchArgs Ag = A;
        const int b0 = gi * Bg;
        Ag.B = std::min(Bg, A.B - b0);
        Ag.kmul = A.kmul + 3 * b0;
        if (A.active) Ag.active = A.active + b0;
        if (A.compat_nt) Ag.compat_nt = A.compat_nt + b0;
        return Ag;
    };
    const BatchArgs A0 = group(0);
    int G = 8;
    while (G < A0.B && G < 64) G <<= 1;
    int bpc = 8;
    qs3_ctx *ctx = bat->lat->ctx;
    if (ctx->autotune) {
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        QS3_HIP(hipStreamIsCapturing(s, &cs));
        if (cs == hipStreamCaptureStatusNone) {
            int cls = 0;
            while ((1 << cls) < A0.B) ++cls;
            const uint32_t key = ((uint32_t)cls << 8) | ((uint32_t)sizeof(CT) << 4) | (uint32_t)MODE;
            KStructure &ks = *bat->ks;
            std::lock_guard<std::mutex> lk(ks.tune_mu);
            auto it = ks.tuned.find(key);
            if (it != ks.tuned.end()) {
                G = it->second.first;
                bpc = it->second.second;
            } else {
                // timed on the first group (its columns of w are written again below)
                QS3_TRY((tune_batch<RT, CT, OT, MODE>(bat, A0, v, w, s, &G, &bpc)));
                ks.tuned[key] = {G, bpc};
            }
        }
    }
    bat->last_groups = ng;
    bat->last_group_width = Bg;
    for (int gi = 0; gi < ng; ++gi) {
        const BatchArgs Ag = group(gi);
        QS3_TRY((launch_batch_g<RT, CT, OT, MODE>(bat, Ag, G, bpc, (const C2g *)v + (size_t)gi * Bg,
                                                  (O2g *)w + (size_t)gi * Bg, s)));
    }
    return QS3_OK;
}

template <typename RT, typename CT, typename OT>
static int batch_mode(qs3_batch *bat, const void *v, void *w, hipStream_t s) {
    // hop lists read each row's resolved hops contiguously: preferred
    if (bat->ks->has_hops) return launch_batch<RT, CT, OT, HOP_LISTS>(bat, v, w, s);
    if (bat->ks->has_table) return launch_batch<RT, CT, OT, HOP_TABLE>(bat, v, w, s);
    return launch_batch<RT, CT, OT, HOP_FLY>(bat, v, w, s);
}

template <typename RT>
static int batch_types(qs3_batch *bat, const void *v, int vtype, void *w, int wtype, hipStream_t s) {
    if (vtype == QS3_C128 && wtype == QS3_C128) return batch_mode<RT, double, double>(bat, v, w, s);
    if (vtype == QS3_C64 && wtype == QS3_C128) return batch_mode<RT, float, double>(bat, v, w, s);
    set_error("unsupported dtype pair for a momentum matvec");
    return QS3_EINVAL;
}

template <>
int hv_batch_K<KI>(qs3_batch *bat, const void *v, int vtype, void *w, int wtype, hipStream_t s) {
    if constexpr (WIDE_OK) {
        if (bat->bt->wide) return batch_types<uint64_t>(bat, v, vtype, w, wtype, s);
    }
    return batch_types<uint32_t>(bat, v, vtype, w, wtype, s);
}

template <typename RT, bool TABLE>
static int row_k_t(qs3_sector *sec, uint64_t u, int cap, int64_t *cols, double *vals,
                   double *diag, int *nnz) {
    qs3_ctx *ctx = sec->lat->ctx;
    DevBuf buf;
    size_t capb = std::max(cap, 1);
    QS3_TRY(buf.alloc(ctx, capb * 24 + 64));
    int64_t *dc = (int64_t *)buf.ptr;
    double *dv = (double *)(dc + capb);
    double *dd = dv + 2 * capb;
    int *dn = (int *)(dd + 1);
    BatchArgs A = batch_args(sec->bat);
    hipLaunchKernelGGL((k_row_k<KI, RT, TABLE>), dim3(1), dim3(1), 0, 0, A,
                       sec->bat->bt->dev.as<RT>(), u, cap, dc, dv, dd, dn);
    QS3_HIP(hipGetLastError());
    QS3_HIP(hipDeviceSynchronize());
    int n = 0;
    QS3_HIP(hipMemcpy(&n, dn, sizeof(int), hipMemcpyDeviceToHost));
    QS3_HIP(hipMemcpy(diag, dd, sizeof(double), hipMemcpyDeviceToHost));
    int m = std::min(n, cap);
    if (m > 0) {
        QS3_HIP(hipMemcpy(cols, dc, sizeof(int64_t) * m, hipMemcpyDeviceToHost));
        QS3_HIP(hipMemcpy(vals, dv, sizeof(double) * 2 * m, hipMemcpyDeviceToHost));
    }
    *nnz = n;
    return QS3_OK;
}

template <>
int row_k_K<KI>(qs3_sector *sec, uint64_t u, int cap, int64_t *cols, double *vals, double *diag,
                int *nnz) {
    const bool tabm = sec->bat->ks->has_table;
    if constexpr (WIDE_OK) {
        if (sec->bat->bt->wide)
            return tabm ? row_k_t<uint64_t, true>(sec, u, cap, cols, vals, diag, nnz)
                        : row_k_t<uint64_t, false>(sec, u, cap, cols, vals, diag, nnz);
    }
    return tabm ? row_k_t<uint32_t, true>(sec, u, cap, cols, vals, diag, nnz)
                : row_k_t<uint32_t, false>(sec, u, cap, cols, vals, diag, nnz);
}


// ------------------------------------------------------------------ momentum observables
template <typename RT, bool TABLE>
static int corr_k_t(qs3_sector *sec, const double *phi_union, int ndisp, const int32_t *disp,
                    std::vector<double> &zz, std::vector<double> &nrm, std::vector<double> &pr,
                    std::vector<double> &pim, hipStream_t s) {
    qs3_batch *bat = sec->bat;
    BatchArgs A = batch_args(bat);
    const int nchunk = (int)std::max<uint64_t>(1, std::min<uint64_t>((A.n_reps + 1023) / 1024,
                                                                      (2048 + ndisp - 1) / ndisp));
    DevBuf part;
    QS3_TRY(part.alloc(sec->lat->ctx, sizeof(double2) * 2 * (size_t)ndisp * nchunk));
    hipLaunchKernelGGL((k_corr_k<KI, RT, TABLE>), dim3(ndisp, nchunk), dim3(256), 0, s, A,
                       bat->bt->dev.as<RT>(), disp, nchunk, (const double2 *)phi_union,
                       part.as<double2>());
    QS3_HIP(hipGetLastError());
    std::vector<double2> h(2 * (size_t)ndisp * nchunk);
    QS3_HIP(hipMemcpyAsync(h.data(), part.ptr, sizeof(double2) * h.size(), hipMemcpyDeviceToHost, s));
    QS3_HIP(hipStreamSynchronize(s));
    zz.assign(ndisp, 0.0);
    nrm.assign(ndisp, 0.0);
    pr.assign(ndisp, 0.0);
    pim.assign(ndisp, 0.0);
    for (int d = 0; d < ndisp; ++d)
        for (int c = 0; c < nchunk; ++c) {
            const double2 a = h[((size_t)d * nchunk + c) * 2], b = h[((size_t)d * nchunk + c) * 2 + 1];
            zz[d] += a.x;
            nrm[d] += a.y;
            pr[d] += b.x;
            pim[d] += b.y;
        }
    return QS3_OK;
}

template <>
int corr_k_K<KI>(qs3_sector *sec, const double *phi_union, int ndisp, const int32_t *disp,
                 std::vector<double> &zz, std::vector<double> &nrm, std::vector<double> &pr,
                 std::vector<double> &pim, hipStream_t s) {
    const bool tabm = sec->bat->ks->has_table;
    if constexpr (WIDE_OK) {
        if (sec->bat->bt->wide)
            return tabm ? corr_k_t<uint64_t, true>(sec, phi_union, ndisp, disp, zz, nrm, pr, pim, s)
                        : corr_k_t<uint64_t, false>(sec, phi_union, ndisp, disp, zz, nrm, pr, pim, s);
    }
    return tabm ? corr_k_t<uint32_t, true>(sec, phi_union, ndisp, disp, zz, nrm, pr, pim, s)
                : corr_k_t<uint32_t, false>(sec, phi_union, ndisp, disp, zz, nrm, pr, pim, s);
}

#if QS3_INST_K <= 5
template <typename RTa, typename RTb, bool TABLE>
static int smq_t(qs3_batch *src, qs3_batch *dst, const int32_t *qmul, const double2 *subph, const double *phi,
                 double *out, hipStream_t s) {
    SmqArgs S{batch_args(src), batch_args(dst), qmul, subph};
    const int G = S.dst.G, B = S.dst.B;
    const int per = (B + G - 1) / G;
    const uint64_t rows_per = 256 / G;
    const unsigned grid = (unsigned)((S.dst.n_reps + rows_per - 1) / rows_per);
    const RTa *ta = src->bt->dev.as<RTa>();
    const RTb *tb = dst->bt->dev.as<RTb>();
#define QS3_SMQ(BPL)                                                                                  \
    hipLaunchKernelGGL((k_smq<KI, RTa, RTb, TABLE, BPL>), dim3(grid), dim3(256), 0, s, S, ta, tb,      \
                       (const double2 *)phi, (double2 *)out)
    if (per <= 1) QS3_SMQ(1);
    else if (per <= 2) QS3_SMQ(2);
    else if (per <= 4) QS3_SMQ(4);
    else if (per <= 16) QS3_SMQ(16);
    else {
        set_error("at most 1024 momenta per S^-_q batch");
        return QS3_EINVAL;
    }
#undef QS3_SMQ
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

template <typename RTa, typename RTb>
static int smq_mode(qs3_batch *src, qs3_batch *dst, const int32_t *qmul, const double2 *subph, const double *phi,
                    double *out, hipStream_t s) {
    if (src->ks->has_table) return smq_t<RTa, RTb, true>(src, dst, qmul, subph, phi, out, s);
    return smq_t<RTa, RTb, false>(src, dst, qmul, subph, phi, out, s);
}

template <>
int smq_K<KI>(qs3_batch *src, qs3_batch *dst, const int32_t *qmul, const double2 *subph, const double *phi,
              double *out, hipStream_t s) {
    const bool wa = src->bt->wide, wb = dst->bt->wide;
    if constexpr (KI >= 3) {
        if (wa && wb) return smq_mode<uint64_t, uint64_t>(src, dst, qmul, subph, phi, out, s);
    }
    if constexpr (KI >= 2) {
        if (!wa && wb) return smq_mode<uint32_t, uint64_t>(src, dst, qmul, subph, phi, out, s);
    }
    QS3_REQUIRE(!wa && !wb, QS3_EINVAL, "internal: rank width");
    return smq_mode<uint32_t, uint32_t>(src, dst, qmul, subph, phi, out, s);
}
#endif  // S^-_q targets at most 6 down spins

// S^+_q: source KI down spins, targets KI - 1
template <typename RTa, typename RTb, bool TABLE>
static int spq_t(qs3_batch *src, qs3_batch *dst, const int32_t *qmul, const double2 *subph, const double *phi,
                 double *out, hipStream_t s) {
    SmqArgs S{batch_args(src), batch_args(dst), qmul, subph};
    const int G = S.dst.G, B = S.dst.B;
    const int per = (B + G - 1) / G;
    const uint64_t rows_per = 256 / G;
    const unsigned grid = (unsigned)((S.dst.n_reps + rows_per - 1) / rows_per);
    const RTa *ta = src->bt->dev.as<RTa>();
    const RTb *tb = dst->bt->dev.as<RTb>();
#define QS3_SPQ(BPL)                                                                                  \
    hipLaunchKernelGGL((k_spq<KI, RTa, RTb, TABLE, BPL>), dim3(grid), dim3(256), 0, s, S, ta, tb,      \
                       (const double2 *)phi, (double2 *)out)
    if (per <= 1) QS3_SPQ(1);
    else if (per <= 2) QS3_SPQ(2);
    else if (per <= 4) QS3_SPQ(4);
    else if (per <= 16) QS3_SPQ(16);
    else {
        set_error("at most 1024 momenta per S^+_q batch");
        return QS3_EINVAL;
    }
#undef QS3_SPQ
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

template <typename RTa, typename RTb>
static int spq_mode(qs3_batch *src, qs3_batch *dst, const int32_t *qmul, const double2 *subph, const double *phi,
                    double *out, hipStream_t s) {
    if (src->ks->has_table) return spq_t<RTa, RTb, true>(src, dst, qmul, subph, phi, out, s);
    return spq_t<RTa, RTb, false>(src, dst, qmul, subph, phi, out, s);
}

template <>
int spq_K<KI>(qs3_batch *src, qs3_batch *dst, const int32_t *qmul, const double2 *subph, const double *phi,
              double *out, hipStream_t s) {
    if constexpr (KI == 0) {
        set_error("S^+_q needs N_down >= 1");
        return QS3_EINVAL;
    } else {
        const bool wa = src->bt->wide, wb = dst->bt->wide;
        if constexpr (KI >= 4) {
            if (wa && wb) return spq_mode<uint64_t, uint64_t>(src, dst, qmul, subph, phi, out, s);
        }
        if constexpr (KI >= 3) {
            if (wa && !wb) return spq_mode<uint64_t, uint32_t>(src, dst, qmul, subph, phi, out, s);
        }
        QS3_REQUIRE(!wa && !wb, QS3_EINVAL, "internal: rank width");
        return spq_mode<uint32_t, uint32_t>(src, dst, qmul, subph, phi, out, s);
    }
}

// S^z_q: source and targets share the KI-down structure
template <typename RT>
static int szq_t(qs3_batch *src, qs3_batch *dst, const int32_t *qmul, const double2 *subph, const double *phi,
                 double *out, hipStream_t s) {
    SmqArgs S{batch_args(src), batch_args(dst), qmul, subph};
    const uint64_t n = S.dst.n_reps * (uint64_t)S.dst.B;
    if (n == 0) return QS3_OK;
    hipLaunchKernelGGL((k_szq<KI, RT>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, S,
                       src->bt->dev.as<RT>(), (const double2 *)phi, (double2 *)out);
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

template <>
int szq_K<KI>(qs3_batch *src, qs3_batch *dst, const int32_t *qmul, const double2 *subph, const double *phi,
              double *out, hipStream_t s) {
    QS3_REQUIRE(src->ks == dst->ks, QS3_EINVAL, "internal: S^z_q keeps the structure");
    if constexpr (WIDE_OK) {
        if (src->bt->wide) return szq_t<uint64_t>(src, dst, qmul, subph, phi, out, s);
    }
    return szq_t<uint32_t>(src, dst, qmul, subph, phi, out, s);
}

// ------------------------------------------------------------------ dense blocks
#if QS3_INST_K <= 6
template <typename RT, bool TABLE>
static int dense_k_t(qs3_sector *sec, const int64_t *u2c, double *A, hipStream_t s) {
    BatchArgs B = batch_args(sec->bat);
    const unsigned grid = (unsigned)((B.n_reps + 255) / 256);
    hipLaunchKernelGGL((k_dense_k<KI, RT, TABLE>), dim3(grid), dim3(256), 0, s, B, sec->bt->dev.as<RT>(), u2c,
                       (uint64_t)sec->dim, (double2 *)A);
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

template <>
int dense_k_K<KI>(qs3_sector *sec, const int64_t *u2c, double *A, hipStream_t s) {
    if (sec->bat->ks->n_reps == 0 || sec->dim == 0) return QS3_OK;
    const bool tabm = sec->bat->ks->has_table;
    if constexpr (WIDE_OK) {
        if (sec->bt->wide)
            return tabm ? dense_k_t<uint64_t, true>(sec, u2c, A, s) : dense_k_t<uint64_t, false>(sec, u2c, A, s);
    }
    return tabm ? dense_k_t<uint32_t, true>(sec, u2c, A, s) : dense_k_t<uint32_t, false>(sec, u2c, A, s);
}
#endif

// ------------------------------------------------------------------ structure build
template <typename RT>
static int build_t(qs3_lattice *lat, const BinomTable &bt, KStructure *ks, hipStream_t s) {
    constexpr int K = KI;
    qs3_ctx *ctx = lat->ctx;
    LatArgs L = lat_args(lat);
    const RT *tab = bt.dev.as<RT>();
    BuildArgs A{L, bt.D, 0};
    uint64_t nblk = std::min<uint64_t>((bt.D + 1023) / 1024, 65536);
    nblk = std::max<uint64_t>(nblk, 1);
    A.chunk = (bt.D + nblk - 1) / nblk;
    nblk = (bt.D + A.chunk - 1) / A.chunk;
    DevBuf cnt;
    QS3_TRY(cnt.alloc(ctx, sizeof(unsigned long long) * (nblk + 1)));
    hipLaunchKernelGGL((k_count_reps<K, RT>), dim3(nblk), dim3(256), 0, s, A, tab,
                       cnt.as<unsigned long long>());
    QS3_HIP(hipGetLastError());
    std::vector<unsigned long long> h(nblk + 1, 0);
    QS3_HIP(hipMemcpyAsync(h.data(), cnt.ptr, sizeof(unsigned long long) * nblk,
                           hipMemcpyDeviceToHost, s));
    QS3_HIP(hipStreamSynchronize(s));
    unsigned long long tot = 0;
    for (uint64_t b = 0; b < nblk; ++b) {
        unsigned long long c = h[b];
        h[b] = tot;
        tot += c;
    }
    ks->n_reps = tot;
    QS3_REQUIRE(tot < (1ull << 32), QS3_EINVAL, "more than 2^32 representatives");
    QS3_HIP(hipMemcpyAsync(cnt.ptr, h.data(), sizeof(unsigned long long) * nblk,
                           hipMemcpyHostToDevice, s));
    QS3_TRY(ks->reps.alloc(ctx, sizeof(uint64_t) * std::max<uint64_t>(tot, 1)));
    hipLaunchKernelGGL((k_write_reps<K, RT>), dim3(nblk), dim3(256), 0, s, A, tab,
                       cnt.as<unsigned long long>(), ks->reps.as<uint64_t>());
    QS3_HIP(hipGetLastError());
    QS3_TRY(ks->stab.alloc(ctx, sizeof(uint16_t) * std::max<uint64_t>(tot, 1)));
    if (tot)
        hipLaunchKernelGGL((k_stab<K, RT>), dim3((tot + 255) / 256), dim3(256), 0, s, L, tab, tot,
                           ks->reps.as<uint64_t>(), ks->stab.as<uint16_t>());
    QS3_HIP(hipGetLastError());
    // directory over the rank range
    int Dbits = 1;
    while (Dbits < 64 && (1ull << Dbits) < bt.D) ++Dbits;
    int want = 1;
    while (want < 24 && (1ull << want) < tot) ++want;
    ks->dir_bits = std::min(want, Dbits);
    ks->dir_shift = Dbits - ks->dir_bits;
    uint64_t nb = (bt.D >> ks->dir_shift) + 1;
    QS3_TRY(ks->dir.alloc(ctx, sizeof(uint32_t) * (nb + 2)));
    hipLaunchKernelGGL(k_dir, dim3((nb + 256) / 256), dim3(256), 0, s, tot, ks->reps.as<uint64_t>(),
                       ks->dir_shift, nb, ks->dir.as<uint32_t>());
    QS3_HIP(hipGetLastError());
    // rank -> (representative, translation) table when it fits comfortably
    uint64_t tbytes = bt.D * sizeof(uint64_t);
    uint64_t used = ctx->used.load();
    uint64_t free_b = ctx->budget > used ? ctx->budget - used : 0;
    ks->has_table = tbytes <= ctx->table_limit && tbytes <= free_b / 4;
    if (ks->has_table) {
        QS3_TRY(ks->table.alloc(ctx, tbytes));
        hipLaunchKernelGGL((k_table<K, RT>), dim3((bt.D + 255) / 256), dim3(256), 0, s, A, tab,
                           ks->reps.as<uint64_t>(), ks->dir.as<uint32_t>(), ks->dir_shift,
                           ks->table.as<uint64_t>());
        QS3_HIP(hipGetLastError());
    }
#if QS3_INST_K <= 6
    // and the hops of every representative row, resolved once, when they fit
    // (K * degree entries per row instead of one per rank; the batched H.v
    // prefers them, the other kernels use the table or canonicalise)
    ks->hmax = K * lat->max_degree;
    const uint64_t hbytes = tot * (uint64_t)ks->hmax * sizeof(uint64_t);
    used = ctx->used.load();
    free_b = ctx->budget > used ? ctx->budget - used : 0;
    ks->has_hops = ks->hmax > 0 && tot > 0 && hbytes <= ctx->hop_list_limit && hbytes <= free_b / 4;
    if (ks->has_hops) {
        QS3_TRY(ks->hops.alloc(ctx, hbytes));
        BatchArgs HA{};
        HA.L = L;
        HA.n_reps = tot;
        HA.reps = ks->reps.as<uint64_t>();
        HA.stab = ks->stab.as<uint16_t>();
        HA.dir = ks->dir.as<uint32_t>();
        HA.dir_shift = ks->dir_shift;
        hipLaunchKernelGGL((k_hoplist<K, RT>), dim3((tot + 255) / 256), dim3(256), 0, s, HA, tab, ks->hmax,
                           ks->hops.as<uint64_t>());
        QS3_HIP(hipGetLastError());
    }
#endif
    ks->h_reps.resize(tot);
    ks->h_stab.resize(tot);
    if (tot) {
        QS3_HIP(hipMemcpyAsync(ks->h_reps.data(), ks->reps.ptr, sizeof(uint64_t) * tot,
                               hipMemcpyDeviceToHost, s));
        QS3_HIP(hipMemcpyAsync(ks->h_stab.data(), ks->stab.ptr, sizeof(uint16_t) * tot,
                               hipMemcpyDeviceToHost, s));
    }
    QS3_HIP(hipStreamSynchronize(s));
    return QS3_OK;
}

template <>
int build_kstruct_K<KI>(qs3_lattice *lat, const BinomTable &bt, KStructure *ks, hipStream_t s) {
    if constexpr (WIDE_OK) {
        if (bt.wide) return build_t<uint64_t>(lat, bt, ks, s);
    }
    return build_t<uint32_t>(lat, bt, ks, s);
}
#endif

// dense fixed-N_down blocks (every N_down)
template <>
int dense_u1_K<KI>(qs3_sector *sec, double *A, hipStream_t s) {
    const uint64_t d = sec->dim;
    if (d == 0) return QS3_OK;
    const unsigned grid = (unsigned)((d + 255) / 256);
    if constexpr (WIDE_OK) {
        if (sec->bt->wide) {
            hipLaunchKernelGGL((k_dense_u1<KI, uint64_t>), dim3(grid), dim3(256), 0, s, lat_args(sec->lat),
                               sec->bt->dev.as<uint64_t>(), (uint64_t)d, A);
            QS3_HIP(hipGetLastError());
            return QS3_OK;
        }
    }
    hipLaunchKernelGGL((k_dense_u1<KI, uint32_t>), dim3(grid), dim3(256), 0, s, lat_args(sec->lat),
                       sec->bt->dev.as<uint32_t>(), (uint32_t)d, A);
    QS3_HIP(hipGetLastError());
    return QS3_OK;
}

}  // namespace qs3
