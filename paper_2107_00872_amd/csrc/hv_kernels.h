// Matrix-free H.v of the XXZ model (Sec. 3.5, Alg. 9) for gfx950, pull form:
// every output row is one gather, so no atomics are needed.
//
//  * k_hv_u1      fixed-N_down sector, one row per lane, consecutive ranks on
//                 consecutive lanes (hops of the same down spin then land on
//                 near-contiguous ranks), binomial columns and the adjacency in
//                 LDS, XCD-contiguous row ranges.
//  * k_hv_batch   any number B of momentum sectors of one (lattice, N_down) in
//                 the [representative][sector] layout: a group of G lanes owns a
//                 row, resolves every hop once (rank -> representative index and
//                 translation, by table lookup or on-the-fly canonicalisation)
//                 and each lane applies the hop to its own sectors with their
//                 phases e^{ik.t}; one gather per hop reads G contiguous
//                 complex elements.
//  * structure build: representatives of every orbit, stabiliser sizes, the
//    search directory and the rank -> (representative, translation) table.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <type_traits>

#include "qs3_device.h"
#include "qs3_impl.h"
#include "qs3_hv.h"

namespace qs3 {

// ------------------------------------------------------------------ helpers
template <typename T>
struct Cplx;
template <>
struct Cplx<double> {
    using type = double2;
};
template <>
struct Cplx<float> {
    using type = float2;
};

// phase tables of at most this many entries are staged in LDS
constexpr int PHASE_LDS = 2048;

template <typename RT>
__device__ __forceinline__ void load_lds_tables(unsigned char *smem, const LatArgs &L,
                                                const RT *binom_g, int K, const RT **tab,
                                                const int **ptr, const uint16_t **nbr) {
    int ntab = K >= 2 ? (K - 1) << binom_shift(L.N) : 0;
    RT *s_tab = (RT *)smem;
    for (int i = threadIdx.x; i < ntab; i += blockDim.x) s_tab[i] = binom_g[i];
    int *s_ptr = (int *)(smem + ((ntab * sizeof(RT) + 15) & ~size_t(15)));
    for (int i = threadIdx.x; i <= L.N; i += blockDim.x) s_ptr[i] = L.ptr[i];
    uint16_t *s_nbr = (uint16_t *)(s_ptr + L.N + 1);
    for (int i = threadIdx.x; i < L.n_edges; i += blockDim.x) s_nbr[i] = L.nbr[i];
    __syncthreads();
    *tab = s_tab;
    *ptr = s_ptr;
    *nbr = s_nbr;
}

template <typename RT>
static size_t lds_bytes(const qs3_lattice *lat, int K) {
    size_t ntab = K >= 2 ? (size_t)(K - 1) << binom_shift(lat->N) : 0;
    return ((ntab * sizeof(RT) + 15) & ~size_t(15)) + sizeof(int) * (lat->N + 1) +
           sizeof(uint16_t) * lat->h_nbr.size() + 16;
}

// ------------------------------------------------------------------ U(1)
// One output row of the fixed-N_down H.v (Alg. 9 with sigma = all ranks):
// the Ising diagonal E_FM - sum over (down site, up neighbour) of Jz/2, and
// Jxy/2 v[rank'] for every hop of a down spin to an up neighbour.
//
// ZM > 0 (every site has exactly ZM neighbours, stored contiguously from
// ZM * site): all K*ZM candidate hops are ranked first and their gathers
// issued together (a slot that is no hop reads the row's own element and is
// dropped by a select), so a row waits for one memory latency instead of one
// per hop and carries no divergent branches; site-dependent couplings come
// with them, one (J_xy/2, J_z/2) pair per edge, and are summed in the plain
// loop's order.  ZM = 0: a plain loop over each down spin's neighbours (any
// degree, any couplings).
// UM (with ZM > 0): 1 one coupling constant, 2 site-dependent couplings, 0
// decided at run time from L.uniform.
template <int K, typename RT, typename VT, int ZM, int UM = 0>
__device__ __forceinline__ VT hv_row_u1(const LatArgs &L, const Binom<RT> &Bn, const int *ptr,
                                        const uint16_t *nbr, RT row, const VT *__restrict__ v) {
    int c[K > 0 ? K : 1];
    unrank<K, RT>(row, L.N, Bn, c);
    HopRanker<K, RT> hr;
    hr.init(c, Bn);
    if constexpr (ZM > 0) {
        constexpr int NH = (K > 0 ? K : 1) * ZM;
        VT x[NH];
        uint64_t okm = 0;  // bit h: slot h is a hop
        StaticFor<0, K>::run([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            const int e0 = c[m] * ZM;
#pragma unroll
            for (int q = 0; q < ZM; ++q) {
                RT rp;
                const bool up = hr.template hop<m>(c, row, (int)nbr[e0 + q], Bn, &rp);
                okm |= up ? (uint64_t(1) << (m * ZM + q)) : uint64_t(0);
                x[m * ZM + q] = v[up ? rp : row];
            }
        });
        if (UM == 1 || (UM == 0 && L.uniform)) {
            VT acc = 0;
#pragma unroll
            for (int h = 0; h < NH; ++h) acc += ((okm >> h) & 1u) ? x[h] : (VT)0;
            const VT diag = (VT)L.ez4 - (VT)L.u_jz_h * (VT)__popcll(okm);
            return diag * v[row] + (VT)L.u_jxy_h * acc;
        }
        VT acc = 0, dz = 0;
        StaticFor<0, K>::run([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            const int e0 = c[m] * ZM;
#pragma unroll
            for (int q = 0; q < ZM; ++q) {
                const bool up = (okm >> (m * ZM + q)) & 1u;
                VT jx, jzv;
                if constexpr (sizeof(VT) == 8) {
                    const double2 jp = L.jp_h[e0 + q];
                    jx = (VT)jp.x;
                    jzv = (VT)jp.y;
                } else {
                    const float2 jp = L.jp_hf[e0 + q];
                    jx = (VT)jp.x;
                    jzv = (VT)jp.y;
                }
                acc = up ? acc + jx * x[m * ZM + q] : acc;
                dz = up ? dz + jzv : dz;
            }
        });
        return ((VT)L.ez4 - dz) * v[row] + acc;
    }
    const bool UNIF = L.uniform != 0;
    VT acc = 0, dz = 0;
    StaticFor<0, K>::run([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        const int e0 = ptr[c[m]], e1 = ptr[c[m] + 1];
        for (int e = e0; e < e1; ++e) {
            const int j = nbr[e];
            RT rp;
            const bool up = hr.template hop<m>(c, row, j, Bn, &rp);
            if (up) {
                const VT x = v[rp];
                if (UNIF) {
                    acc += x;
                    dz += (VT)1;
                } else if (sizeof(VT) == 8) {
                    acc += (VT)L.jxy_h[e] * x;
                    dz += (VT)L.jz_h[e];
                } else {
                    acc += (VT)L.jxy_hf[e] * x;
                    dz += (VT)L.jz_hf[e];
                }
            }
        }
    });
    VT diag, off;
    if (UNIF) {
        diag = (VT)L.ez4 - (VT)L.u_jz_h * dz;
        off = (VT)L.u_jxy_h * acc;
    } else {
        diag = (VT)L.ez4 - dz;
        off = acc;
    }
    return diag * v[row] + off;
}

template <int K, typename RT, typename VT, typename OT, int ZM, int UM>
__global__ __launch_bounds__(256) void k_hv_u1(LatArgs L, const RT *__restrict__ binom_g, RT D,
                                               const VT *__restrict__ v, OT *__restrict__ w) {
    extern __shared__ __align__(16) unsigned char smem[];
    const RT *tab;
    const int *ptr;
    const uint16_t *nbr;
    load_lds_tables<RT>(smem, L, binom_g, K, &tab, &ptr, &nbr);
    Binom<RT> Bn{tab, binom_shift(L.N)};

    const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
    const uint64_t ntiles = ((uint64_t)D + 255) / 256;
    const uint64_t t0 = ntiles * lb / gridDim.x, t1 = ntiles * (lb + 1) / gridDim.x;
    for (uint64_t tile = t0; tile < t1; ++tile) {
        const uint64_t row64 = tile * 256 + threadIdx.x;
        if (row64 >= (uint64_t)D) break;
        w[row64] = (OT)hv_row_u1<K, RT, VT, ZM, UM>(L, Bn, ptr, nbr, (RT)row64, v);
    }
}

// ------------------------------------------------------------------ batch (momentum)

template <int K, typename RT, bool TABLE>
__device__ __forceinline__ void resolve_hop(const BatchArgs &A, const Binom<RT> &Bn, const Geom &g,
                                            const int (&c)[K > 0 ? K : 1], int m, int j, RT rp,
                                            uint32_t *u2, int *tx, int *ty, int *tz) {
    if (TABLE) {
        uint64_t ent = A.table[rp];
        *u2 = (uint32_t)ent;
        uint32_t t = (uint32_t)(ent >> 32);
        *tx = t & 1023u;
        *ty = (t >> 10) & 1023u;
        *tz = (t >> 20) & 1023u;
    } else {
        int n2[K > 0 ? K : 1], best[K > 0 ? K : 1];
#pragma unroll
        for (int t = 0; t < K; ++t) n2[t] = (t == m) ? j : c[t];
        sortK<K>(n2);
        canonicalize<K>(n2, g, best, *tx, *ty, *tz);
        uint64_t r = 0;
#pragma unroll
        for (int t = 0; t < K; ++t) r += (uint64_t)Bn.C(best[t], t + 1);
        *u2 = (uint32_t)find_rep(A.reps, A.dir, A.dir_shift, r);
    }
}

// Hop number h of a row (down spins ascending, each site's bonds in order):
// the spin index m and the edge e.
template <int K>
__device__ __forceinline__ void hop_of(int h, const int (&off)[K + 1], const int (&c)[K > 0 ? K : 1],
                                       const int *ptr, int *m, int *e) {
    int mm = 0;
#pragma unroll
    for (int t = 1; t < K; ++t) mm += (off[t] <= h) ? 1 : 0;
    int o = 0, cm = 0;
#pragma unroll
    for (int t = 0; t < K; ++t) {
        o = (t == mm) ? off[t] : o;
        cm = (t == mm) ? c[t] : cm;
    }
    *m = mm;
    *e = ptr[cm] + (h - o);
}

// The momentum kernel.  A group of G lanes owns a row; in rounds of G, lane l
// resolves hop (round * G + l) -- its target rank, representative index and
// translation (table lookup or canonicalisation), stabiliser ratio -- so the
// group pays each hop's resolution once and in parallel.  The resolved hops
// are then broadcast lane by lane with wavefront shuffles and every lane
// applies them to its own sectors with the phase e^{ik_b.t}; the gather of
// one hop reads G contiguous complex elements.  A lane's sectors are
// b = lane + (p * BPL + i) * G for pass p < NP and i < BPL: wide batches run
// several passes over the row (hops resolved again per pass) so that the
// accumulators and gathers of one pass fit in few registers.  Each sector
// sums its hops in hop order whatever BPL, NP and G are.  The phase table
// e^{2 pi i P / M} is staged in LDS after the lattice tables when
// A.ph_lds_off >= 0.
template <int K, typename RT, typename CT, typename OT, int MODE, int BPL, int NP>
__global__ __launch_bounds__(256) void k_hv_batch(BatchArgs A, const RT *__restrict__ binom_g,
                                                  const typename Cplx<CT>::type *__restrict__ v,
                                                  typename Cplx<OT>::type *__restrict__ w) {
    using C2 = typename Cplx<CT>::type;
    using O2 = typename Cplx<OT>::type;
    constexpr int QC = BPL >= 8 ? 1 : 8 / BPL;  // hops whose gathers are in flight together
    extern __shared__ __align__(16) unsigned char smem[];
    const RT *tab;
    const int *ptr;
    const uint16_t *nbr;
    const bool ph_lds = A.ph_lds_off >= 0;
    // the phase table in LDS; float32 products stage it as float2 (8-byte
    // entries, no conversion per term; the values are the same)
    constexpr bool F32 = std::is_same<CT, float>::value;
    double2 *s_ph = (double2 *)(smem + (ph_lds ? A.ph_lds_off : 0));
    float2 *s_phf = (float2 *)s_ph;
    if (ph_lds)
        for (int i = threadIdx.x; i < A.M; i += blockDim.x) {
            if constexpr (F32) s_phf[i] = make_float2((float)A.phase[i].x, (float)A.phase[i].y);
            else s_ph[i] = A.phase[i];
        }
    load_lds_tables<RT>(smem, A.L, binom_g, K, &tab, &ptr, &nbr);
    Binom<RT> Bn{tab, binom_shift(A.L.N)};
    Geom g{A.L.lx, A.L.ly, A.L.lz, A.L.lx * A.L.ly, A.L.coords, A.L.ns};

    const int G = A.G, B = A.B;
    const uint64_t LD = (uint64_t)A.ld;
    const bool UNIF = A.L.uniform != 0;
    const int lane = threadIdx.x % G;
    const int slot = threadIdx.x / G;
    const int rows_per_tile = blockDim.x / G;
    const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
    const uint64_t ntiles = (A.n_reps + rows_per_tile - 1) / rows_per_tile;
    const uint64_t t0 = ntiles * lb / gridDim.x, t1 = ntiles * (lb + 1) / gridDim.x;
    for (uint64_t tile = t0; tile < t1; ++tile) {
        const uint64_t u = tile * rows_per_tile + slot;
        if (u >= A.n_reps) break;
        const uint64_t R64 = A.reps[u];
        const RT R = (RT)R64;
        const int su = A.stab[u];
        const int ntu = su > 1 ? A.nt_of[u] : -1;
        int c[K > 0 ? K : 1];
        unrank<K, RT>(R, A.L.N, Bn, c);
        HopRanker<K, RT> hr;
        hr.init(c, Bn);
        int off[K + 1];
        off[0] = 0;
#pragma unroll
        for (int m = 0; m < K; ++m) off[m + 1] = off[m] + (ptr[c[m] + 1] - ptr[c[m]]);
        const int nh = off[K];
        const CT isq = (CT)(1.0 / A.L.sqrt_tab[su]);
#pragma unroll 1
        for (int pass = 0; pass < NP; ++pass) {
            int kx[BPL], ky[BPL], kz[BPL];
            bool bval[BPL];
#pragma unroll
            for (int i = 0; i < BPL; ++i) {
                const int b = lane + (pass * BPL + i) * G;
                bval[i] = b < B && (!A.active || A.active[b < B ? b : 0]);
                const int bb = bval[i] ? b : 0;
                kx[i] = A.kmul[3 * bb];
                ky[i] = A.kmul[3 * bb + 1];
                kz[i] = A.kmul[3 * bb + 2];
            }
            bool any = false;
#pragma unroll
            for (int i = 0; i < BPL; ++i) any |= bval[i];
            // a pass whose sectors are all absent or inactive in every lane of the group
            if (!__any(any)) continue;
            CT accr[BPL], acci[BPL];
#pragma unroll
            for (int i = 0; i < BPL; ++i) accr[i] = acci[i] = 0;
            CT dz = 0;
            for (int base = 0; base < nh; base += G) {
                // ---- resolve hop base + lane
                const int h = base + lane;
                uint32_t u2 = 0, tp = 0;
                int nt2 = -1;
                double coef = 0.0, jzv = 0.0;
                bool ok = false;
                if (h < nh) {
                    int m, e;
                    hop_of<K>(h, off, c, ptr, &m, &e);
                    const int j = nbr[e];
                    RT rp;
                    bool hop = true, ntf = true;
                    int tx = 0, ty = 0, tz = 0;
                    if (MODE == HOP_LISTS) {
                        // resolved once at structure build: occupied targets are ~0
                        const uint64_t ent = A.hops[u * (uint64_t)A.hmax + h];
                        hop = ent != ~0ull;
                        ntf = (ent & HOP_NT_BIT) != 0;
                        u2 = (uint32_t)ent;
                        const uint32_t t = (uint32_t)(ent >> 32);
                        tx = t & 1023u;
                        ty = (t >> 10) & 1023u;
                        tz = (t >> 20) & 1023u;
                    } else {
                        hop = hr.hop_rt(m, c, R, j, Bn, &rp);
                        if (hop) resolve_hop<K, RT, MODE == HOP_TABLE>(A, Bn, g, c, m, j, rp, &u2, &tx, &ty, &tz);
                    }
                    if (hop) {
                        const int s2 = ntf ? A.stab[u2] : 1;
                        nt2 = s2 > 1 ? A.nt_of[u2] : -1;
                        tp = (uint32_t)(tx | (ty << 10) | (tz << 20));
                        const double jxy = UNIF ? A.L.u_jxy_h : A.L.jxy_h[e];
                        coef = jxy * (s2 == 1 ? 1.0 : A.L.sqrt_tab[s2]) * (double)isq;  // sqrt(1) = 1
                        jzv = UNIF ? A.L.u_jz_h : A.L.jz_h[e];
                        ok = true;
                    }
                }
                // ---- apply the round's hops to this lane's sectors, QC hops at a
                // time (QC * BPL gathers): their gathers and phase loads are all
                // issued before any is consumed; a slot that applies nothing reads
                // element 0 and is dropped by a select.  Groups narrower than QC
                // go one hop at a time.
                const int cnt = min(G, nh - base);
                if (G < QC) {
                    for (int q = 0; q < cnt; ++q) {
                        const int bok = __shfl((int)ok, q, G);
                        if (!bok) continue;
                        const uint32_t bu = (uint32_t)__shfl((int)u2, q, G);
                        const uint32_t bt = (uint32_t)__shfl((int)tp, q, G);
                        const int bnt = __shfl(nt2, q, G);
                        const CT bc = (CT)__shfl(coef, q, G);
                        dz += (CT)__shfl(jzv, q, G);
                        const int tx = bt & 1023u, ty = (bt >> 10) & 1023u, tz = (bt >> 20) & 1023u;
                        const C2 *vrow = v + (uint64_t)bu * LD;
#pragma unroll
                        for (int i = 0; i < BPL; ++i) {
                            if (!bval[i]) continue;
                            const int b = lane + (pass * BPL + i) * G;
                            if (bnt >= 0 && !A.compat_nt[(size_t)bnt * LD + b]) continue;
                            int P = kx[i] * tx + ky[i] * ty + kz[i] * tz;
                            const int qq = (int)((double)P * A.invM);
                            P -= qq * A.M;
                            P += (P < 0) ? A.M : 0;
                            P -= (P >= A.M) ? A.M : 0;
                            CT phx, phy;
                            if constexpr (F32) {
                                const float2 q = ph_lds ? s_phf[P]
                                                        : make_float2((float)A.phase[P].x, (float)A.phase[P].y);
                                phx = q.x;
                                phy = q.y;
                            } else {
                                const double2 ph = ph_lds ? s_ph[P] : A.phase[P];
                                phx = (CT)ph.x;
                                phy = (CT)ph.y;
                            }
                            const C2 x = vrow[b];
                            const CT pr = bc * phx, pi = bc * phy;
                            accr[i] += pr * x.x - pi * x.y;
                            acci[i] += pr * x.y + pi * x.x;
                        }
                    }
                    continue;
                }
                for (int q0 = 0; q0 < cnt; q0 += QC) {
                    bool hok[QC];
                    uint32_t hu[QC];
                    int htx[QC], hty[QC], htz[QC], hnt[QC];
                    CT hc[QC];
#pragma unroll
                    for (int r = 0; r < QC; ++r) {
                        const int q = q0 + r;
                        const int qs = q < cnt ? q : 0;
                        const int okq = __shfl((int)ok, qs, G);
                        hok[r] = q < cnt && okq != 0;
                        hu[r] = (uint32_t)__shfl((int)u2, qs, G);
                        const uint32_t bt = (uint32_t)__shfl((int)tp, qs, G);
                        htx[r] = bt & 1023u;
                        hty[r] = (bt >> 10) & 1023u;
                        htz[r] = (bt >> 20) & 1023u;
                        hnt[r] = __shfl(nt2, qs, G);
                        hc[r] = (CT)__shfl(coef, qs, G);
                        const CT jz = (CT)__shfl(jzv, qs, G);
                        if (hok[r]) dz += jz;
                    }
                    C2 x[QC][BPL];
                    int Pi[QC][BPL];
#pragma unroll
                    for (int r = 0; r < QC; ++r) {
#pragma unroll
                        for (int i = 0; i < BPL; ++i) {
                            const int b = lane + (pass * BPL + i) * G;
                            bool use = hok[r] && bval[i];
                            if (use && hnt[r] >= 0) use = A.compat_nt[(size_t)hnt[r] * LD + b] != 0;
                            int P = kx[i] * htx[r] + ky[i] * hty[r] + kz[i] * htz[r];
                            const int qq = (int)((double)P * A.invM);
                            P -= qq * A.M;
                            P += (P < 0) ? A.M : 0;
                            P -= (P >= A.M) ? A.M : 0;
                            const uint64_t idx = use ? (uint64_t)hu[r] * LD + b : 0;
                            x[r][i] = v[idx];
                            Pi[r][i] = use ? P : 0;
                            if (!use) {
                                x[r][i].x = 0;
                                x[r][i].y = 0;
                            }
                        }
                    }
#pragma unroll
                    for (int r = 0; r < QC; ++r) {
#pragma unroll
                        for (int i = 0; i < BPL; ++i) {
                            CT phx, phy;
                            if constexpr (F32) {
                                const int Pq = Pi[r][i];
                                const float2 q = ph_lds ? s_phf[Pq]
                                                        : make_float2((float)A.phase[Pq].x, (float)A.phase[Pq].y);
                                phx = q.x;
                                phy = q.y;
                            } else {
                                const double2 ph = ph_lds ? s_ph[Pi[r][i]] : A.phase[Pi[r][i]];
                                phx = (CT)ph.x;
                                phy = (CT)ph.y;
                            }
                            const CT pr = hc[r] * phx, pi = hc[r] * phy;
                            accr[i] += pr * x[r][i].x - pi * x[r][i].y;
                            acci[i] += pr * x[r][i].y + pi * x[r][i].x;
                        }
                    }
                }
            }
            const CT diag = (CT)A.L.ez4 - dz;
            O2 *wrow = w + u * LD;
            const C2 *vself = v + u * LD;
#pragma unroll
            for (int i = 0; i < BPL; ++i) {
                if (!bval[i]) continue;
                const int b = lane + (pass * BPL + i) * G;
                const bool okr = ntu < 0 || A.compat_nt[(size_t)ntu * LD + b];
                O2 o;
                if (okr) {
                    C2 x = vself[b];
                    o.x = (OT)(diag * x.x + accr[i]);
                    o.y = (OT)(diag * x.y + acci[i]);
                } else {
                    o.x = 0;
                    o.y = 0;
                }
                wrow[b] = o;
            }
        }
    }
}

// A single momentum sector (a batch of one): one lane per representative row,
// and the row's hops taken QC at a time -- every hop of a chunk is resolved
// (hop-list entry, table entry or canonicalisation), then its stabiliser,
// phase and v gathers are all issued before any is consumed, so a row waits
// for a few memory latencies instead of one per hop.  The sum runs over the
// hops in the same order and with the same arithmetic as k_hv_batch.
template <int K, typename RT, typename CT, typename OT, int MODE>
__global__ __launch_bounds__(256) void k_hv_one(BatchArgs A, const RT *__restrict__ binom_g,
                                                const typename Cplx<CT>::type *__restrict__ v,
                                                typename Cplx<OT>::type *__restrict__ w) {
    using C2 = typename Cplx<CT>::type;
    using O2 = typename Cplx<OT>::type;
    constexpr int QC = 8;
    extern __shared__ __align__(16) unsigned char smem[];
    const RT *tab;
    const int *ptr;
    const uint16_t *nbr;
    load_lds_tables<RT>(smem, A.L, binom_g, K, &tab, &ptr, &nbr);
    if (A.active && !A.active[0]) return;  // an inactive sector's rows stay untouched
    Binom<RT> Bn{tab, binom_shift(A.L.N)};
    Geom g{A.L.lx, A.L.ly, A.L.lz, A.L.lx * A.L.ly, A.L.coords, A.L.ns};
    const bool UNIF = A.L.uniform != 0;
    const int kx = A.kmul[0], ky = A.kmul[1], kz = A.kmul[2];
    const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
    const uint64_t ntiles = (A.n_reps + 255) / 256;
    const uint64_t t0 = ntiles * lb / gridDim.x, t1 = ntiles * (lb + 1) / gridDim.x;
    for (uint64_t tile = t0; tile < t1; ++tile) {
        const uint64_t u = tile * 256 + threadIdx.x;
        if (u >= A.n_reps) break;
        const int su = A.stab[u];
        if (su > 1 && !A.compat_nt[A.nt_of[u]]) {
            w[u] = O2{0, 0};
            continue;
        }
        const RT R = (RT)A.reps[u];
        int c[K > 0 ? K : 1];
        unrank<K, RT>(R, A.L.N, Bn, c);
        HopRanker<K, RT> hr;
        hr.init(c, Bn);
        int off[K + 1];
        off[0] = 0;
#pragma unroll
        for (int m = 0; m < K; ++m) off[m + 1] = off[m] + (ptr[c[m] + 1] - ptr[c[m]]);
        const int nh = off[K];
        const CT isq = (CT)(1.0 / A.L.sqrt_tab[su]);
        const uint64_t *hrow = MODE == HOP_LISTS ? A.hops + u * (uint64_t)A.hmax : nullptr;
        CT accr = 0, acci = 0, dz = 0;
        for (int h0 = 0; h0 < nh; h0 += QC) {
            bool hok[QC], hnt[QC];
            uint32_t hu[QC];
            int he[QC], P[QC];
#pragma unroll
            for (int r = 0; r < QC; ++r) {
                const int h = h0 + r;
                int m = 0, e = 0;
                if (h < nh) hop_of<K>(h, off, c, ptr, &m, &e);
                he[r] = e;
                uint32_t u2 = 0;
                int tx = 0, ty = 0, tz = 0;
                bool ok = false, ntf = true;
                if (MODE == HOP_LISTS) {
                    const uint64_t ent = h < nh ? hrow[h] : ~0ull;
                    ok = ent != ~0ull;
                    ntf = (ent & HOP_NT_BIT) != 0;
                    u2 = (uint32_t)ent;
                    const uint32_t t = (uint32_t)(ent >> 32);
                    tx = t & 1023u;
                    ty = (t >> 10) & 1023u;
                    tz = (t >> 20) & 1023u;
                } else if (h < nh) {
                    const int j = nbr[e];
                    RT rp;
                    ok = hr.hop_rt(m, c, R, j, Bn, &rp);
                    if (ok) resolve_hop<K, RT, MODE == HOP_TABLE>(A, Bn, g, c, m, j, rp, &u2, &tx, &ty, &tz);
                }
                hok[r] = ok;
                hnt[r] = ok && ntf;
                hu[r] = ok ? u2 : (uint32_t)u;
                int p = kx * tx + ky * ty + kz * tz;
                const int qq = (int)((double)p * A.invM);
                p -= qq * A.M;
                p += (p < 0) ? A.M : 0;
                p -= (p >= A.M) ? A.M : 0;
                P[r] = ok ? p : 0;
            }
            // every gather of the chunk in flight together
            int s2[QC];
            C2 x[QC];
            double2 ph[QC];
#pragma unroll
            for (int r = 0; r < QC; ++r) {
                s2[r] = hnt[r] ? A.stab[hu[r]] : 1;
                x[r] = v[hu[r]];
                ph[r] = A.phase[P[r]];
            }
#pragma unroll
            for (int r = 0; r < QC; ++r) {
                if (!hok[r]) continue;
                const int e = he[r];
                dz += (CT)(UNIF ? A.L.u_jz_h : A.L.jz_h[e]);
                // a target whose stabiliser is incompatible with k is not in the sector
                if (s2[r] > 1 && !A.compat_nt[A.nt_of[hu[r]]]) continue;
                const double jxy = UNIF ? A.L.u_jxy_h : A.L.jxy_h[e];
                const CT hc = (CT)(jxy * (s2[r] == 1 ? 1.0 : A.L.sqrt_tab[s2[r]]) * (double)isq);
                const CT pr = hc * (CT)ph[r].x, pi = hc * (CT)ph[r].y;
                accr += pr * x[r].x - pi * x[r].y;
                acci += pr * x[r].y + pi * x[r].x;
            }
        }
        const CT diag = (CT)A.L.ez4 - dz;
        const C2 xs = v[u];
        O2 o;
        o.x = (OT)(diag * xs.x + accr);
        o.y = (OT)(diag * xs.y + acci);
        w[u] = o;
    }
}

// A single momentum sector with per-representative hop lists on a lattice with
// one exchange and one Ising constant: a row needs neither its state nor the
// lattice tables, its hop-list entries (target representative and
// translation, ~0 for an occupied target) give every term.  A lane loads its
// row's entries (16-byte loads), then issues the v gathers of every hop of the
// row together, so a row waits for two memory round trips.  Rows whose own
// stabiliser and whose targets' stabilisers are all trivial (no entry carries
// HOP_NT_BIT) -- every row of a lattice whose orbits are all full -- take each
// term as one LDS read of (J_xy/2) e^{ik.t}, staged per cell translation t
// (from A.tP, the phase index of t, and the phase table), in a branch-free
// loop (an empty slot is dropped by a select).  For a flagged target the
// class byte A.gcls (its stabiliser size s, 0 when it is not in the sector) is
// gathered with v, and a wavefront holding such rows evaluates every term as
// (J_xy/2) sqrt(s_b) / sqrt(s_a) e^{ik.t} instead.  LPR = 2 splits a row's
// slots between two neighbouring lanes (half the registers per lane, so a
// sector of a few hundred thousand rows is resident in one wave of the
// machine), each summing its half in hop order, and the first half's sums
// are added to the second's.  The phase indices, the phase table and the
// first row's entries share one memory round trip.
// Dynamic LDS: the staged terms (N_T CT pairs), the phase table (M double2),
// sqrt(0..15) and the phase indices (N_T uint16).  The terms and their
// arithmetic are those of k_hv_one and k_hv_batch (with sqrt(1) = 1 exactly,
// (CT)(J_xy/2 * 1 * 1) * (CT)phase is the staged term), and with LPR = 1 so is
// their order.
template <typename CT, typename OT, int HM, int LPR>
__global__ __launch_bounds__(256) void k_hv_one_lists(BatchArgs A,
                                                      const typename Cplx<CT>::type *__restrict__ v,
                                                      typename Cplx<OT>::type *__restrict__ w) {
    using C2 = typename Cplx<CT>::type;
    using O2 = typename Cplx<OT>::type;
    static_assert(LPR == 1 || LPR == 2, "one or two lanes per row");
    constexpr int HH = HM / LPR;      // hop slots per lane
    constexpr int RPB = 256 / LPR;    // rows per block and tile
    extern __shared__ __align__(16) unsigned char smem[];
    if (A.active && !A.active[0]) return;  // an inactive sector's rows stay untouched
    const int lx = A.L.lx, lxy = A.L.lx * A.L.ly;
    const int nt = lxy * A.L.lz;
    const int M = A.M;
    C2 *s_pt = (C2 *)smem;
    double2 *s_phase = (double2 *)(smem + (((size_t)nt * sizeof(C2) + 15) & ~size_t(15)));
    double *s_sq = (double *)(s_phase + M);
    uint16_t *s_P = (uint16_t *)(s_sq + 16);
    const double jxy = A.L.u_jxy_h;
    const int hmax = A.hmax;
    const CT jz = (CT)A.L.u_jz_h;
    const int sub = LPR == 1 ? 0 : (int)(threadIdx.x & 1u);  // which half of the row's slots
    const int rl = (int)threadIdx.x / LPR;
    const uint32_t lb = xcd_block(blockIdx.x, gridDim.x);
    const uint64_t ntiles = (A.n_reps + RPB - 1) / RPB;
    const uint64_t t0 = ntiles * lb / gridDim.x, t1 = ntiles * (lb + 1) / gridDim.x;
    uint64_t ent[HH];
    int su = 1;
    C2 xs = C2{0, 0};
    // the lane's slots of a row's entries, the row's stabiliser and own element
    auto load_row = [&](uint64_t u) {
        const uint64_t *hrow = A.hops + u * (uint64_t)hmax;
        if (LPR == 1 && (hmax & 1) == 0) {
            const uint4 *p = (const uint4 *)hrow;
#pragma unroll
            for (int i = 0; i < HH / 2; ++i) {
                uint4 q = make_uint4(~0u, ~0u, ~0u, ~0u);
                if (2 * i < hmax) q = p[i];
                ent[2 * i] = (uint64_t)q.x | ((uint64_t)q.y << 32);
                ent[2 * i + 1] = (uint64_t)q.z | ((uint64_t)q.w << 32);
            }
        } else {
#pragma unroll
            for (int j = 0; j < HH; ++j) {
                const int h = sub * HH + j;
                ent[j] = h < hmax ? hrow[h] : ~0ull;
            }
        }
        su = A.stab[u];
        xs = v[u];
    };
    // ---- one round trip: phase indices (first 1024), phase table (first 256),
    // sqrt(0..15) and the first row's entries
    uint16_t rP[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int t = threadIdx.x + 256 * j;
        rP[j] = t < nt ? A.tP[t] : 0;
    }
    double2 rph = make_double2(0.0, 0.0);
    if ((int)threadIdx.x < M) rph = A.phase[threadIdx.x];
    const double rsq = threadIdx.x < 16 ? A.L.sqrt_tab[threadIdx.x < (unsigned)A.L.N ? threadIdx.x : 0] : 0.0;
    const uint64_t u0 = t0 * RPB + rl;
    if (t0 < t1 && u0 < A.n_reps) load_row(u0);
    if ((int)threadIdx.x < M) s_phase[threadIdx.x] = rph;
    for (int i = threadIdx.x + 256; i < M; i += 256) s_phase[i] = A.phase[i];
    if (threadIdx.x < 16) s_sq[threadIdx.x] = rsq;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int t = threadIdx.x + 256 * j;
        if (t < nt) s_P[t] = rP[j];
    }
    for (int t = threadIdx.x + 1024; t < nt; t += 256) s_P[t] = A.tP[t];
    __syncthreads();
    for (int t = threadIdx.x; t < nt; t += 256) {
        const double2 ph = s_phase[s_P[t]];
        const CT hc = (CT)jxy;
        s_pt[t] = C2{hc * (CT)ph.x, hc * (CT)ph.y};
    }
    __syncthreads();
    for (uint64_t tile = t0; tile < t1; ++tile) {
        const uint64_t u = tile * RPB + rl;
        if (u >= A.n_reps) break;  // both lanes of a row leave together
        if (tile != t0) load_row(u);
        uint32_t hu[HH];
        int ti[HH];
        uint32_t okm = 0, flm = 0;  // bit j: slot j is a hop; its target's stabiliser is non-trivial
#pragma unroll
        for (int j = 0; j < HH; ++j) {
            const bool ok = ent[j] != ~0ull;
            hu[j] = ok ? (uint32_t)ent[j] : (uint32_t)u;
            okm |= ok ? (1u << j) : 0u;
            flm |= (ok && (ent[j] & HOP_NT_BIT)) ? (1u << j) : 0u;
            const uint32_t t = (uint32_t)(ent[j] >> 32);
            ti[j] = ok ? (int)(t & 1023u) + lx * (int)((t >> 10) & 1023u) + lxy * (int)((t >> 20) & 1023u) : 0;
        }
        // every gather of the lane's slots in flight together, with the class
        // of each flagged target and of the row itself
        C2 x[HH];
        int cl[HH];
#pragma unroll
        for (int j = 0; j < HH; ++j) {
            x[j] = v[hu[j]];
            cl[j] = ((flm >> j) & 1u) ? (int)A.gcls[hu[j]] : 1;
        }
        const int cu = su > 1 ? (int)A.gcls[u] : 1;
        CT accr = 0, acci = 0, dz = 0;
        if (!__any(su > 1 || flm != 0)) {
#pragma unroll
            for (int j = 0; j < HH; ++j) {
                const bool ok = (okm >> j) & 1u;
                const C2 pt = s_pt[ti[j]];
                const CT ar = accr + (pt.x * x[j].x - pt.y * x[j].y);
                const CT ai = acci + (pt.x * x[j].y + pt.y * x[j].x);
                accr = ok ? ar : accr;
                acci = ok ? ai : acci;
                dz = ok ? dz + jz : dz;
            }
        } else {
            // a target outside the sector (class 0) contributes only to the diagonal
            const CT isq = (CT)(1.0 / s_sq[cu > 0 ? cu : 1]);
#pragma unroll
            for (int j = 0; j < HH; ++j) {
                const bool ok = (okm >> j) & 1u;
                const bool use = ok && cl[j] != 0;
                const double2 ph = s_phase[s_P[ti[j]]];
                const CT hc = (CT)(jxy * s_sq[cl[j]] * (double)isq);
                const CT pr = hc * (CT)ph.x, pi = hc * (CT)ph.y;
                const CT ar = accr + (pr * x[j].x - pi * x[j].y);
                const CT ai = acci + (pr * x[j].y + pi * x[j].x);
                accr = use ? ar : accr;
                acci = use ? ai : acci;
                dz = ok ? dz + jz : dz;
            }
        }
        if (LPR == 2) {
            // first half's sums plus the second half's, in that order on both lanes
            const CT orr = __shfl_xor(accr, 1), oi = __shfl_xor(acci, 1), od = __shfl_xor(dz, 1);
            accr = sub == 0 ? accr + orr : orr + accr;
            acci = sub == 0 ? acci + oi : oi + acci;
            dz = sub == 0 ? dz + od : od + dz;
        }
        if (sub == 0) {
            const bool zero = cu == 0;  // the row's own orbit is not in the sector
            const CT diag = (CT)A.L.ez4 - dz;
            O2 o;
            o.x = zero ? (OT)0 : (OT)(diag * xs.x + accr);
            o.y = zero ? (OT)0 : (OT)(diag * xs.y + acci);
            w[u] = o;
        }
    }
}

// ------------------------------------------------------------------ structure build
template <int K, typename RT>
__device__ __forceinline__ bool is_orbit_min(const int (&c)[K > 0 ? K : 1], const Geom &g) {
    // early-exit variant of canonicalize(): is c itself the minimum image?
    int x[K > 0 ? K : 1], y[K > 0 ? K : 1], z[K > 0 ? K : 1], sb[K > 0 ? K : 1];
#pragma unroll
    for (int m = 0; m < K; ++m) {
        uint32_t p = g.coords[c[m]];
        x[m] = p & 1023u;
        y[m] = (p >> 10) & 1023u;
        z[m] = (p >> 20) & 1023u;
        sb[m] = (int)(p >> 30);
    }
    // c must have coordinate 0 occupied on every axis
    bool hx = g.lx == 1, hy = g.ly == 1, hz = g.lz == 1;
#pragma unroll
    for (int m = 0; m < K; ++m) {
        hx |= x[m] == 0;
        hy |= y[m] == 0;
        hz |= z[m] == 0;
    }
    if (K == 0) return true;  // the empty set is its own orbit
    if (!(hx && hy && hz)) return false;
    const int nx = g.lx > 1 ? K : 1, ny = g.ly > 1 ? K : 1, nz = g.lz > 1 ? K : 1;
    for (int iz = 0; iz < nz; ++iz) {
        int tz = z[iz] == 0 ? 0 : g.lz - z[iz];
        for (int iy = 0; iy < ny; ++iy) {
            int ty = y[iy] == 0 ? 0 : g.ly - y[iy];
            for (int ix = 0; ix < nx; ++ix) {
                int tx = x[ix] == 0 ? 0 : g.lx - x[ix];
                int img[K > 0 ? K : 1];
#pragma unroll
                for (int m = 0; m < K; ++m)
                    img[m] = sb[m] + g.ns * (wrap_add(x[m], tx, g.lx) + g.lx * wrap_add(y[m], ty, g.ly) +
                                             g.lxy * wrap_add(z[m], tz, g.lz));
                sortK<K>(img);
                int cmp = 0;
#pragma unroll
                for (int m = K - 1; m >= 0; --m)
                    if (cmp == 0) cmp = (img[m] < c[m]) ? -1 : (img[m] > c[m] ? 1 : 0);
                if (cmp < 0) return false;
            }
        }
    }
    return true;
}


template <int K, typename RT>
__global__ __launch_bounds__(256) void k_count_reps(BuildArgs A, const RT *__restrict__ binom_g,
                                                    unsigned long long *counts) {
    Binom<RT> Bn{binom_g, binom_shift(A.L.N)};
    Geom g{A.L.lx, A.L.ly, A.L.lz, A.L.lx * A.L.ly, A.L.coords, A.L.ns};
    const uint64_t lo = (uint64_t)blockIdx.x * A.chunk;
    const uint64_t hi = min(A.D, lo + A.chunk);
    unsigned long long cnt = 0;
    for (uint64_t r = lo + threadIdx.x; r < hi; r += blockDim.x) {
        int c[K > 0 ? K : 1];
        unrank<K, RT>((RT)r, A.L.N, Bn, c);
        cnt += is_orbit_min<K, RT>(c, g) ? 1 : 0;
    }
    __shared__ unsigned long long red[256];
    red[threadIdx.x] = cnt;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = red[0];
}

template <int K, typename RT>
__global__ __launch_bounds__(256) void k_write_reps(BuildArgs A, const RT *__restrict__ binom_g,
                                                    const unsigned long long *offsets,
                                                    uint64_t *reps) {
    Binom<RT> Bn{binom_g, binom_shift(A.L.N)};
    Geom g{A.L.lx, A.L.ly, A.L.lz, A.L.lx * A.L.ly, A.L.coords, A.L.ns};
    const uint64_t lo = (uint64_t)blockIdx.x * A.chunk;
    const uint64_t hi = min(A.D, lo + A.chunk);
    __shared__ unsigned int wave_cnt[4];
    unsigned long long base = offsets[blockIdx.x];
    const int wid = threadIdx.x / 64, ln = threadIdx.x % 64;
    for (uint64_t r0 = lo; r0 < hi; r0 += blockDim.x) {
        uint64_t r = r0 + threadIdx.x;
        bool f = false;
        if (r < hi) {
            int c[K > 0 ? K : 1];
            unrank<K, RT>((RT)r, A.L.N, Bn, c);
            f = is_orbit_min<K, RT>(c, g);
        }
        unsigned long long bal = __ballot(f);
        unsigned int before = __popcll(bal & ((1ull << ln) - 1ull));
        if (ln == 0) wave_cnt[wid] = __popcll(bal);
        __syncthreads();
        unsigned int woff = 0, tot = 0;
        for (int k = 0; k < (int)(blockDim.x / 64); ++k) {
            if (k < wid) woff += wave_cnt[k];
            tot += wave_cnt[k];
        }
        if (f) reps[base + woff + before] = r;
        base += tot;
        __syncthreads();
    }
}

template <int K, typename RT>
__global__ __launch_bounds__(256) void k_stab(LatArgs L, const RT *__restrict__ binom_g,
                                              uint64_t n_reps, const uint64_t *__restrict__ reps,
                                              uint16_t *stab) {
    Binom<RT> Bn{binom_g, binom_shift(L.N)};
    Geom g{L.lx, L.ly, L.lz, L.lx * L.ly, L.coords, L.ns};
    uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_reps) return;
    int c[K > 0 ? K : 1];
    unrank<K, RT>((RT)reps[u], L.N, Bn, c);
    int x[K > 0 ? K : 1], y[K > 0 ? K : 1], z[K > 0 ? K : 1], sb[K > 0 ? K : 1];
#pragma unroll
    for (int m = 0; m < K; ++m) {
        uint32_t p = g.coords[c[m]];
        x[m] = p & 1023u;
        y[m] = (p >> 10) & 1023u;
        z[m] = (p >> 20) & 1023u;
        sb[m] = (int)(p >> 30);
    }
    // every stabiliser element maps the representative onto itself, so it is
    // one of the candidate shifts; count each distinct shift once (first spin
    // carrying a given coordinate value).
    int count = 0;
    const int nx = g.lx > 1 ? K : 1, ny = g.ly > 1 ? K : 1, nz = g.lz > 1 ? K : 1;
    for (int iz = 0; iz < nz; ++iz) {
        bool dz = false;
        for (int q = 0; q < iz; ++q) dz |= z[q] == z[iz];
        if (dz) continue;
        int tz = z[iz] == 0 ? 0 : g.lz - z[iz];
        for (int iy = 0; iy < ny; ++iy) {
            bool dy = false;
            for (int q = 0; q < iy; ++q) dy |= y[q] == y[iy];
            if (dy) continue;
            int ty = y[iy] == 0 ? 0 : g.ly - y[iy];
            for (int ix = 0; ix < nx; ++ix) {
                bool dx = false;
                for (int q = 0; q < ix; ++q) dx |= x[q] == x[ix];
                if (dx) continue;
                int tx = x[ix] == 0 ? 0 : g.lx - x[ix];
                int img[K > 0 ? K : 1];
#pragma unroll
                for (int m = 0; m < K; ++m)
                    img[m] = sb[m] + g.ns * (wrap_add(x[m], tx, g.lx) + g.lx * wrap_add(y[m], ty, g.ly) +
                                             g.lxy * wrap_add(z[m], tz, g.lz));
                sortK<K>(img);
                bool eq = true;
#pragma unroll
                for (int m = 0; m < K; ++m) eq &= img[m] == c[m];
                count += eq ? 1 : 0;
            }
        }
    }
    stab[u] = (uint16_t)(K == 0 ? L.lx * L.ly * L.lz : count);
}

static __global__ void k_dir(uint64_t n_reps, const uint64_t *__restrict__ reps, int shift, uint64_t nb,
                      uint32_t *dir) {
    uint64_t b = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nb) return;
    uint64_t key = b << shift;
    uint64_t lo = 0, hi = n_reps;
    while (lo < hi) {
        uint64_t mid = (lo + hi) >> 1;
        if (reps[mid] < key) lo = mid + 1; else hi = mid;
    }
    dir[b] = (uint32_t)lo;
}

template <int K, typename RT>
__global__ __launch_bounds__(256) void k_table(BuildArgs A, const RT *__restrict__ binom_g,
                                               const uint64_t *__restrict__ reps,
                                               const uint32_t *__restrict__ dir, int shift,
                                               uint64_t *table) {
    Binom<RT> Bn{binom_g, binom_shift(A.L.N)};
    Geom g{A.L.lx, A.L.ly, A.L.lz, A.L.lx * A.L.ly, A.L.coords, A.L.ns};
    uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= A.D) return;
    int c[K > 0 ? K : 1], best[K > 0 ? K : 1];
    unrank<K, RT>((RT)r, A.L.N, Bn, c);
    int tx, ty, tz;
    canonicalize<K>(c, g, best, tx, ty, tz);
    uint64_t rr = 0;
#pragma unroll
    for (int t = 0; t < K; ++t) rr += (uint64_t)Bn.C(best[t], t + 1);
    uint32_t u = (uint32_t)find_rep(reps, dir, shift, rr);
    table[r] = pack_ent(u, tx, ty, tz);
}

// Hop lists: for representative u, entry h (the row's hops in the kernel's
// order: down spins ascending, each site's bonds in order) is the packed
// (representative index, translation) of the hop's target, with HOP_NT_BIT
// when the target's stabiliser is non-trivial, or ~0 when the target site is
// occupied; entries nh..hmax-1 are ~0.  A.stab must be complete.
template <int K, typename RT>
__global__ __launch_bounds__(256) void k_hoplist(BatchArgs A, const RT *__restrict__ binom_g, int hmax,
                                                 uint64_t *__restrict__ hops) {
    Binom<RT> Bn{binom_g, binom_shift(A.L.N)};
    Geom g{A.L.lx, A.L.ly, A.L.lz, A.L.lx * A.L.ly, A.L.coords, A.L.ns};
    const uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= A.n_reps) return;
    const RT R = (RT)A.reps[u];
    int c[K > 0 ? K : 1];
    unrank<K, RT>(R, A.L.N, Bn, c);
    HopRanker<K, RT> hr;
    hr.init(c, Bn);
    uint64_t *out = hops + u * (uint64_t)hmax;
    int h = 0;
    StaticFor<0, K>::run([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        for (int e = A.L.ptr[c[m]]; e < A.L.ptr[c[m] + 1]; ++e, ++h) {
            const int j = A.L.nbr[e];
            RT rp;
            uint64_t ent = ~0ull;
            if (hr.template hop<m>(c, R, j, Bn, &rp)) {
                uint32_t u2;
                int tx, ty, tz;
                resolve_hop<K, RT, false>(A, Bn, g, c, m, j, rp, &u2, &tx, &ty, &tz);
                ent = pack_ent(u2, tx, ty, tz) | (A.stab[u2] > 1 ? HOP_NT_BIT : 0ull);
            }
            out[h] = ent;
        }
    });
    for (; h < hmax; ++h) out[h] = ~0ull;
}

// ------------------------------------------------------------------ dense blocks
// The dense Hamiltonian block of a sector (the matrix Alg. 4 / Alg. 8 build),
// column major (element (i, j) at j * d + i), one row per thread from the
// same hop rules as H.v; A must be zero on entry.  Fixed N_down:
template <int K, typename RT>
__global__ __launch_bounds__(256) void k_dense_u1(LatArgs L, const RT *__restrict__ binom_g, RT D,
                                                  double *__restrict__ A) {
    Binom<RT> Bn{binom_g, binom_shift(L.N)};
    const uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= (uint64_t)D) return;
    const uint64_t d = (uint64_t)D;
    int c[K > 0 ? K : 1];
    unrank<K, RT>((RT)r, L.N, Bn, c);
    HopRanker<K, RT> hr;
    hr.init(c, Bn);
    double dz = 0.0;
    StaticFor<0, K>::run([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        for (int e = L.ptr[c[m]]; e < L.ptr[c[m] + 1]; ++e) {
            RT rp;
            if (!hr.template hop<m>(c, (RT)r, (int)L.nbr[e], Bn, &rp)) continue;
            A[(uint64_t)rp * d + r] += L.uniform ? L.u_jxy_h : L.jxy_h[e];
            dz += L.uniform ? L.u_jz_h : L.jz_h[e];
        }
    });
    A[r * d + r] += L.ez4 - dz;
}

// Momentum sector (a batch of one): row u of the union is basis state
// u2c[u] (-1: not in the sector); elements as in k_hv_batch.
template <int K, typename RT, bool TABLE>
__global__ __launch_bounds__(256) void k_dense_k(BatchArgs A, const RT *__restrict__ binom_g,
                                                 const int64_t *__restrict__ u2c, uint64_t d,
                                                 double2 *__restrict__ M) {
    Binom<RT> Bn{binom_g, binom_shift(A.L.N)};
    Geom g{A.L.lx, A.L.ly, A.L.lz, A.L.lx * A.L.ly, A.L.coords, A.L.ns};
    const uint64_t u = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= A.n_reps) return;
    const int64_t i = u2c[u];
    if (i < 0) return;
    const RT R = (RT)A.reps[u];
    int c[K > 0 ? K : 1];
    unrank<K, RT>(R, A.L.N, Bn, c);
    HopRanker<K, RT> hr;
    hr.init(c, Bn);
    const double isq = 1.0 / A.L.sqrt_tab[A.stab[u]];
    double dz = 0.0;
    StaticFor<0, K>::run([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        for (int e = A.L.ptr[c[m]]; e < A.L.ptr[c[m] + 1]; ++e) {
            const int j = A.L.nbr[e];
            RT rp;
            if (!hr.template hop<m>(c, R, j, Bn, &rp)) continue;
            uint32_t u2;
            int tx, ty, tz;
            resolve_hop<K, RT, TABLE>(A, Bn, g, c, m, j, rp, &u2, &tx, &ty, &tz);
            dz += A.L.uniform ? A.L.u_jz_h : A.L.jz_h[e];
            const int64_t jc = u2c[u2];
            if (jc < 0) continue;
            const double coef = (A.L.uniform ? A.L.u_jxy_h : A.L.jxy_h[e]) * A.L.sqrt_tab[A.stab[u2]] * isq;
            int P = A.kmul[0] * tx + A.kmul[1] * ty + A.kmul[2] * tz;
            P %= A.M;
            const double2 ph = A.phase[P];
            double2 &dst = M[(uint64_t)jc * d + (uint64_t)i];
            dst.x += coef * ph.x;
            dst.y += coef * ph.y;
        }
    });
    M[(uint64_t)i * d + (uint64_t)i].x += A.L.ez4 - dz;
}

// ------------------------------------------------------------------ debug rows
template <int K, typename RT>
__global__ void k_row_u1(LatArgs L, const RT *binom_g, RT row, int cap, int64_t *cols,
                         double *vals, double *diag, int *nnz) {
    Binom<RT> Bn{binom_g, binom_shift(L.N)};
    int c[K > 0 ? K : 1];
    unrank<K, RT>(row, L.N, Bn, c);
    HopRanker<K, RT> hr;
    hr.init(c, Bn);
    int n = 0;
    double dz = 0;
    StaticFor<0, K>::run([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        for (int e = L.ptr[c[m]]; e < L.ptr[c[m] + 1]; ++e) {
            int j = L.nbr[e];
            RT rp;
            const bool up = hr.template hop<m>(c, row, j, Bn, &rp);
            if (!up) continue;
            double jxy = L.uniform ? L.u_jxy_h : L.jxy_h[e];
            dz += L.uniform ? L.u_jz_h : L.jz_h[e];
            if (n < cap) {
                cols[n] = (int64_t)rp;
                vals[n] = jxy;
            }
            ++n;
        }
    });
    *diag = L.ez4 - dz;
    *nnz = n;
}

template <int K, typename RT, bool TABLE>
__global__ void k_row_k(BatchArgs A, const RT *binom_g, uint64_t u, int cap, int64_t *cols,
                        double *vals, double *diag, int *nnz) {
    Binom<RT> Bn{binom_g, binom_shift(A.L.N)};
    Geom g{A.L.lx, A.L.ly, A.L.lz, A.L.lx * A.L.ly, A.L.coords, A.L.ns};
    const RT R = (RT)A.reps[u];
    const int su = A.stab[u];
    int c[K > 0 ? K : 1];
    unrank<K, RT>(R, A.L.N, Bn, c);
    HopRanker<K, RT> hr;
    hr.init(c, Bn);
    int n = 0;
    double dz = 0;
    const double isq = 1.0 / A.L.sqrt_tab[su];
    StaticFor<0, K>::run([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        for (int e = A.L.ptr[c[m]]; e < A.L.ptr[c[m] + 1]; ++e) {
            int j = A.L.nbr[e];
            RT rp;
            const bool up = hr.template hop<m>(c, R, j, Bn, &rp);
            if (!up) continue;
            uint32_t u2;
            int tx, ty, tz;
            resolve_hop<K, RT, TABLE>(A, Bn, g, c, m, j, rp, &u2, &tx, &ty, &tz);
            const int s2 = A.stab[u2];
            const int nt2 = s2 > 1 ? A.nt_of[u2] : -1;
            dz += A.L.uniform ? A.L.u_jz_h : A.L.jz_h[e];
            if (nt2 >= 0 && !A.compat_nt[nt2]) continue;  // B == 1
            const double coef = (A.L.uniform ? A.L.u_jxy_h : A.L.jxy_h[e]) * A.L.sqrt_tab[s2] * isq;
            int P = A.kmul[0] * tx + A.kmul[1] * ty + A.kmul[2] * tz;
            P %= A.M;
            if (n < cap) {
                cols[n] = (int64_t)u2;
                vals[2 * n] = coef * A.phase[P].x;
                vals[2 * n + 1] = coef * A.phase[P].y;
            }
            ++n;
        }
    });
    *diag = A.L.ez4 - dz;
    *nnz = n;
}


// ------------------------------------------------------------------ small sectors
// One row of a single momentum sector (a batch of one, union layout), hops
// resolved one after the other.
template <int K, typename RT, bool TABLE>
__device__ __forceinline__ double2 hv_row_k1(const BatchArgs &A, const Binom<RT> &Bn, const Geom &g,
                                             const int *ptr, const uint16_t *nbr, uint64_t u,
                                             const double2 *__restrict__ v) {
    const int su = A.stab[u];
    if (su > 1 && !A.compat_nt[A.nt_of[u]]) return make_double2(0.0, 0.0);
    const bool UNIF = A.L.uniform != 0;
    const RT R = (RT)A.reps[u];
    int c[K > 0 ? K : 1];
    unrank<K, RT>(R, A.L.N, Bn, c);
    HopRanker<K, RT> hr;
    hr.init(c, Bn);
    const double isq = 1.0 / A.L.sqrt_tab[su];
    double ar = 0, ai = 0, dz = 0;
    StaticFor<0, K>::run([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        for (int e = ptr[c[m]]; e < ptr[c[m] + 1]; ++e) {
            const int j = nbr[e];
            RT rp;
            if (!hr.template hop<m>(c, R, j, Bn, &rp)) continue;
            uint32_t u2;
            int tx, ty, tz;
            resolve_hop<K, RT, TABLE>(A, Bn, g, c, m, j, rp, &u2, &tx, &ty, &tz);
            dz += UNIF ? A.L.u_jz_h : A.L.jz_h[e];
            const int s2 = A.stab[u2];
            if (s2 > 1 && !A.compat_nt[A.nt_of[u2]]) continue;
            const double coef = (UNIF ? A.L.u_jxy_h : A.L.jxy_h[e]) * A.L.sqrt_tab[s2] * isq;
            int P = A.kmul[0] * tx + A.kmul[1] * ty + A.kmul[2] * tz;
            P %= A.M;
            const double2 ph = A.phase[P], x = v[u2];
            const double pr = coef * ph.x, pi = coef * ph.y;
            ar += pr * x.x - pi * x.y;
            ai += pr * x.y + pi * x.x;
        }
    });
    const double diag = A.L.ez4 - dz;
    const double2 x = v[u];
    return make_double2(diag * x.x + ar, diag * x.y + ai);
}



__device__ __forceinline__ void dot_acc(double x, double y, double2 &s) { s.x += x * y; }
__device__ __forceinline__ void dot_acc(double2 x, double2 y, double2 &s) {
    s.x += x.x * y.x + x.y * y.y;
    s.y += x.x * y.y - x.y * y.x;
}
__device__ __forceinline__ double2 wave_sum2(double2 v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        v.x += __shfl_down(v.x, off, 64);
        v.y += __shfl_down(v.y, off, 64);
    }
    return v;
}

// Sum over the workgroup, fixed order (waves in order), result in every thread.
__device__ __forceinline__ double2 block_sum_all(double2 v, double2 *red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    v = wave_sum2(v);
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double2 s = make_double2(0.0, 0.0);
    for (int q = 0; q < nw; ++q) {
        s.x += red[q].x;
        s.y += red[q].y;
    }
    return s;
}

// A whole Lanczos cycle of one small sector in one workgroup: H.v rows, alpha,
// the three-term update, classical Gram-Schmidt against every earlier vector
// (the second pass where the first cancelled more than half of |w|^2) and the
// normalisation, with the Krylov basis in global memory (it stays in L2 for
// the sizes this kernel is used for).  A single workgroup is bound by the
// latency of its loads from L2, so every pass keeps many independent loads in
// flight: the Gram-Schmidt dot products take VPI basis vectors per wavefront
// at a time (their loads issued together, their wavefront sums interleaved),
// and the update prefetches UC basis elements of a row before subtracting
// them in slot order.  CPLX: momentum sector (union layout), else fixed-N_down
// (ZM > 0: the unrolled all-hops-in-flight row of k_hv_u1).
template <int K, typename RT, bool CPLX, bool TABLE, int ZM>
__global__ __launch_bounds__(1024) void k_lanczos_small(SmallArgs S, BatchArgs A, const RT *__restrict__ binom_g) {
    using ET = typename std::conditional<CPLX, double2, double>::type;
    constexpr int VPI = CPLX ? 2 : 4;  // basis vectors per wavefront per round of the dot products
    constexpr int UC = CPLX ? 16 : 32; // basis elements prefetched per row in the update
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double2 red[16];
    __shared__ double2 hsh[520];
    const RT *tab;
    const int *ptr;
    const uint16_t *nbr;
    load_lds_tables<RT>(smem, A.L, binom_g, K, &tab, &ptr, &nbr);
    Binom<RT> Bn{tab, binom_shift(A.L.N)};
    Geom g{A.L.lx, A.L.ly, A.L.lz, A.L.lx * A.L.ly, A.L.coords, A.L.ns};
    const int tid = threadIdx.x, nt = blockDim.x;
    const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
    const uint64_t n = S.n;
    auto P = [&](int j) { return (ET *)(S.Psi + (size_t)j * S.stride); };
    ET *W = (ET *)S.W;
    for (int x = S.x0; x < S.x1; ++x) {
        const int prev = (x == S.x0) ? S.prev_first : x - 1;
        // ---- W = H psi_x
        if constexpr (CPLX) {
            const double2 *px = P(x);
            for (uint64_t r = tid; r < n; r += nt) W[r] = hv_row_k1<K, RT, TABLE>(A, Bn, g, ptr, nbr, r, px);
        } else {
            const double *px = P(x);
            for (uint64_t r = tid; r < n; r += nt) W[r] = hv_row_u1<K, RT, double, ZM>(A.L, Bn, ptr, nbr, (RT)r, px);
        }
        __syncthreads();
        // ---- alpha = Re <psi_x, W>; W -= alpha psi_x + beta_prev psi_prev
        double2 s = make_double2(0.0, 0.0);
        for (uint64_t r = tid; r < n; r += nt) dot_acc(P(x)[r], W[r], s);
        const double a = block_sum_all(s, red).x;
        const double bp = prev >= 0 ? S.ab[S.slots + prev] : 0.0;
        for (uint64_t r = tid; r < n; r += nt) {
            if constexpr (CPLX) {
                double2 w = W[r];
                const double2 p0 = P(x)[r];
                w.x -= a * p0.x;
                w.y -= a * p0.y;
                if (prev >= 0) {
                    const double2 p1 = P(prev)[r];
                    w.x -= bp * p1.x;
                    w.y -= bp * p1.y;
                }
                W[r] = w;
            } else {
                double w = W[r] - a * P(x)[r];
                if (prev >= 0) w -= bp * P(prev)[r];
                W[r] = w;
            }
        }
        if (tid == 0) S.ab[x] = a;
        __syncthreads();
        // ---- classical Gram-Schmidt against slots 0..x: one pass, and a
        // second where the first cancelled more than half of |W|^2.  Dot
        // products: wavefront q takes slots q, q + nw, ... VPI at a time (slot
        // x + 1 stands for W itself, giving |W|^2); each sum runs over rows
        // lane, lane + 64, ... and then a fixed shuffle tree.
        auto cgs_dots = [&](bool self) {
            const int jmax = x + (self ? 1 : 0);
            for (int j0 = wave; j0 <= jmax; j0 += nw * VPI) {
                double2 h[VPI];
#pragma unroll
                for (int c = 0; c < VPI; ++c) h[c] = make_double2(0.0, 0.0);
                for (uint64_t r = lane; r < n; r += 64) {
                    const ET w = W[r];
                    ET xv[VPI];
#pragma unroll
                    for (int c = 0; c < VPI; ++c) {
                        const int j = j0 + c * nw;
                        xv[c] = j <= x ? P(j)[r] : w;
                    }
#pragma unroll
                    for (int c = 0; c < VPI; ++c) dot_acc(xv[c], w, h[c]);
                }
#pragma unroll
                for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
                    for (int c = 0; c < VPI; ++c) {
                        h[c].x += __shfl_down(h[c].x, off, 64);
                        h[c].y += __shfl_down(h[c].y, off, 64);
                    }
                }
                if (lane == 0) {
#pragma unroll
                    for (int c = 0; c < VPI; ++c)
                        if (j0 + c * nw <= jmax) hsh[j0 + c * nw] = h[c];
                }
            }
            __syncthreads();
        };
        auto cgs_update = [&]() -> double {
            double2 acc = make_double2(0.0, 0.0);
            for (uint64_t r = tid; r < n; r += nt) {
                ET w = W[r];
                for (int j0 = 0; j0 <= x; j0 += UC) {
                    ET pv[UC];
#pragma unroll
                    for (int c = 0; c < UC; ++c)
                        if (j0 + c <= x) pv[c] = P(j0 + c)[r];
#pragma unroll
                    for (int c = 0; c < UC; ++c) {
                        if (j0 + c > x) break;
                        const double2 hc = hsh[j0 + c];
                        if constexpr (CPLX) {
                            w.x -= pv[c].x * hc.x - pv[c].y * hc.y;
                            w.y -= pv[c].x * hc.y + pv[c].y * hc.x;
                        } else {
                            w -= pv[c] * hc.x;
                        }
                    }
                }
                W[r] = w;
                if constexpr (CPLX) acc.x += w.x * w.x + w.y * w.y;
                else acc.x += w * w;
            }
            return block_sum_all(acc, red).x;
        };
        double nrm2;
        if (S.reorth > 0) {
            cgs_dots(true);
            const double before = hsh[x + 1].x;
            nrm2 = cgs_update();
            if (S.reorth > 1 && nrm2 < 0.5 * before) {
                __syncthreads();
                cgs_dots(false);
                nrm2 = cgs_update();
            }
        } else {
            double2 acc = make_double2(0.0, 0.0);
            for (uint64_t r = tid; r < n; r += nt) dot_acc(W[r], W[r], acc);
            nrm2 = block_sum_all(acc, red).x;
        }
        const double beta = sqrt(fmax(nrm2, 0.0));
        const double sc = beta > 0.0 ? 1.0 / beta : 0.0;
        for (uint64_t r = tid; r < n; r += nt) {
            if constexpr (CPLX) {
                const double2 w = W[r];
                P(x + 1)[r] = make_double2(w.x * sc, w.y * sc);
            } else {
                P(x + 1)[r] = W[r] * sc;
            }
        }
        if (tid == 0) S.ab[S.slots + x] = beta;
        __syncthreads();
    }
}

}  // namespace qs3
