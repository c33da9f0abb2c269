// Device kernels of the observables (Sec. 3.6, Sec. 4.2) and of S^-_q
// (Sec. 3.8), all as gathers with per-block partial sums (deterministic).
#pragma once
#include "hv_kernels.h"

namespace qs3 {

// Reduced-space site map: the e-th site (0-based) of {0..N-1} minus {lo, hi}
// (lo < hi; hi = -1 removes only lo).
__device__ __forceinline__ int skip_sites(int e, int lo, int hi) {
    int s = e + (e >= lo ? 1 : 0);
    if (hi >= 0) s += (s >= hi ? 1 : 0);
    return s;
}

template <int K, typename RT>
__device__ __forceinline__ RT rank_sorted(int (&t)[K > 0 ? K : 1], const Binom<RT> &Bn) {
    sortK<K>(t);
    RT r = 0;
#pragma unroll
    for (int m = 0; m < K; ++m) r += Bn.C(t[m], m + 1);
    return r;
}

__device__ __forceinline__ void block_sum2(double2 v, double2 *out) {
    __shared__ double2 red[256];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            red[threadIdx.x] = make_double2(red[threadIdx.x].x + red[threadIdx.x + s].x,
                                            red[threadIdx.x].y + red[threadIdx.x + s].y);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}

// <x_i> numerator: sum over states containing site i of |phi|^2 (fixed-N_down,
// real).  grid = (N, nchunk); subsets of K-1 sites of the other N-1.
template <int K, typename RT>
__global__ __launch_bounds__(256) void k_site_prob(LatArgs L, const RT *__restrict__ binom_g, uint64_t cnt,
                                                   int nchunk, const double *__restrict__ phi,
                                                   double2 *__restrict__ partial) {
    Binom<RT> Bn{binom_g, binom_shift(L.N)};
    const int i = blockIdx.x;
    const uint64_t per = (cnt + nchunk - 1) / nchunk;
    const uint64_t s0 = per * blockIdx.y, s1 = min(cnt, s0 + per);
    double acc = 0;
    for (uint64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
        int t[K > 0 ? K : 1];
        if (K >= 2) {
            int e[(K - 1) > 0 ? (K - 1) : 1];
            unrank<(K - 1 > 0 ? K - 1 : 0), RT>((RT)s, L.N - 1, Bn, e);
#pragma unroll
            for (int m = 0; m + 1 < K; ++m) t[m] = skip_sites(e[m], i, -1);
        }
        if (K >= 1) t[K - 1] = i;
        const double p = phi[rank_sorted<K, RT>(t, Bn)];
        acc += p * p;
    }
    block_sum2(make_double2(acc, 0.0), &partial[(size_t)blockIdx.x * nchunk + blockIdx.y]);
}

// Pair sums (fixed-N_down, real): q_ij = sum over states containing i and j of
// |phi|^2 (subsets of K-2 of the other N-2 sites) and
// pm_ij = sum_S phi(S + j) phi(S + i) (subsets S of K-1 of the other N-2).
// grid = (n_pairs, nchunk).
template <int K, typename RT>
__global__ __launch_bounds__(256) void k_pair_u1(LatArgs L, const RT *__restrict__ binom_g,
                                                 const int32_t *__restrict__ pi, const int32_t *__restrict__ pj,
                                                 uint64_t cnt_q, uint64_t cnt_pm, int nchunk,
                                                 const double *__restrict__ phi,
                                                 double2 *__restrict__ partial) {
    Binom<RT> Bn{binom_g, binom_shift(L.N)};
    const int p = blockIdx.x;
    const int i = pi[p], j = pj[p];
    const int lo = min(i, j), hi = max(i, j);
    double aq = 0, apm = 0;
    if (K >= 2) {
        const uint64_t per = (cnt_q + nchunk - 1) / nchunk;
        const uint64_t s0 = per * blockIdx.y, s1 = min(cnt_q, s0 + per);
        for (uint64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
            int t[K > 0 ? K : 1];
            if (K >= 3) {
                int e[(K - 2) > 0 ? (K - 2) : 1];
                unrank<(K - 2 > 0 ? K - 2 : 0), RT>((RT)s, L.N - 2, Bn, e);
#pragma unroll
                for (int m = 0; m + 2 < K; ++m) t[m] = skip_sites(e[m], lo, hi);
            }
            t[K - 2] = i;
            t[K - 1] = j;
            const double v = phi[rank_sorted<K, RT>(t, Bn)];
            aq += v * v;
        }
    }
    if (K >= 1) {
        const uint64_t per = (cnt_pm + nchunk - 1) / nchunk;
        const uint64_t s0 = per * blockIdx.y, s1 = min(cnt_pm, s0 + per);
        for (uint64_t s = s0 + threadIdx.x; s < s1; s += blockDim.x) {
            int ti[K > 0 ? K : 1], tj[K > 0 ? K : 1];
            if (K >= 2) {
                int e[(K - 1) > 0 ? (K - 1) : 1];
                unrank<(K - 1 > 0 ? K - 1 : 0), RT>((RT)s, L.N - 2, Bn, e);
#pragma unroll
                for (int m = 0; m + 1 < K; ++m) ti[m] = tj[m] = skip_sites(e[m], lo, hi);
            }
            ti[K - 1] = i;
            tj[K - 1] = j;
            apm += phi[rank_sorted<K, RT>(tj, Bn)] * phi[rank_sorted<K, RT>(ti, Bn)];
        }
    }
    block_sum2(make_double2(aq, apm), &partial[(size_t)blockIdx.x * nchunk + blockIdx.y]);
}

// One chunk of the Gram factor of <S^+_i S^-_j> (fixed N_down, real phi):
// for the (K-1)-subsets beta of ranks b0 .. b0 + nc - 1 and every site r,
// U[r * nc + (beta - b0)] = phi(beta + {r}) when r is not in beta, else 0.
// Then sum_beta U[beta][i] U[beta][j] = sum_S phi(S + i) phi(S + j) over the
// (K-1)-subsets S avoiding i and j, the pair sum of Sec. 3.6 for i != j.  With
// r inserted at position p of beta's sorted sites e, its rank is
// sum_{m<p} C(e_m, m+1) + C(r, p+1) + sum_{m>=p} C(e_m, m+2); the two sums
// move by one term each time r passes a site of beta.
template <int K, typename RT>
__global__ __launch_bounds__(256) void k_pm_rows(int N, const RT *__restrict__ binom_g, uint64_t b0, uint64_t nc,
                                                 const double *__restrict__ phi, double *__restrict__ U) {
    constexpr int M = K - 1;
    Binom<RT> Bn{binom_g, binom_shift(N)};
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nc) return;
    int e[M > 0 ? M : 1];
    RT low = 0, high = 0;
    RT cl[M > 0 ? M : 1], ch[M > 0 ? M : 1];
    if constexpr (M > 0) {
        unrank<M, RT>((RT)(b0 + t), N, Bn, e);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            cl[m] = Bn.C(e[m], m + 1);
            ch[m] = Bn.C(e[m], m + 2);
            high += ch[m];
        }
    }
    int p = 0;
    int nxt = M > 0 ? e[0] : N;
    for (int r = 0; r < N; ++r) {
        double v = 0.0;
        if (r == nxt) {
            // r is in beta: step past it
#pragma unroll
            for (int m = 0; m < M; ++m)
                if (m == p) {
                    low += cl[m];
                    high -= ch[m];
                }
            ++p;
            nxt = N;
#pragma unroll
            for (int m = 0; m < M; ++m)
                if (m == p) nxt = e[m];
        } else {
            v = phi[low + Bn.C(r, p + 1) + high];
        }
        U[(size_t)r * nc + t] = v;
    }
}

// Gram matrix of the factor above, split over row chunks: block (c, t) takes
// rows [c * rc, (c + 1) * rc) of U (nc x N, column major) and the 64 x 64 tile
// pair t = (ti <= tj) of G = U^T U on the matrix cores: 16-row panels of both
// column blocks are staged in LDS, and each of the four wavefronts forms one
// 32 x 32 quadrant as 2 x 2 blocks of v_mfma_f64_16x16x4 (A: lane l holds
// A[l % 16][l / 16], B: lane l holds B[l / 16][l % 16], D: element r of lane l
// is D[4 r + l / 16][l % 16]), four k-steps of 4 per panel.
// part[((c * ntp + t) * 64 + i) * 64 + j] = the chunk's sum for G[64 ti + i][64 tj + j].
template <int TS>
__global__ __launch_bounds__(256) void k_gram_tiles(const double *__restrict__ U, uint64_t nc, int N, uint64_t rc,
                                                    const int2 *__restrict__ tiles, int ntp,
                                                    double *__restrict__ part) {
    static_assert(TS == 64, "four wavefronts of 32 x 32 outputs per 64 x 64 tile");
    typedef double d4 __attribute__((ext_vector_type(4)));
    constexpr int LD = 64 + 4;  // padded panel rows
    __shared__ double As[16][LD], Bs[16][LD];
    const int2 tp = tiles[blockIdx.y];
    const int i0 = tp.x * 64, j0 = tp.y * 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wi = (wave >> 1) * 32, wj = (wave & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;
    const uint64_t r0 = (uint64_t)blockIdx.x * rc;
    const uint64_t r1 = r0 + rc < nc ? r0 + rc : nc;
    d4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
    for (uint64_t k0 = r0; k0 < r1; k0 += 16) {
        // 2 x 16 x 64 loads by 256 threads: k fastest, so 16 consecutive rows
        // of one column are contiguous
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int idx = threadIdx.x + q * 256;  // 0 .. 1023
            const int k = idx & 15, c = idx >> 4;   // c: 0 .. 63
            const uint64_t kr = k0 + k;
            const int ci = i0 + c, cj = j0 + c;
            As[k][c] = (kr < r1 && ci < N) ? U[(size_t)ci * nc + kr] : 0.0;
            Bs[k][c] = (kr < r1 && cj < N) ? U[(size_t)cj * nc + kr] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
            double a[2], b[2];
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                a[q] = As[kk + lk][wi + q * 16 + li];
                b[q] = Bs[kk + lk][wj + q * 16 + li];
            }
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[x], b[y], acc[x][y], 0, 0, 0);
        }
        __syncthreads();
    }
    double *out = part + ((size_t)blockIdx.x * ntp + blockIdx.y) * 4096;
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                out[(wi + x * 16 + 4 * r + lk) * 64 + wj + y * 16 + li] = acc[x][y][r];
}

// G[i + j N] (and G[j + i N]) = sum over the chunks, in chunk order, of the
// tile partials: one thread per element of every tile pair.
// First stage of the ordered sum over chunks: group g of gsz consecutive
// chunks, one thread per element of every tile pair, summed in chunk order
// into part2[(g * ntp + t) * 4096 + w] (the layout of the chunk partials).
template <int TS>
__global__ __launch_bounds__(256) void k_gram_group(const double *__restrict__ part, int nchunk, int ntp, int gsz,
                                                    double *__restrict__ part2) {
    static_assert(TS == 64, "64 x 64 tiles");
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (uint64_t)ntp * 4096) return;
    const int g = blockIdx.y;
    const int c0 = g * gsz, c1 = c0 + gsz < nchunk ? c0 + gsz : nchunk;
    double s = 0.0;
    for (int c = c0; c < c1; ++c) s += part[(size_t)c * ntp * 4096 + e];
    part2[(size_t)g * ntp * 4096 + e] = s;
}

template <int TS>
__global__ __launch_bounds__(256) void k_gram_reduce(const double *__restrict__ part, int nchunk,
                                                     const int2 *__restrict__ tiles, int ntp, int N,
                                                     double *__restrict__ G) {
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (uint64_t)ntp * 4096) return;
    const int t = (int)(e >> 12), w = (int)(e & 4095);
    const int i = tiles[t].x * 64 + (w >> 6), j = tiles[t].y * 64 + (w & 63);
    if (i >= N || j >= N) return;
    double s = 0.0;
    for (int c = 0; c < nchunk; ++c) s += part[((size_t)c * ntp + t) * 4096 + w];
    G[(size_t)i + (size_t)j * N] = s;
    G[(size_t)j + (size_t)i * N] = s;
}

// Momentum sector (union layout, one column): for the pair class disp[dd]
// (packed cell displacement d | s<<24 | t<<28: place s of a cell and place t
// of the cell d further on) accumulate over the rows of the chunk
//   zz: |phi_u|^2 * #{down spins at (r, s) whose partner (r + d, t) is down}
//   pm: conj(phi_u) * (O_d phi)_u with O_d = sum_r s^+_(r,s) s^-_(r+d,t); the pull
//       form applies O_d^+ (a down spin at place t of cell r moves to place s
//       of cell r - d) with the
//       momentum-basis element e^{ik.t} sqrt(s'/s_u)
//   nrm: |phi_u|^2
// grid = (n_disp, nchunk); partial[(dd * nchunk + chunk) * 2 + {0,1}].
template <int K, typename RT, bool TABLE>
__global__ __launch_bounds__(256) void k_corr_k(BatchArgs A, const RT *__restrict__ binom_g,
                                                const int32_t *__restrict__ disp, int nchunk,
                                                const double2 *__restrict__ phi,
                                                double2 *__restrict__ partial) {
    Binom<RT> Bn{binom_g, binom_shift(A.L.N)};
    Geom g{A.L.lx, A.L.ly, A.L.lz, A.L.lx * A.L.ly, A.L.coords, A.L.ns};
    const int dd = blockIdx.x;
    const int dp = disp[dd];
    const int dcell = dp & 0xffffff, ss = (dp >> 24) & 15, tt = (dp >> 28) & 15;
    const int dx = dcell % g.lx, dy = (dcell / g.lx) % g.ly, dz = dcell / g.lxy;
    const uint64_t per = (A.n_reps + nchunk - 1) / nchunk;
    const uint64_t u0 = per * blockIdx.y, u1 = min(A.n_reps, u0 + per);
    double azz = 0, anr = 0, apr = 0, api = 0;
    for (uint64_t u = u0 + threadIdx.x; u < u1; u += blockDim.x) {
        const int su = A.stab[u];
        if (su > 1 && !A.compat_nt[A.nt_of[u]]) continue;
        const double2 f = phi[u];
        const double f2 = f.x * f.x + f.y * f.y;
        const RT R = (RT)A.reps[u];
        int c[K > 0 ? K : 1];
        unrank<K, RT>(R, A.L.N, Bn, c);
        int tr[K > 0 ? K : 1], back[K > 0 ? K : 1];
#pragma unroll
        for (int m = 0; m < K; ++m) {
            const uint32_t pc = g.coords[c[m]];
            const int x = pc & 1023u, y = (pc >> 10) & 1023u, z = (pc >> 20) & 1023u, sm = (int)(pc >> 30);
            // partner of a down spin at place s of cell r: place t of cell r + d
            tr[m] = sm == ss ? tt + g.ns * (wrap_add(x, dx, g.lx) + g.lx * wrap_add(y, dy, g.ly) +
                                            g.lxy * wrap_add(z, dz, g.lz))
                             : -1;
            // O_d^+ moves a down spin at place t of cell r to place s of cell r - d
            back[m] = sm == tt ? ss + g.ns * (wrap_add(x, dx ? g.lx - dx : 0, g.lx) +
                                              g.lx * wrap_add(y, dy ? g.ly - dy : 0, g.ly) +
                                              g.lxy * wrap_add(z, dz ? g.lz - dz : 0, g.lz))
                               : -1;
        }
        int npair = 0;
#pragma unroll
        for (int m = 0; m < K; ++m)
#pragma unroll
            for (int q = 0; q < K; ++q) npair += (tr[m] == c[q]) ? 1 : 0;
        azz += f2 * (double)npair;
        anr += f2;
        HopRanker<K, RT> hr;
        hr.init(c, Bn);
        double sr = 0, si = 0;
        const double isq = 1.0 / A.L.sqrt_tab[su];
        StaticFor<0, K>::run([&](auto mc) {
            constexpr int m = decltype(mc)::value;
            RT rp;
            const int j = back[m];
            if (j < 0 || !hr.template hop<m>(c, R, j, Bn, &rp)) return;
            uint32_t u2;
            int tx, ty, tz;
            resolve_hop<K, RT, TABLE>(A, Bn, g, c, m, j, rp, &u2, &tx, &ty, &tz);
            const int s2 = A.stab[u2];
            if (s2 > 1 && !A.compat_nt[A.nt_of[u2]]) return;
            int P = A.kmul[0] * tx + A.kmul[1] * ty + A.kmul[2] * tz;
            P %= A.M;
            const double2 ph = A.phase[P];
            const double coef = A.L.sqrt_tab[s2] * isq;
            const double2 x = phi[u2];
            sr += coef * (ph.x * x.x - ph.y * x.y);
            si += coef * (ph.x * x.y + ph.y * x.x);
        });
        // conj(f) * (sr + i si)
        apr += f.x * sr + f.y * si;
        api += f.x * si - f.y * sr;
    }
    __shared__ double2 red[256][2];
    red[threadIdx.x][0] = make_double2(azz, anr);
    red[threadIdx.x][1] = make_double2(apr, api);
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int q = 0; q < 2; ++q)
                red[threadIdx.x][q] = make_double2(red[threadIdx.x][q].x + red[threadIdx.x + s][q].x,
                                                   red[threadIdx.x][q].y + red[threadIdx.x + s][q].y);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[((size_t)dd * nchunk + blockIdx.y) * 2] = red[0][0];
        partial[((size_t)dd * nchunk + blockIdx.y) * 2 + 1] = red[0][1];
    }
}

// S^-_q as a gather (Sec. 3.8, Alg. 11 read row by row).  Target rows are the
// representatives beta of the (K+1)-down structure, columns b the sectors
// k + q_b.  For every down spin r0 of beta, a' = beta minus r0 has the
// representative alpha = T^t a' in the K-down structure and contributes
//   e^{-i q_b.R_r0 + i k.t} sqrt(s_alpha / (N s_beta)) phi_alpha,
// the matrix element <beta, k+q | S^-_q | alpha, k> from the definition of the
// momentum states (Eq. (akstate)).
struct SmqArgs {
    BatchArgs src;    // K-down structure, source sector (B = 1)
    BatchArgs dst;    // (K+1)-down structure, target sectors (B = n_q)
    const int32_t *qmul;  // 3 * B: Q_a (M / L_a) mod M
    const double2 *subph;  // B * ns: e^{-i q_b . offset_s} of the places in a cell (1 for one site per cell)
};

template <int K, typename RTa, typename RTb, bool TABLE, int BPL>
__global__ __launch_bounds__(256) void k_smq(SmqArgs S, const RTa *__restrict__ binom_a,
                                             const RTb *__restrict__ binom_b,
                                             const double2 *__restrict__ phi,
                                             double2 *__restrict__ out) {
    constexpr int K1 = K + 1;
    const BatchArgs &A = S.src;
    const BatchArgs &D = S.dst;
    Binom<RTa> Ba{binom_a, binom_shift(A.L.N)};
    Binom<RTb> Bb{binom_b, binom_shift(A.L.N)};
    Geom g{A.L.lx, A.L.ly, A.L.lz, A.L.lx * A.L.ly, A.L.coords, A.L.ns};
    const int G = D.G, B = D.B;
    const int lane = threadIdx.x % G, slot = threadIdx.x / G;
    const int rows_per = blockDim.x / G;
    const uint64_t u = (uint64_t)blockIdx.x * rows_per + slot;
    if (u >= D.n_reps) return;
    const int sb = D.stab[u];
    const int ntb = sb > 1 ? D.nt_of[u] : -1;
    int c[K1];
    unrank<K1, RTb>((RTb)D.reps[u], A.L.N, Bb, c);
    double accr[BPL], acci[BPL];
#pragma unroll
    for (int i = 0; i < BPL; ++i) accr[i] = acci[i] = 0.0;
    const double isb = 1.0 / (A.L.sqrt_tab[sb] * sqrt((double)A.L.N));
#pragma unroll
    for (int m = 0; m < K1; ++m) {
        int a[K > 0 ? K : 1];
#pragma unroll
        for (int t = 0; t < K; ++t) a[t] = c[t < m ? t : t + 1];
        uint32_t ua;
        int tx, ty, tz;
        if (TABLE) {
            RTa r = 0;
#pragma unroll
            for (int t = 0; t < K; ++t) r += Ba.C(a[t], t + 1);
            const uint64_t ent = A.table[r];
            ua = (uint32_t)ent;
            const uint32_t tt = (uint32_t)(ent >> 32);
            tx = tt & 1023u;
            ty = (tt >> 10) & 1023u;
            tz = (tt >> 20) & 1023u;
        } else {
            int best[K > 0 ? K : 1];
            canonicalize<K>(a, g, best, tx, ty, tz);
            uint64_t r = 0;
#pragma unroll
            for (int t = 0; t < K; ++t) r += (uint64_t)Ba.C(best[t], t + 1);
            ua = (uint32_t)find_rep(A.reps, A.dir, A.dir_shift, r);
        }
        const int sa = A.stab[ua];
        if (sa > 1 && !A.compat_nt[A.nt_of[ua]]) continue;
        const double2 f = phi[ua];
        const double coef = A.L.sqrt_tab[sa] * isb;
        const uint32_t pr0 = g.coords[c[m]];
        const int x0 = pr0 & 1023u, y0 = (pr0 >> 10) & 1023u, z0 = (pr0 >> 20) & 1023u, s0 = (int)(pr0 >> 30);
        const int Pk = A.kmul[0] * tx + A.kmul[1] * ty + A.kmul[2] * tz;
#pragma unroll
        for (int i = 0; i < BPL; ++i) {
            const int b = lane + i * G;
            if (b >= B) continue;
            int P = Pk - (S.qmul[3 * b] * x0 + S.qmul[3 * b + 1] * y0 + S.qmul[3 * b + 2] * z0);
            P %= A.M;
            if (P < 0) P += A.M;
            const double2 pc = A.phase[P], so = S.subph[b * g.ns + s0];
            const double2 ph = make_double2(pc.x * so.x - pc.y * so.y, pc.x * so.y + pc.y * so.x);
            accr[i] += coef * (ph.x * f.x - ph.y * f.y);
            acci[i] += coef * (ph.x * f.y + ph.y * f.x);
        }
    }
#pragma unroll
    for (int i = 0; i < BPL; ++i) {
        const int b = lane + i * G;
        if (b >= B) continue;
        const bool ok = ntb < 0 || D.compat_nt[(size_t)ntb * B + b];
        out[u * B + b] = ok ? make_double2(accr[i], acci[i]) : make_double2(0.0, 0.0);
    }
}

// S^+_q as a gather (Sec. 3.8: the procedure of Alg. 11 for S^+).  Target
// rows are the representatives beta of the (K-1)-down structure, columns b
// the sectors k + q_b.  For every up site r0 of beta, a' = beta plus r0 has
// the representative alpha = T^t a' in the K-down structure and contributes
//   e^{-i q_b.R_r0 + i k.t} sqrt(s_alpha / (N s_beta)) phi_alpha.
template <int K, typename RTa, typename RTb, bool TABLE, int BPL>
__global__ __launch_bounds__(256) void k_spq(SmqArgs S, const RTa *__restrict__ binom_a,
                                             const RTb *__restrict__ binom_b,
                                             const double2 *__restrict__ phi,
                                             double2 *__restrict__ out) {
    constexpr int K1 = K - 1;
    const BatchArgs &A = S.src;
    const BatchArgs &D = S.dst;
    Binom<RTa> Ba{binom_a, binom_shift(A.L.N)};
    Binom<RTb> Bb{binom_b, binom_shift(A.L.N)};
    Geom g{A.L.lx, A.L.ly, A.L.lz, A.L.lx * A.L.ly, A.L.coords, A.L.ns};
    const int G = D.G, B = D.B;
    const int lane = threadIdx.x % G, slot = threadIdx.x / G;
    const int rows_per = blockDim.x / G;
    const uint64_t u = (uint64_t)blockIdx.x * rows_per + slot;
    if (u >= D.n_reps) return;
    const int sb = D.stab[u];
    const int ntb = sb > 1 ? D.nt_of[u] : -1;
    int c[K1 > 0 ? K1 : 1];
    if (K1 > 0) unrank<K1, RTb>((RTb)D.reps[u], A.L.N, Bb, c);
    double accr[BPL], acci[BPL];
#pragma unroll
    for (int i = 0; i < BPL; ++i) accr[i] = acci[i] = 0.0;
    const double isb = 1.0 / (A.L.sqrt_tab[sb] * sqrt((double)A.L.N));
    int m = 0;  // down spins of beta below r0
    for (int r0 = 0; r0 < A.L.N; ++r0) {
        if (m < K1 && c[m] == r0) {
            ++m;
            continue;
        }
        int a[K];
#pragma unroll
        for (int t = 0; t < K; ++t) a[t] = t < m ? c[t] : (t == m ? r0 : c[t > 0 ? t - 1 : 0]);
        uint32_t ua;
        int tx, ty, tz;
        if (TABLE) {
            RTa r = 0;
#pragma unroll
            for (int t = 0; t < K; ++t) r += Ba.C(a[t], t + 1);
            const uint64_t ent = A.table[r];
            ua = (uint32_t)ent;
            const uint32_t tt = (uint32_t)(ent >> 32);
            tx = tt & 1023u;
            ty = (tt >> 10) & 1023u;
            tz = (tt >> 20) & 1023u;
        } else {
            int best[K];
            canonicalize<K>(a, g, best, tx, ty, tz);
            uint64_t r = 0;
#pragma unroll
            for (int t = 0; t < K; ++t) r += (uint64_t)Ba.C(best[t], t + 1);
            ua = (uint32_t)find_rep(A.reps, A.dir, A.dir_shift, r);
        }
        const int sa = A.stab[ua];
        if (sa > 1 && !A.compat_nt[A.nt_of[ua]]) continue;
        const double2 f = phi[ua];
        const double coef = A.L.sqrt_tab[sa] * isb;
        const uint32_t pr0 = g.coords[r0];
        const int x0 = pr0 & 1023u, y0 = (pr0 >> 10) & 1023u, z0 = (pr0 >> 20) & 1023u, s0 = (int)(pr0 >> 30);
        const int Pk = A.kmul[0] * tx + A.kmul[1] * ty + A.kmul[2] * tz;
#pragma unroll
        for (int i = 0; i < BPL; ++i) {
            const int b = lane + i * G;
            if (b >= B) continue;
            int P = Pk - (S.qmul[3 * b] * x0 + S.qmul[3 * b + 1] * y0 + S.qmul[3 * b + 2] * z0);
            P %= A.M;
            if (P < 0) P += A.M;
            const double2 pc = A.phase[P], so = S.subph[b * g.ns + s0];
            const double2 ph = make_double2(pc.x * so.x - pc.y * so.y, pc.x * so.y + pc.y * so.x);
            accr[i] += coef * (ph.x * f.x - ph.y * f.y);
            acci[i] += coef * (ph.x * f.y + ph.y * f.x);
        }
    }
#pragma unroll
    for (int i = 0; i < BPL; ++i) {
        const int b = lane + i * G;
        if (b >= B) continue;
        const bool ok = ntb < 0 || D.compat_nt[(size_t)ntb * B + b];
        out[u * B + b] = ok ? make_double2(accr[i], acci[i]) : make_double2(0.0, 0.0);
    }
}

// S^z_q on a momentum sector (Sec. 3.8 for S^z): s^z_r leaves every state in
// place, so source (sector k) and target (k + q_b) share the representatives
// and the map is diagonal: row u of sector b is
//   phi_u N^{-1/2} (N/2 [q_b = 0] - sum_{r down in u} e^{-i q_b.R_r})
// on rows compatible with both sectors, 0 elsewhere.
template <int K, typename RT>
__global__ __launch_bounds__(256) void k_szq(SmqArgs S, const RT *__restrict__ binom,
                                             const double2 *__restrict__ phi,
                                             double2 *__restrict__ out) {
    const BatchArgs &A = S.src;
    const BatchArgs &D = S.dst;
    Binom<RT> Bn{binom, binom_shift(A.L.N)};
    const uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= D.n_reps * (uint64_t)D.B) return;
    const uint64_t u = e / (uint64_t)D.B;
    const int b = (int)(e - u * (uint64_t)D.B);
    const int su = D.stab[u];
    const bool ok = su == 1 || (A.compat_nt[A.nt_of[u]] && D.compat_nt[(size_t)D.nt_of[u] * D.B + b]);
    double2 o = make_double2(0.0, 0.0);
    if (ok) {
        int c[K > 0 ? K : 1];
        if (K > 0) unrank<K, RT>((RT)D.reps[u], A.L.N, Bn, c);
        const int qx = S.qmul[3 * b], qy = S.qmul[3 * b + 1], qz = S.qmul[3 * b + 2];
        double sr = (qx == 0 && qy == 0 && qz == 0) ? 0.5 * A.L.N : 0.0, si = 0.0;
#pragma unroll
        for (int m = 0; m < K; ++m) {
            const uint32_t p = A.L.coords[c[m]];
            int P = qx * (int)(p & 1023u) + qy * (int)((p >> 10) & 1023u) + qz * (int)((p >> 20) & 1023u);
            P %= A.M;
            // e^{-i q.R} = conj(e^{+i q.x_cell}) * e^{-i q.offset}, subtracted
            const double2 pc = A.phase[P], so = S.subph[b * A.L.ns + (int)(p >> 30)];
            sr -= pc.x * so.x + pc.y * so.y;
            si -= pc.x * so.y - pc.y * so.x;
        }
        const double inv = 1.0 / sqrt((double)A.L.N);
        const double2 f = phi[u];
        o = make_double2(inv * (sr * f.x - si * f.y), inv * (sr * f.y + si * f.x));
    }
    out[e] = o;
}

}  // namespace qs3
