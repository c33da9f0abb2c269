/*
 * Plain CPU oracle for the QS^3 hot path (arXiv 2107.00872), for the sizes the
 * Python oracle cannot reach.  TEST INFRASTRUCTURE: only the tests, the smoke
 * check and the benchmark's CPU-baseline leg load this library.  It shares no
 * code with the HIP library.
 *
 * Everything is in the paper's 1-based notation: ranks a = 1..C(N,K), states
 * are ascending down-spin tuples n[1..K] of sites 1..N.  Each routine computes
 * what the paper defines, written from the definition:
 *
 *   rank      a = 1 + sum_m C(n_m - 1, m)                          Eq. (a_of_n)
 *   unrank    the tuple whose rank is a: a - 1 written in the combinatorial
 *             number system, digits found from the largest binomial down
 *             (Sec. 3.1); this also covers the ranks the printed search range
 *             of Alg. 1 cannot return
 *   hop       the exchange term of a bond with one end down moves that down
 *             spin to the other end: drop it, insert the other site, keep the
 *             tuple ascending (Sec. 3.2)
 *   orbit     T^t moves every down spin by the lattice vector t; the
 *             representative of a state is the minimum rank over its orbit and
 *             l the first translation number reaching it (Sec. 3.3)
 *   N_{a,k}   the squared norm of Eq. (akstate)'s sum: N sum_{t in stab(a)}
 *             e^{ik.t}, i.e. N |stab(a)| when e^{ik.t} = 1 on the stabiliser,
 *             else 0; nonzero only for the orbit minimum (Sec. 3.3)
 *
 * and follows the steps of the method in the paper's order: the H.v of Alg. 9
 * takes one row at a time and runs over every bond of the model for it (the
 * Ising term +-Jz/4, and Jxy/2 times the exchanged state's amplitude), finds
 * the exchanged state's representative by searching all N translations and
 * its position in sigma by a binary search; S^-_q scatters over sites and
 * rows as Sec. 3.8 does.  OpenMP runs over rows.
 *
 * The cached-structure variant (orc_kstruct_*) resolves each hop of each
 * orbit representative once -- target representative and translation, by
 * the same all-translation search -- and reuses that list for every momentum
 * and every Lanczos step; row sums are formed in the same bond order.
 *
 * Readings applied (the same as the Python oracle):
 *  - the k-basis element is (Jxy/2) e^{+ik.t_l} R_{a'}/R_a with R = sqrt(N_{a,k})
 *    (Alg. 8/9 print sqrt(R'/R)); S^-_q uses R'_b/(R_a sqrt N) (Alg. 11 prints
 *    sqrt(R'/(R N)));
 *  - N_{a,k} is tested against 1e-8 rather than 0;
 *  - site r has coordinates r-1 = x + Lx(y + Ly z); translation j = 1..N is the
 *    vector coords(j mod N), so j = N is the identity; any translation reaching
 *    the minimum gives the same phase for a compatible k.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXK 32
#define MAXN 4096

typedef struct {
    int N, K, lx, ly, lz;
    uint64_t *binom; /* binom[k*(K+2) + m] = C(k, m), k = 0..N, m = 0..K+1 */
} geo_t;

static uint64_t Cb(const geo_t *g, int k, int m) {
    if (m < 0 || k < m || k < 0) return 0;
    return g->binom[(size_t)k * (g->K + 2) + m];
}

/* Pascal's rule C(k, m) = C(k-1, m-1) + C(k-1, m) */
static int geo_init(geo_t *g, int lx, int ly, int lz, int K) {
    g->lx = lx; g->ly = ly; g->lz = lz; g->N = lx * ly * lz; g->K = K;
    if (g->N > MAXN || K + 1 > MAXK || K < 0) return -1;
    g->binom = (uint64_t *)calloc((size_t)(g->N + 1) * (K + 2), sizeof(uint64_t));
    for (int k = 0; k <= g->N; ++k) {
        for (int m = 0; m <= K + 1; ++m) {
            uint64_t v;
            if (m == 0) v = 1;
            else if (k < m) v = 0;
            else v = g->binom[(size_t)(k - 1) * (K + 2) + m - 1] + g->binom[(size_t)(k - 1) * (K + 2) + m];
            g->binom[(size_t)k * (K + 2) + m] = v;
        }
    }
    return 0;
}

static void geo_free(geo_t *g) { free(g->binom); }

/* Eq. (a_of_n) */
static uint64_t rank_of(const geo_t *g, const int *n, int K) {
    uint64_t a = 1;
    for (int m = 1; m <= K; ++m) a += Cb(g, n[m] - 1, m);
    return a;
}

/* The tuple with rank a.  a - 1 = sum_m C(n_m - 1, m) with n_1 < ... < n_K
 * is unique; from m = K down, n_m - 1 is the largest c below the digit above
 * with C(c, m) <= the remainder (found by bisection on the increasing column
 * C(., m), which is 0 at c = m - 1). */
static void unrank(const geo_t *g, uint64_t a, int K, int *n) {
    uint64_t s = a - 1;
    int top = g->N - 1; /* n_m - 1 <= top */
    for (int m = K; m >= 1; --m) {
        int lo = m - 1, hi = top;
        while (lo < hi) {
            int mid = (lo + hi + 1) / 2;
            if (Cb(g, mid, m) <= s) lo = mid; else hi = mid - 1;
        }
        n[m] = lo + 1;
        s -= Cb(g, lo, m);
        top = lo - 1;
    }
}

static int is_down(const int *n, int K, int r) {
    for (int i = 1; i <= K; ++i)
        if (n[i] == r) return 1;
    return 0;
}

static void sort_tuple(int *n, int K) {
    for (int i = 2; i <= K; ++i) {
        int v = n[i], j = i - 1;
        while (j >= 1 && n[j] > v) { n[j + 1] = n[j]; --j; }
        n[j + 1] = v;
    }
}

/* the down spin at site `from` moves to the empty site `to` */
static void move_spin(const int *n, int K, int from, int to, int *out) {
    int o = 1;
    for (int i = 1; i <= K; ++i)
        if (n[i] != from) out[o++] = n[i];
    out[o] = to;
    sort_tuple(out, K);
}

static void coords(const geo_t *g, int r, int *x, int *y, int *z) {
    int i = r - 1;
    *x = i % g->lx; *y = (i / g->lx) % g->ly; *z = i / (g->lx * g->ly);
}

/* the vector of translation number j = 1..N (j = N: the identity) */
static void tvec(const geo_t *g, int j, int *t) {
    coords(g, (j % g->N) + 1, &t[0], &t[1], &t[2]);
}

static double kdot(const geo_t *g, const int *Kv, const int *t) {
    return 2.0 * M_PI * ((double)Kv[0] * t[0] / g->lx + (double)Kv[1] * t[1] / g->ly +
                         (double)Kv[2] * t[2] / g->lz);
}

/* T^t n: every down spin moved by t (periodic), as an ascending tuple */
static void translate(const geo_t *g, const int *n, int K, const int *t, int *out) {
    for (int m = 1; m <= K; ++m) {
        int x, y, z;
        coords(g, n[m], &x, &y, &z);
        x = (x + t[0]) % g->lx; y = (y + t[1]) % g->ly; z = (z + t[2]) % g->lz;
        out[m] = 1 + x + g->lx * (y + g->ly * z);
    }
    sort_tuple(out, K);
}

/* minimum rank over the orbit of n and the first translation number reaching it */
static uint64_t canonical(const geo_t *g, const int *n, int K, int *ell) {
    int n2[MAXK + 1], t[3];
    uint64_t best = 0;
    for (int j = 1; j <= g->N; ++j) {
        tvec(g, j, t);
        translate(g, n, K, t, n2);
        uint64_t a = rank_of(g, n2, K);
        if (j == 1 || a < best) { best = a; *ell = j; }
    }
    return best;
}

/* N_{a,k}; 0 unless a is the minimum rank of its orbit */
static double orbit_norm(const geo_t *g, uint64_t a, int K, const int *Kv) {
    int n[MAXK + 1], n2[MAXK + 1], t[3];
    unrank(g, a, K, n);
    double s = 0.0;
    for (int j = 1; j <= g->N; ++j) {
        tvec(g, j, t);
        translate(g, n, K, t, n2);
        uint64_t a2 = rank_of(g, n2, K);
        if (a2 < a) return 0.0;
        if (a2 == a) s += cos(kdot(g, Kv, t));
    }
    double Nak = s * g->N;
    return Nak > 1e-8 ? Nak : 0.0;
}

/* position (1-based) of x in the ascending sigma[0..d-1], or 0 if absent */
static int64_t find_sorted(const uint64_t *sigma, int64_t d, uint64_t x) {
    int64_t lo = 0, hi = d;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (sigma[mid] < x) lo = mid + 1; else hi = mid;
    }
    return (lo < d && sigma[lo] == x) ? lo + 1 : 0;
}

/* ---------------------------------------------------------------- exports */

uint64_t orc_binom(int n, int k) {
    if (k < 0 || n < k) return 0;
    uint64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (uint64_t)(n - k + i) / (uint64_t)i;
    return r;
}

/* rank / unrank in the paper's 1-based form, for a batch of states */
int orc_f_bar(int N, int K, int64_t count, const uint64_t *a, int32_t *n_out) {
    geo_t g;
    if (geo_init(&g, N, 1, 1, K)) return -1;
    int n[MAXK + 1];
    for (int64_t i = 0; i < count; ++i) {
        unrank(&g, a[i], K, n);
        for (int m = 1; m <= K; ++m) n_out[i * K + m - 1] = n[m];
    }
    geo_free(&g);
    return 0;
}

int orc_F(int N, int K, int64_t count, const int32_t *n_in, uint64_t *a_out) {
    geo_t g;
    if (geo_init(&g, N, 1, 1, K)) return -1;
    int n[MAXK + 1];
    for (int64_t i = 0; i < count; ++i) {
        for (int m = 1; m <= K; ++m) n[m] = n_in[i * K + m - 1];
        a_out[i] = rank_of(&g, n, K);
    }
    geo_free(&g);
    return 0;
}

/* Alg. 9 with sigma = every rank (U(1) only).  Rows are given 1-based in `rows`
 * (count nrows), or all rows when rows == NULL.  Bonds are 1-based (r < r').
 * phi, psi real; psi[i] is the result for rows[i] (or row i+1). */
int orc_hv_u1(int N, int K, int nb, const int32_t *br, const int32_t *brp, const double *jxy,
              const double *jz, const uint64_t *rows, int64_t nrows, const double *phi,
              double *psi, int nthreads) {
    geo_t g;
    if (geo_init(&g, N, 1, 1, K)) return -1;
    int64_t total = rows ? nrows : (int64_t)Cb(&g, N, K);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < total; ++i) {
        uint64_t a = rows ? rows[i] : (uint64_t)(i + 1);
        int n[MAXK + 1], n2[MAXK + 1];
        unrank(&g, a, K, n);
        double acc = 0.0;
        for (int b = 0; b < nb; ++b) {
            int dr = is_down(n, K, br[b]), drp = is_down(n, K, brp[b]);
            if (dr == drp) {
                acc += jz[b] / 4.0 * phi[a - 1];
            } else {
                acc -= jz[b] / 4.0 * phi[a - 1];
                if (dr) move_spin(n, K, br[b], brp[b], n2);
                else move_spin(n, K, brp[b], br[b], n2);
                acc += jxy[b] / 2.0 * phi[rank_of(&g, n2, K) - 1];
            }
        }
        psi[i] = acc;
    }
    geo_free(&g);
    return 0;
}

/* One U(1) row in bond order: cols (0-based ranks) and values; returns the
 * number of off-diagonal entries, the diagonal in *diag. */
int orc_row_u1(int N, int K, int nb, const int32_t *br, const int32_t *brp, const double *jxy,
               const double *jz, uint64_t a, double *diag, uint64_t *cols, double *vals) {
    geo_t g;
    if (geo_init(&g, N, 1, 1, K)) return -1;
    int n[MAXK + 1], n2[MAXK + 1], cnt = 0;
    unrank(&g, a, K, n);
    double dg = 0.0;
    for (int b = 0; b < nb; ++b) {
        int dr = is_down(n, K, br[b]), drp = is_down(n, K, brp[b]);
        if (dr == drp) {
            dg += jz[b] / 4.0;
        } else {
            dg -= jz[b] / 4.0;
            if (dr) move_spin(n, K, br[b], brp[b], n2);
            else move_spin(n, K, brp[b], br[b], n2);
            cols[cnt] = rank_of(&g, n2, K) - 1;
            vals[cnt] = jxy[b] / 2.0;
            ++cnt;
        }
    }
    *diag = dg;
    geo_free(&g);
    return cnt;
}

/* sigma (ascending representatives with N_{a,k} > 0) and R = sqrt(N_{a,k}),
 * over every rank, parallel over contiguous rank ranges.  First call with
 * sigma == NULL for d, then with buffers of that size. */
int64_t orc_mk_list(int lx, int ly, int lz, int K, const int32_t *Kv, uint64_t *sigma, double *R,
                    int nthreads) {
    geo_t g;
    if (geo_init(&g, lx, ly, lz, K)) return -1;
    uint64_t D = Cb(&g, g.N, K);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    int64_t *cnt = (int64_t *)calloc((size_t)nt + 1, sizeof(int64_t));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        uint64_t lo = D * (uint64_t)tid / nt + 1, hi = D * (uint64_t)(tid + 1) / nt;
        int64_t c = 0;
        for (uint64_t a = lo; a <= hi; ++a)
            if (orbit_norm(&g, a, K, Kv) > 0) ++c;
        cnt[tid + 1] = c;
    }
    for (int t = 0; t < nt; ++t) cnt[t + 1] += cnt[t];
    int64_t d = cnt[nt];
    if (sigma) {
#pragma omp parallel
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            uint64_t lo = D * (uint64_t)tid / nt + 1, hi = D * (uint64_t)(tid + 1) / nt;
            int64_t o = cnt[tid];
            for (uint64_t a = lo; a <= hi; ++a) {
                double Nak = orbit_norm(&g, a, K, Kv);
                if (Nak > 0) { sigma[o] = a; R[o] = sqrt(Nak); ++o; }
            }
        }
    }
    free(cnt);
    geo_free(&g);
    return d;
}

/* orbit representative and translation number for a batch of ranks */
int orc_representative(int lx, int ly, int lz, int K, int64_t count, const uint64_t *a,
                       uint64_t *rep, int32_t *ell) {
    geo_t g;
    if (geo_init(&g, lx, ly, lz, K)) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
        int n[MAXK + 1], l = 0;
        unrank(&g, a[i], K, n);
        rep[i] = canonical(&g, n, K, &l);
        ell[i] = l;
    }
    geo_free(&g);
    return 0;
}

/* The terms of k-block row al (1-based) in bond order: diagonal, and for each
 * exchanged bond whose target's representative is in sigma, its 1-based
 * position and the element (Jxy/2) e^{ik.t_l} R_b / R_a.  Returns the count. */
static int row_k_terms(const geo_t *g, const int *Kv, int nb, const int32_t *br, const int32_t *brp,
                       const double *jxy, const double *jz, const uint64_t *sigma, const double *R,
                       int64_t d, int64_t al, double *diag, int64_t *cols, double *vr, double *vi) {
    int n[MAXK + 1], n2[MAXK + 1], t[3], cnt = 0, K = g->K;
    unrank(g, sigma[al - 1], K, n);
    double dg = 0.0;
    for (int b = 0; b < nb; ++b) {
        int dr = is_down(n, K, br[b]), drp = is_down(n, K, brp[b]);
        if (dr == drp) {
            dg += jz[b] / 4.0;
            continue;
        }
        dg -= jz[b] / 4.0;
        if (dr) move_spin(n, K, br[b], brp[b], n2);
        else move_spin(n, K, brp[b], br[b], n2);
        int ell = 0;
        uint64_t rep = canonical(g, n2, K, &ell);
        int64_t ap = find_sorted(sigma, d, rep);
        if (!ap) continue;
        tvec(g, ell, t);
        double ph = kdot(g, Kv, t);
        double c = jxy[b] / 2.0 * R[ap - 1] / R[al - 1];
        cols[cnt] = ap;
        vr[cnt] = c * cos(ph);
        vi[cnt] = c * sin(ph);
        ++cnt;
    }
    *diag = dg;
    return cnt;
}

/* Alg. 9 in the k basis.  phi, psi complex (interleaved re, im).  Rows are
 * 1-based indices into sigma (or all when rows == NULL). */
int orc_hv_k(int lx, int ly, int lz, int K, const int32_t *Kv, int nb, const int32_t *br,
             const int32_t *brp, const double *jxy, const double *jz, const uint64_t *sigma,
             const double *R, int64_t d, const int64_t *rows, int64_t nrows, const double *phi,
             double *psi, int nthreads) {
    geo_t g;
    if (geo_init(&g, lx, ly, lz, K)) return -1;
    int64_t total = rows ? nrows : d;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        int64_t *cols = (int64_t *)malloc(sizeof(int64_t) * (nb + 1));
        double *vr = (double *)malloc(sizeof(double) * (nb + 1));
        double *vi = (double *)malloc(sizeof(double) * (nb + 1));
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < total; ++i) {
            int64_t al = rows ? rows[i] : i + 1;
            double dg;
            int cnt = row_k_terms(&g, Kv, nb, br, brp, jxy, jz, sigma, R, d, al, &dg, cols, vr, vi);
            double ar = dg * phi[2 * (al - 1)], ai = dg * phi[2 * (al - 1) + 1];
            for (int h = 0; h < cnt; ++h) {
                double xr = phi[2 * (cols[h] - 1)], xi = phi[2 * (cols[h] - 1) + 1];
                ar += vr[h] * xr - vi[h] * xi;
                ai += vr[h] * xi + vi[h] * xr;
            }
            psi[2 * i] = ar;
            psi[2 * i + 1] = ai;
        }
        free(cols); free(vr); free(vi);
    }
    geo_free(&g);
    return 0;
}

/* Row al (1-based) of the k block in bond order: cols (0-based sigma
 * indices), complex vals interleaved; returns count, diag in *diag. */
int orc_row_k(int lx, int ly, int lz, int K, const int32_t *Kv, int nb, const int32_t *br,
              const int32_t *brp, const double *jxy, const double *jz, const uint64_t *sigma,
              const double *R, int64_t d, int64_t al, double *diag, int64_t *cols, double *vals) {
    geo_t g;
    if (geo_init(&g, lx, ly, lz, K)) return -1;
    int64_t *c1 = (int64_t *)malloc(sizeof(int64_t) * (nb + 1));
    double *vr = (double *)malloc(sizeof(double) * (nb + 1));
    double *vi = (double *)malloc(sizeof(double) * (nb + 1));
    int cnt = row_k_terms(&g, Kv, nb, br, brp, jxy, jz, sigma, R, d, al, diag, c1, vr, vi);
    for (int h = 0; h < cnt; ++h) {
        cols[h] = c1[h] - 1;
        vals[2 * h] = vr[h];
        vals[2 * h + 1] = vi[h];
    }
    free(c1); free(vr); free(vi);
    geo_free(&g);
    return cnt;
}

/* psi1 = S^-_q phi (Sec. 3.8): every site r that is up in a representative
 * sigma_al gets a down spin; the resulting state lands on its representative
 * b (if in sigma1) with (R1_b / (R_al sqrt N)) e^{-i(q.R_r + (k+q).t_l)}.
 * Scattered over r and al (per-thread buffers, summed in thread order). */
int orc_smq(int lx, int ly, int lz, int K, const int32_t *Kv, const uint64_t *sigma,
            const double *R, int64_t d, const double *phi, const uint64_t *sigma1,
            const double *R1, int64_t d1, const int32_t *Qv, double *psi1, int nthreads) {
    geo_t g, g1;
    if (geo_init(&g, lx, ly, lz, K)) return -1;
    if (geo_init(&g1, lx, ly, lz, K + 1)) { geo_free(&g); return -1; }
    int kq[3] = {Kv[0] + Qv[0], Kv[1] + Qv[1], Kv[2] + Qv[2]};
    double sqN = sqrt((double)g.N);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    double *buf = (double *)calloc((size_t)nt * 2 * d1, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *out = buf + (size_t)tid * 2 * d1;
#pragma omp for schedule(static)
        for (int r = 1; r <= g.N; ++r) {
            int Rr[3], t[3];
            coords(&g, r, &Rr[0], &Rr[1], &Rr[2]);
            for (int64_t al = 1; al <= d; ++al) {
                int n[MAXK + 2], n2[MAXK + 2];
                unrank(&g, sigma[al - 1], K, n);
                if (is_down(n, K, r)) continue;
                for (int m = 1; m <= K; ++m) n2[m] = n[m];
                n2[K + 1] = r;
                sort_tuple(n2, K + 1);
                int ell = 0;
                uint64_t rep = canonical(&g1, n2, K + 1, &ell);
                int64_t bi = find_sorted(sigma1, d1, rep);
                if (!bi) continue;
                tvec(&g, ell, t);
                double ph = -(kdot(&g, Qv, Rr) + kdot(&g, kq, t));
                double c = R1[bi - 1] / (R[al - 1] * sqN);
                double cr = c * cos(ph), ci = c * sin(ph);
                double vr = phi[2 * (al - 1)], vi = phi[2 * (al - 1) + 1];
                out[2 * (bi - 1)] += cr * vr - ci * vi;
                out[2 * (bi - 1) + 1] += cr * vi + ci * vr;
            }
        }
    }
    memset(psi1, 0, sizeof(double) * 2 * d1);
    for (int t = 0; t < nt; ++t)
        for (int64_t i = 0; i < 2 * d1; ++i) psi1[i] += buf[(size_t)t * 2 * d1 + i];
    free(buf);
    geo_free(&g);
    geo_free(&g1);
    return 0;
}

/* ------------------------------------------------ cached-structure variant
 * The orbit representatives of every momentum at once (every orbit minimum),
 * each with its stabiliser and its row's hops resolved once: for every bond
 * with one end down, in bond order, the representative of the exchanged state
 * (its position among all representatives) and the translation number
 * reaching it, found by the all-translation search above.  A momentum k then
 * selects the representatives with N_{a,k} > 0, and H.v in that sector reuses
 * the resolved hops with the phases e^{ik.t_l}. */
typedef struct {
    geo_t g;
    int64_t nrep;
    uint64_t *rep;   /* ascending */
    int64_t *soff;   /* stabiliser translations of rep u: stab[soff[u] .. soff[u+1]) */
    int32_t *stab;
    double *diag;    /* Ising diagonal of rep u's row */
    int64_t *hoff;   /* hops of rep u: [hoff[u], hoff[u+1]) */
    int64_t *hcol;   /* position of the target's representative */
    int32_t *hell;   /* translation number reaching it */
    double *hval;    /* Jxy/2 of the bond */
} kstruct_t;

void orc_kstruct_free(void *p) {
    kstruct_t *s = (kstruct_t *)p;
    if (!s) return;
    free(s->rep); free(s->soff); free(s->stab); free(s->diag);
    free(s->hoff); free(s->hcol); free(s->hell); free(s->hval);
    geo_free(&s->g);
    free(s);
}

static int is_orbit_min(const geo_t *g, uint64_t a, int K) {
    int n[MAXK + 1], n2[MAXK + 1], t[3];
    unrank(g, a, K, n);
    for (int j = 1; j <= g->N; ++j) {
        tvec(g, j, t);
        translate(g, n, K, t, n2);
        if (rank_of(g, n2, K) < a) return 0;
    }
    return 1;
}

void *orc_kstruct_build(int lx, int ly, int lz, int K, int nb, const int32_t *br, const int32_t *brp,
                        const double *jxy, const double *jz, int nthreads) {
    kstruct_t *s = (kstruct_t *)calloc(1, sizeof(kstruct_t));
    if (!s || geo_init(&s->g, lx, ly, lz, K)) { free(s); return NULL; }
    const geo_t *g = &s->g;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    const uint64_t D = Cb(g, g->N, K);
    /* orbit minima, in rank order: count per contiguous range, then write */
    int64_t *cnt = (int64_t *)calloc((size_t)nt + 1, sizeof(int64_t));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        uint64_t lo = D * (uint64_t)tid / nt + 1, hi = D * (uint64_t)(tid + 1) / nt;
        int64_t c = 0;
        for (uint64_t a = lo; a <= hi; ++a) c += is_orbit_min(g, a, K);
        cnt[tid + 1] = c;
    }
    for (int t = 0; t < nt; ++t) cnt[t + 1] += cnt[t];
    s->nrep = cnt[nt];
    s->rep = (uint64_t *)malloc(sizeof(uint64_t) * (s->nrep + 1));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        uint64_t lo = D * (uint64_t)tid / nt + 1, hi = D * (uint64_t)(tid + 1) / nt;
        int64_t o = cnt[tid];
        for (uint64_t a = lo; a <= hi; ++a)
            if (is_orbit_min(g, a, K)) s->rep[o++] = a;
    }
    free(cnt);
    const int64_t R_ = s->nrep;
    /* stabilisers and hop counts */
    int32_t *ns = (int32_t *)calloc((size_t)R_ + 1, sizeof(int32_t));
    int32_t *nh = (int32_t *)calloc((size_t)R_ + 1, sizeof(int32_t));
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t u = 0; u < R_; ++u) {
        int n[MAXK + 1], n2[MAXK + 1], t[3];
        unrank(g, s->rep[u], K, n);
        for (int j = 1; j <= g->N; ++j) {
            tvec(g, j, t);
            translate(g, n, K, t, n2);
            if (rank_of(g, n2, K) == s->rep[u]) ns[u]++;
        }
        for (int b = 0; b < nb; ++b)
            if (is_down(n, K, br[b]) != is_down(n, K, brp[b])) nh[u]++;
    }
    s->soff = (int64_t *)malloc(sizeof(int64_t) * (R_ + 1));
    s->hoff = (int64_t *)malloc(sizeof(int64_t) * (R_ + 1));
    s->soff[0] = s->hoff[0] = 0;
    for (int64_t u = 0; u < R_; ++u) {
        s->soff[u + 1] = s->soff[u] + ns[u];
        s->hoff[u + 1] = s->hoff[u] + nh[u];
    }
    free(ns); free(nh);
    s->stab = (int32_t *)malloc(sizeof(int32_t) * (s->soff[R_] + 1));
    s->diag = (double *)malloc(sizeof(double) * (R_ + 1));
    s->hcol = (int64_t *)malloc(sizeof(int64_t) * (s->hoff[R_] + 1));
    s->hell = (int32_t *)malloc(sizeof(int32_t) * (s->hoff[R_] + 1));
    s->hval = (double *)malloc(sizeof(double) * (s->hoff[R_] + 1));
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
    for (int64_t u = 0; u < R_; ++u) {
        int n[MAXK + 1], n2[MAXK + 1], t[3];
        unrank(g, s->rep[u], K, n);
        int64_t o = s->soff[u];
        for (int j = 1; j <= g->N; ++j) {
            tvec(g, j, t);
            translate(g, n, K, t, n2);
            if (rank_of(g, n2, K) == s->rep[u]) s->stab[o++] = j;
        }
        double dg = 0.0;
        int64_t h = s->hoff[u];
        for (int b = 0; b < nb; ++b) {
            int dr = is_down(n, K, br[b]), drp = is_down(n, K, brp[b]);
            if (dr == drp) {
                dg += jz[b] / 4.0;
                continue;
            }
            dg -= jz[b] / 4.0;
            if (dr) move_spin(n, K, br[b], brp[b], n2);
            else move_spin(n, K, brp[b], br[b], n2);
            int ell = 0;
            uint64_t rep = canonical(g, n2, K, &ell);
            int64_t c = find_sorted(s->rep, R_, rep);
            bad |= (c == 0);
            s->hcol[h] = c - 1;
            s->hell[h] = ell;
            s->hval[h] = jxy[b] / 2.0;
            ++h;
        }
        s->diag[u] = dg;
    }
    if (bad) { orc_kstruct_free(s); return NULL; }
    return s;
}

int64_t orc_kstruct_nrep(void *p) { return ((kstruct_t *)p)->nrep; }
int64_t orc_kstruct_nhops(void *p) { kstruct_t *s = (kstruct_t *)p; return s->hoff[s->nrep]; }

/* the sector of momentum Kv: positions (0-based, ascending) of the
 * representatives with N_{a,k} > 0, their ranks and R = sqrt(N_{a,k}).
 * NULL outputs: count only. */
int64_t orc_kstruct_sector(void *p, const int32_t *Kv, int64_t *members, uint64_t *sigma, double *R) {
    kstruct_t *s = (kstruct_t *)p;
    const geo_t *g = &s->g;
    int64_t d = 0;
    for (int64_t u = 0; u < s->nrep; ++u) {
        double sum = 0.0;
        int t[3];
        for (int64_t o = s->soff[u]; o < s->soff[u + 1]; ++o) {
            tvec(g, s->stab[o], t);
            sum += cos(kdot(g, Kv, t));
        }
        double Nak = sum * g->N;
        if (!(Nak > 1e-8)) continue;
        if (members) members[d] = u;
        if (sigma) sigma[d] = s->rep[u];
        if (R) R[d] = sqrt(Nak);
        ++d;
    }
    return d;
}

/* psi = H phi in the sector (members, R from orc_kstruct_sector), complex
 * interleaved, rows in sector order; each row's terms in bond order. */
int orc_kstruct_hv(void *p, const int32_t *Kv, const int64_t *members, const double *R, int64_t d,
                   const double *phi, double *psi, int nthreads) {
    kstruct_t *s = (kstruct_t *)p;
    const geo_t *g = &s->g;
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (s->nrep + 1));
    if (!pos) return -1;
    for (int64_t u = 0; u < s->nrep; ++u) pos[u] = -1;
    for (int64_t i = 0; i < d; ++i) pos[members[i]] = i;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < d; ++i) {
        const int64_t u = members[i];
        double ar = s->diag[u] * phi[2 * i], ai = s->diag[u] * phi[2 * i + 1];
        for (int64_t h = s->hoff[u]; h < s->hoff[u + 1]; ++h) {
            const int64_t b = pos[s->hcol[h]];
            if (b < 0) continue;
            int t[3];
            tvec(g, s->hell[h], t);
            double ph = kdot(g, Kv, t);
            double c = s->hval[h] * R[b] / R[i];
            double cr = c * cos(ph), ci = c * sin(ph);
            double xr = phi[2 * b], xi = phi[2 * b + 1];
            ar += cr * xr - ci * xi;
            ai += cr * xi + ci * xr;
        }
        psi[2 * i] = ar;
        psi[2 * i + 1] = ai;
    }
    free(pos);
    return 0;
}
