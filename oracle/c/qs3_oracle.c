/*
 * Plain CPU oracle for the QS^3 hot path (arXiv 2107.00872), for the sizes the
 * Python oracle cannot reach.  TEST INFRASTRUCTURE: only the tests, the smoke
 * check and the benchmark's CPU-baseline leg load this library.  It shares no
 * code with the HIP library.
 *
 * Every routine follows the paper's algorithm literally, in its 1-based
 * notation: ranks a = 1..C(N,K) (Eq. (a_of_n)), ascending down-spin tuples
 * n[1..K] of 1-based sites, binary searches (Alg. 2), spin exchange (Alg. 3),
 * the representative search over all N translations (Alg. 7), check_state /
 * mk_list (Alg. 5/6), ham_to_vec (Alg. 9) looping over every bond of every row,
 * and smq_to_vec (Alg. 11).  OpenMP runs over rows as in the paper.
 *
 * Readings applied (the same as the Python oracle):
 *  - f_bar searches k in [m-1, j-1] (Alg. 1's printed range misses m-1);
 *  - binary_search returns p = ls-1, f = false when s0 < s_ls (Alg. 2 silent);
 *  - spin_exchange inserts r' in the f = true branch (Alg. 3 prints r);
 *  - the k-basis element is (Jxy/2) e^{+ik.t_l} R_{a'}/R_a with R = sqrt(N_{a,k})
 *    (Alg. 8/9 print sqrt(R'/R)); S^-_q uses R'_b/(R_a sqrt N) (Alg. 11 prints
 *    sqrt(R'/(R N)));
 *  - N_{a,k} is tested against 1e-8 rather than 0;
 *  - site r has coordinates r-1 = x + Lx(y + Ly z); translation j = 1..N is the
 *    vector coords(j mod N), so j = N is the identity.
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

static uint64_t C_(const geo_t *g, int k, int m) {
    if (m < 0 || k < m || k < 0) return 0;
    return g->binom[(size_t)k * (g->K + 2) + m];
}

static int geo_init(geo_t *g, int lx, int ly, int lz, int K) {
    g->lx = lx; g->ly = ly; g->lz = lz; g->N = lx * ly * lz; g->K = K;
    if (g->N > MAXN || K + 1 > MAXK) return -1;
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

/* Eq. (a_of_n): a = 1 + sum_m C(n_m - 1, m), n[1..K] */
static uint64_t F_(const geo_t *g, const int *n, int K) {
    uint64_t a = 1;
    for (int m = 1; m <= K; ++m) a += C_(g, n[m] - 1, m);
    return a;
}

/* Alg. 2 on the binomial column m over k in [ls, le] (s_k = C(k, m)) */
static int bsearch_binom(const geo_t *g, uint64_t s0, int m, int ls, int le) {
    if (s0 < C_(g, ls, m)) return ls - 1;
    int lo = ls, hi = le;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (C_(g, mid, m) <= s0) lo = mid; else hi = mid - 1;
    }
    return lo;
}

/* Alg. 2 on the tuple n[1..K]: (p, f) */
static int bsearch_tuple(int r, const int *n, int K, int *f) {
    if (K == 0 || r < n[1]) { *f = 0; return 0; }
    int lo = 1, hi = K;
    while (lo < hi) {
        int mid = (lo + hi + 1) / 2;
        if (n[mid] <= r) lo = mid; else hi = mid - 1;
    }
    *f = (n[lo] == r);
    return lo;
}

/* Alg. 1 */
static void f_bar(const geo_t *g, uint64_t a, int K, int *n) {
    uint64_t s = a;
    int j = g->N;
    for (int m = K; m >= 2; --m) {
        int j0 = bsearch_binom(g, s - 1, m, m - 1, j - 1);
        j = j0;
        n[m] = j0 + 1;
        s -= C_(g, j, m);
    }
    if (K >= 1) n[1] = (int)s;
}

/* Alg. 3 */
static void spin_exchange(int r, int p, int f, int rp, int pp, const int *n, int K, int *out) {
    int o = 1;
    if (!f) {
        for (int i = 1; i <= p; ++i) out[o++] = n[i];
        out[o++] = r;
        for (int i = p + 1; i <= pp - 1; ++i) out[o++] = n[i];
        for (int i = pp + 1; i <= K; ++i) out[o++] = n[i];
    } else {
        for (int i = 1; i <= p - 1; ++i) out[o++] = n[i];
        for (int i = p + 1; i <= pp; ++i) out[o++] = n[i];
        out[o++] = rp;
        for (int i = pp + 1; i <= K; ++i) out[o++] = n[i];
    }
}

static void coords(const geo_t *g, int r, int *x, int *y, int *z) {
    int i = r - 1;
    *x = i % g->lx; *y = (i / g->lx) % g->ly; *z = i / (g->lx * g->ly);
}

static void tvec(const geo_t *g, int j, int *t) {
    int s = (j % g->N) + 1;
    coords(g, s, &t[0], &t[1], &t[2]);
}

static double kdot(const geo_t *g, const int *Kv, const int *t) {
    return 2.0 * M_PI * ((double)Kv[0] * t[0] / g->lx + (double)Kv[1] * t[1] / g->ly +
                         (double)Kv[2] * t[2] / g->lz);
}

/* shift_func followed by insertion_sort (Alg. 5 / Alg. 7) */
static void shift_sort(const geo_t *g, const int *n, int K, const int *t, int *out) {
    for (int m = 1; m <= K; ++m) {
        int x, y, z;
        coords(g, n[m], &x, &y, &z);
        x = (x + t[0]) % g->lx; y = (y + t[1]) % g->ly; z = (z + t[2]) % g->lz;
        out[m] = 1 + x + g->lx * (y + g->ly * z);
    }
    for (int i = 2; i <= K; ++i) {
        int v = out[i], j = i - 1;
        while (j >= 1 && out[j] > v) { out[j + 1] = out[j]; --j; }
        out[j + 1] = v;
    }
}

/* Alg. 7 */
static uint64_t representative(const geo_t *g, uint64_t an, int K, int *ell) {
    int n[MAXK + 1], n2[MAXK + 1], t[3];
    uint64_t rep = an;
    *ell = g->N;
    f_bar(g, an, K, n);
    for (int j = 1; j <= g->N; ++j) {
        tvec(g, j, t);
        shift_sort(g, n, K, t, n2);
        uint64_t a = F_(g, n2, K);
        if (a <= rep) { rep = a; *ell = j; }
    }
    return rep;
}

/* Alg. 5 */
static double check_state(const geo_t *g, uint64_t a, int K, const int *Kv) {
    int n[MAXK + 1], n2[MAXK + 1], t[3];
    f_bar(g, a, K, n);
    double cr = 0, ci = 0;
    int nc = 0;
    for (int j = 1; j <= g->N; ++j) {
        tvec(g, j, t);
        shift_sort(g, n, K, t, n2);
        uint64_t a2 = F_(g, n2, K);
        if (a2 < a) return 0.0;
        if (a2 == a) {
            double ph = kdot(g, Kv, t);
            cr += cos(ph); ci += sin(ph); ++nc;
        }
    }
    double Nak = (cr * cr + ci * ci) * g->N / nc;
    return Nak > 1e-8 ? Nak : 0.0;
}

/* Alg. 2 on sigma[0..d-1] (ascending): 1-based index or 0 if absent */
static int64_t bsearch_sigma(const uint64_t *sigma, int64_t d, uint64_t x) {
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
        f_bar(&g, a[i], K, n);
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
        a_out[i] = F_(&g, n, K);
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
    int64_t total = rows ? nrows : (int64_t)C_(&g, N, K);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < total; ++i) {
        uint64_t a = rows ? rows[i] : (uint64_t)(i + 1);
        int n[MAXK + 1], n2[MAXK + 1];
        f_bar(&g, a, K, n);
        double acc = 0.0;
        for (int b = 0; b < nb; ++b) {
            int f, fp;
            int p = bsearch_tuple(br[b], n, K, &f);
            int pp = bsearch_tuple(brp[b], n, K, &fp);
            if (f == fp) {
                acc += jz[b] / 4.0 * phi[a - 1];
            } else {
                acc -= jz[b] / 4.0 * phi[a - 1];
                spin_exchange(br[b], p, f, brp[b], pp, n, K, n2);
                uint64_t a2 = F_(&g, n2, K);
                acc += jxy[b] / 2.0 * phi[a2 - 1];
            }
        }
        psi[i] = acc;
    }
    geo_free(&g);
    return 0;
}

/* Sparsity of one U(1) row in bond order: cols (0-based ranks) and values;
 * returns the number of off-diagonal entries, diag in *diag. */
int orc_row_u1(int N, int K, int nb, const int32_t *br, const int32_t *brp, const double *jxy,
               const double *jz, uint64_t a, double *diag, uint64_t *cols, double *vals) {
    geo_t g;
    if (geo_init(&g, N, 1, 1, K)) return -1;
    int n[MAXK + 1], n2[MAXK + 1], cnt = 0;
    f_bar(&g, a, K, n);
    double dg = 0.0;
    for (int b = 0; b < nb; ++b) {
        int f, fp;
        int p = bsearch_tuple(br[b], n, K, &f);
        int pp = bsearch_tuple(brp[b], n, K, &fp);
        if (f == fp) dg += jz[b] / 4.0;
        else {
            dg -= jz[b] / 4.0;
            spin_exchange(br[b], p, f, brp[b], pp, n, K, n2);
            cols[cnt] = F_(&g, n2, K) - 1;
            vals[cnt] = jxy[b] / 2.0;
            ++cnt;
        }
    }
    *diag = dg;
    geo_free(&g);
    return cnt;
}

/* Alg. 6 (mk_list), parallel over ranks.  First call with sigma == NULL to get
 * d; then with buffers of that size.  R[i] = sqrt(N_{a,k}). */
int64_t orc_mk_list(int lx, int ly, int lz, int K, const int32_t *Kv, uint64_t *sigma, double *R,
                    int nthreads) {
    geo_t g;
    if (geo_init(&g, lx, ly, lz, K)) return -1;
    uint64_t D = C_(&g, g.N, K);
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
    int nt = 1;
#ifdef _OPENMP
    nt = omp_get_max_threads();
#endif
    int64_t *cnt = (int64_t *)calloc((size_t)nt + 1, sizeof(int64_t));
    /* pass 1: count per contiguous chunk */
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        uint64_t lo = D * (uint64_t)tid / nt + 1, hi = D * (uint64_t)(tid + 1) / nt;
        int64_t c = 0;
        for (uint64_t a = lo; a <= hi; ++a)
            if (check_state(&g, a, K, Kv) > 0) ++c;
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
                double Nak = check_state(&g, a, K, Kv);
                if (Nak > 0) { sigma[o] = a; R[o] = sqrt(Nak); ++o; }
            }
        }
    }
    free(cnt);
    geo_free(&g);
    return d;
}

/* Alg. 7 for a batch of ranks */
int orc_representative(int lx, int ly, int lz, int K, int64_t count, const uint64_t *a,
                       uint64_t *rep, int32_t *ell) {
    geo_t g;
    if (geo_init(&g, lx, ly, lz, K)) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
        int l;
        rep[i] = representative(&g, a[i], K, &l);
        ell[i] = l;
    }
    geo_free(&g);
    return 0;
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
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < total; ++i) {
        int64_t al = rows ? rows[i] : i + 1;
        int n[MAXK + 1], n2[MAXK + 1], t[3];
        f_bar(&g, sigma[al - 1], K, n);
        double pr = phi[2 * (al - 1)], pi = phi[2 * (al - 1) + 1];
        double ar = 0.0, ai = 0.0;
        for (int b = 0; b < nb; ++b) {
            int f, fp;
            int p = bsearch_tuple(br[b], n, K, &f);
            int pp = bsearch_tuple(brp[b], n, K, &fp);
            if (f == fp) {
                ar += jz[b] / 4.0 * pr; ai += jz[b] / 4.0 * pi;
            } else {
                ar -= jz[b] / 4.0 * pr; ai -= jz[b] / 4.0 * pi;
                spin_exchange(br[b], p, f, brp[b], pp, n, K, n2);
                uint64_t a2 = F_(&g, n2, K);
                int ell;
                uint64_t rep = representative(&g, a2, K, &ell);
                int64_t ap = bsearch_sigma(sigma, d, rep);
                if (ap) {
                    tvec(&g, ell, t);
                    double ph = kdot(&g, Kv, t);
                    double c = jxy[b] / 2.0 * R[ap - 1] / R[al - 1];
                    double cr = c * cos(ph), ci = c * sin(ph);
                    double vr = phi[2 * (ap - 1)], vi = phi[2 * (ap - 1) + 1];
                    ar += cr * vr - ci * vi;
                    ai += cr * vi + ci * vr;
                }
            }
        }
        psi[2 * i] = ar;
        psi[2 * i + 1] = ai;
    }
    geo_free(&g);
    return 0;
}

/* Row alpha (1-based) of the k block in bond order: cols (0-based sigma
 * indices), complex vals interleaved; returns count, diag in *diag. */
int orc_row_k(int lx, int ly, int lz, int K, const int32_t *Kv, int nb, const int32_t *br,
              const int32_t *brp, const double *jxy, const double *jz, const uint64_t *sigma,
              const double *R, int64_t d, int64_t al, double *diag, int64_t *cols, double *vals) {
    geo_t g;
    if (geo_init(&g, lx, ly, lz, K)) return -1;
    int n[MAXK + 1], n2[MAXK + 1], t[3], cnt = 0;
    f_bar(&g, sigma[al - 1], K, n);
    double dg = 0.0;
    for (int b = 0; b < nb; ++b) {
        int f, fp;
        int p = bsearch_tuple(br[b], n, K, &f);
        int pp = bsearch_tuple(brp[b], n, K, &fp);
        if (f == fp) dg += jz[b] / 4.0;
        else {
            dg -= jz[b] / 4.0;
            spin_exchange(br[b], p, f, brp[b], pp, n, K, n2);
            int ell;
            uint64_t rep = representative(&g, F_(&g, n2, K), K, &ell);
            int64_t ap = bsearch_sigma(sigma, d, rep);
            if (ap) {
                tvec(&g, ell, t);
                double ph = kdot(&g, Kv, t);
                double c = jxy[b] / 2.0 * R[ap - 1] / R[al - 1];
                cols[cnt] = ap - 1;
                vals[2 * cnt] = c * cos(ph);
                vals[2 * cnt + 1] = c * sin(ph);
                ++cnt;
            }
        }
    }
    *diag = dg;
    geo_free(&g);
    return cnt;
}

/* Alg. 11: psi1 = S^-_q phi, scatter over r and alpha (per-thread buffers,
 * summed in thread order). */
int orc_smq(int lx, int ly, int lz, int K, const int32_t *Kv, const uint64_t *sigma,
            const double *R, int64_t d, const double *phi, const uint64_t *sigma1,
            const double *R1, int64_t d1, const int32_t *Qv, double *psi1, int nthreads) {
    geo_t g, g1;
    if (geo_init(&g, lx, ly, lz, K)) return -1;
    if (geo_init(&g1, lx, ly, lz, K + 1)) return -1;
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
                int n[MAXK + 2], n2[MAXK + 2], f;
                f_bar(&g, sigma[al - 1], K, n);
                int p = bsearch_tuple(r, n, K, &f);
                if (f) continue;
                int o = 1;
                for (int i = 1; i <= p; ++i) n2[o++] = n[i];
                n2[o++] = r;
                for (int i = p + 1; i <= K; ++i) n2[o++] = n[i];
                uint64_t b = F_(&g1, n2, K + 1);
                int ell;
                uint64_t rep = representative(&g1, b, K + 1, &ell);
                int64_t bi = bsearch_sigma(sigma1, d1, rep);
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
