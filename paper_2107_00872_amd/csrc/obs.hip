// Observables (Sec. 3.6, Sec. 4.2), S^-_q (Sec. 3.8, Alg. 11) and the
// continued-fraction dynamical structure factor (Sec. 3.9, Eq. (cfe)).
// Device work runs in the gather kernels of obs_kernels.h; the host only sums
// the per-block partials in a fixed order and evaluates Fourier sums and the
// continued fraction (O(N^2 n_q) and O(steps n_omega) scalars).
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstring>
#include <map>
#include <numeric>
#include <unordered_map>
#include <vector>

#include "qs3_hv.h"
#include "qs3_impl.h"
#include "qs3_krylov.h"

namespace qs3 {

#define QS3_SW7(K, CALL)          \
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

static int obs_u1(qs3_sector *sec, const double *phi, int npairs, const int32_t *pi, const int32_t *pj,
                  std::vector<double> &p, std::vector<double> &q, std::vector<double> &pm, hipStream_t s,
                  const int32_t *hpi = nullptr, const int32_t *hpj = nullptr) {
#define QS3_OU1(k) obs_u1_K<k>(sec, phi, npairs, pi, pj, p, q, pm, s, hpi, hpj)
    QS3_SW7(sec->K, QS3_OU1)
#undef QS3_OU1
}

static int corr_k(qs3_sector *sec, const double *phi, int nd, const int32_t *disp, std::vector<double> &zz,
                  std::vector<double> &nr, std::vector<double> &pr, std::vector<double> &pim, hipStream_t s) {
#define QS3_CK(k) corr_k_K<(k > 6 ? 6 : k)>(sec, phi, nd, disp, zz, nr, pr, pim, s)
    QS3_SW7(sec->K, QS3_CK)
#undef QS3_CK
}

static int smq_any(qs3_batch *src, qs3_batch *dst, const int32_t *qmul, const double2 *subph, const double *phi, double *out,
                   hipStream_t s) {
#define QS3_SQ(k) smq_K<(k > 5 ? 5 : k)>(src, dst, qmul, subph, phi, out, s)
    QS3_REQUIRE(src->K <= 5, QS3_EINVAL, "S^-_q needs N_down + 1 <= 6");
    QS3_SW7(src->K, QS3_SQ)
#undef QS3_SQ
}

// S^op_q from the source batch (one sector) into the target batch
static int sq_any(int op, qs3_batch *src, qs3_batch *dst, const int32_t *qmul, const double2 *subph, const double *phi,
                  double *out, hipStream_t s) {
    if (op == QS3_OP_SMINUS) return smq_any(src, dst, qmul, subph, phi, out, s);
#define QS3_SP(k) spq_K<(k > 6 ? 6 : k)>(src, dst, qmul, subph, phi, out, s)
#define QS3_SZ(k) szq_K<(k > 6 ? 6 : k)>(src, dst, qmul, subph, phi, out, s)
    if (op == QS3_OP_SPLUS) {
        QS3_REQUIRE(src->K >= 1 && src->K <= 6, QS3_EINVAL, "S^+_q needs 1 <= N_down <= 6");
        QS3_SW7(src->K, QS3_SP)
    }
    if (op == QS3_OP_SZ) {
        QS3_REQUIRE(src->K <= 6, QS3_EINVAL, "S^z_q needs N_down <= 6");
        QS3_SW7(src->K, QS3_SZ)
    }
#undef QS3_SP
#undef QS3_SZ
    set_error("unknown spin operator");
    return QS3_EINVAL;
}

static int n_down_after(int op, int K) {
    return op == QS3_OP_SMINUS ? K + 1 : (op == QS3_OP_SPLUS ? K - 1 : K);
}

// ---- shared helpers
static int vec_norm2(qs3_sector *sec, const void *vec, double *out, hipStream_t s) {
    // |vec|^2 through the engine's deterministic reduction
    struct NoOp : Operator {
        uint64_t n;
        bool c;
        uint64_t rows() const override { return n; }
        int cols() const override { return 1; }
        bool is_complex() const override { return c; }
        int apply(const double *, double *, hipStream_t) override { return QS3_EINVAL; }
        int apply_f32in(const float *, double *, hipStream_t) override { return QS3_EINVAL; }
    } op;
    op.n = sec->dim;
    op.c = sec->has_k;
    Engine E;
    QS3_TRY(E.init(sec->lat->ctx, &op, 1, QS3_PREC_F64, 0, s));
    std::vector<double> nr;
    QS3_TRY(E.normalize_into_slot0((const double *)vec, &nr));
    *out = nr[0] * nr[0];
    return QS3_OK;
}

// Translation-averaged correlations of a momentum-sector state for every
// displacement d: Czz[d] = (1/N) <sum_r s^z_r s^z_{r+d}>,
// Cpm[d] = (1/N) <sum_r s^+_r s^-_{r+d}> (Sec. 3.6).
// Translation-averaged correlations of a momentum-sector vector for every
// pair class (place s of a cell, place t of the cell d further on), index
// (s * ns + t) * N_T + d:
//   Czz = <s^z_(r,s) s^z_(r+d,t)>, Cpm = <s^+_(r,s) s^-_(r+d,t)>,
// and rho[s] = <number of down spins at place s> / N_T.
static int k_correlations(qs3_sector *sec, const void *vec, std::vector<double> &Czz,
                          std::vector<std::complex<double>> &Cpm, std::vector<double> &rho, hipStream_t s) {
    qs3_lattice *lat = sec->lat;
    const int ns = lat->ns, NT = lat->lx * lat->ly * lat->lz, nc = ns * ns * NT;
    DevBuf un, dd;
    QS3_TRY(un.alloc(lat->ctx, sizeof(double) * 2 * std::max<uint64_t>(sec->bat->ks->n_reps, 1)));
    QS3_TRY(scatter_compact(sec, (const double *)vec, un.as<double>(), s));
    std::vector<int32_t> disp(nc);
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b)
            for (int d = 0; d < NT; ++d) disp[((size_t)a * ns + b) * NT + d] = d | (a << 24) | (b << 28);
    QS3_TRY(dd.alloc(lat->ctx, sizeof(int32_t) * nc));
    QS3_HIP(hipMemcpyAsync(dd.ptr, disp.data(), sizeof(int32_t) * nc, hipMemcpyHostToDevice, s));
    std::vector<double> zz, nr, pr, pim;
    QS3_TRY(corr_k(sec, un.as<double>(), nc, dd.as<int32_t>(), zz, nr, pr, pim, s));
    const double n2 = nr[0];
    QS3_REQUIRE(n2 > 0 && std::isfinite(n2), QS3_ENUMERIC, "zero or non-finite state");
    // a down spin is its own partner in the class (s, s, 0): those sums count the spins
    rho.assign(ns, 0.0);
    for (int a = 0; a < ns; ++a) rho[a] = zz[((size_t)a * ns + a) * NT] / (n2 * NT);
    Czz.assign(nc, 0.0);
    Cpm.assign(nc, 0.0);
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b)
            for (int d = 0; d < NT; ++d) {
                const size_t i = ((size_t)a * ns + b) * NT + d;
                if (a == b && d == 0) {
                    Czz[i] = 0.25;
                    Cpm[i] = 1.0 - rho[a];  // s^+_r s^-_r = 1/2 + s^z_r
                } else {
                    Czz[i] = 0.25 - 0.5 * (rho[a] + rho[b]) + zz[i] / (n2 * NT);
                    Cpm[i] = std::complex<double>(pr[i], pim[i]) / (n2 * NT);
                }
            }
    return QS3_OK;
}

// cell coordinates and place of site i
static void cell_of(const qs3_lattice *lat, int i, int &x, int &y, int &z, int &p) {
    p = i % lat->ns;
    const int c = i / lat->ns;
    x = c % lat->lx;
    y = (c / lat->lx) % lat->ly;
    z = c / (lat->lx * lat->ly);
}

// pair class index (see k_correlations) of the sites (i, j)
static size_t pair_class(const qs3_lattice *lat, int i, int j) {
    int xi, yi, zi, pi, xj, yj, zj, pj;
    cell_of(lat, i, xi, yi, zi, pi);
    cell_of(lat, j, xj, yj, zj, pj);
    const int dx = (xj - xi + lat->lx) % lat->lx, dy = (yj - yi + lat->ly) % lat->ly,
              dz = (zj - zi + lat->lz) % lat->lz;
    const size_t NT = (size_t)lat->lx * lat->ly * lat->lz;
    return ((size_t)pi * lat->ns + pj) * NT + dx + (size_t)lat->lx * (dy + (size_t)lat->ly * dz);
}

// e^{-i q_b . offset_s} for the momenta qvecs (3 ints each, taken modulo the
// lattice lengths) and every place s of a cell, into dev ([b][s], double2)
static int sub_phases(const qs3_lattice *lat, int n_q, const int32_t *qvecs, DevBuf &dev, hipStream_t s) {
    const int ns = lat->ns;
    const int L[3] = {lat->lx, lat->ly, lat->lz};
    std::vector<double2> h((size_t)n_q * ns);
    for (int b = 0; b < n_q; ++b)
        for (int p = 0; p < ns; ++p) {
            double ph = 0;
            for (int a = 0; a < 3; ++a) {
                const int qa = ((qvecs[3 * b + a] % L[a]) + L[a]) % L[a];
                ph += 2.0 * M_PI * qa * lat->basis[3 * p + a] / L[a];
            }
            h[(size_t)b * ns + p] = ph == 0.0 ? make_double2(1.0, 0.0) : make_double2(std::cos(ph), -std::sin(ph));
        }
    QS3_TRY(dev.alloc(lat->ctx, sizeof(double2) * h.size()));
    QS3_HIP(hipMemcpyAsync(dev.ptr, h.data(), sizeof(double2) * h.size(), hipMemcpyHostToDevice, s));
    return QS3_OK;
}

// position of site i: its cell's coordinates plus its place's offset
static void position_of(const qs3_lattice *lat, int i, double *R) {
    int x, y, z, p;
    cell_of(lat, i, x, y, z, p);
    R[0] = x + lat->basis[3 * p];
    R[1] = y + lat->basis[3 * p + 1];
    R[2] = z + lat->basis[3 * p + 2];
}

}  // namespace qs3

using namespace qs3;

extern "C" {

int qs3_sz(qs3_sector *sec, const void *vec, double *out, void *stream) {
    QS3_REQUIRE(sec && vec && out, QS3_EINVAL, "NULL argument");
    hipSetDevice(sec->lat->ctx->device);
    hipStream_t s = (hipStream_t)stream;
    const int N = sec->lat->N;
    double n2 = 0;
    QS3_TRY(vec_norm2(sec, vec, &n2, s));
    QS3_REQUIRE(n2 > 0 && std::isfinite(n2), QS3_ENUMERIC, "zero or non-finite state");
    if (sec->has_k) {
        if (sec->lat->ns == 1) {
            // the translation-averaged s^z_r is (1/N) sum_r s^z_r = M / N in the sector
            for (int i = 0; i < N; ++i) out[i] = (0.5 * N - sec->K) / N;
            return QS3_OK;
        }
        // several places per cell: 1/2 - (down spins at the site's place) / N_T
        std::vector<double> Czz, rho;
        std::vector<std::complex<double>> Cpm;
        QS3_TRY(k_correlations(sec, vec, Czz, Cpm, rho, s));
        for (int i = 0; i < N; ++i) out[i] = 0.5 - rho[i % sec->lat->ns];
        return QS3_OK;
    }
    std::vector<double> p, q, pm;
    QS3_TRY(obs_u1(sec, (const double *)vec, 0, nullptr, nullptr, p, q, pm, s));
    for (int i = 0; i < N; ++i) out[i] = 0.5 - p[i] / n2;
    return QS3_OK;
}

int qs3_sisj(qs3_sector *sec, const void *vec, int n_pairs, const int32_t *pi, const int32_t *pj,
             double *zz, double *pm, void *stream) {
    QS3_REQUIRE(sec && vec && (n_pairs == 0 || (pi && pj && zz && pm)), QS3_EINVAL, "NULL argument");
    hipSetDevice(sec->lat->ctx->device);
    hipStream_t s = (hipStream_t)stream;
    const int N = sec->lat->N;
    for (int p = 0; p < n_pairs; ++p)
        QS3_REQUIRE(pi[p] >= 0 && pi[p] < N && pj[p] >= 0 && pj[p] < N, QS3_EINVAL, "site out of range");
    if (sec->has_k) {
        std::vector<double> Czz, rho;
        std::vector<std::complex<double>> Cpm;
        QS3_TRY(k_correlations(sec, vec, Czz, Cpm, rho, s));
        for (int p = 0; p < n_pairs; ++p) {
            const size_t d = pair_class(sec->lat, pi[p], pj[p]);
            zz[p] = Czz[d];
            pm[2 * p] = Cpm[d].real();
            pm[2 * p + 1] = Cpm[d].imag();
        }
        return QS3_OK;
    }
    double n2 = 0;
    QS3_TRY(vec_norm2(sec, vec, &n2, s));
    QS3_REQUIRE(n2 > 0 && std::isfinite(n2), QS3_ENUMERIC, "zero or non-finite state");
    // the pair sums are symmetric in (i, j) and the kernel forms the same
    // products in the same order for both orders: one launch row per
    // unordered pair
    std::vector<int32_t> hi_, hj_;
    std::vector<int> which(n_pairs, -1);
    std::unordered_map<int64_t, int> uniq;
    for (int p = 0; p < n_pairs; ++p)
        if (pi[p] != pj[p]) {
            const int lo = std::min(pi[p], pj[p]), hi = std::max(pi[p], pj[p]);
            auto ins = uniq.emplace((int64_t)lo * N + hi, (int)hi_.size());
            if (ins.second) {
                hi_.push_back(lo);
                hj_.push_back(hi);
            }
            which[p] = ins.first->second;
        }
    DevBuf dpi, dpj;
    const int np = (int)hi_.size();
    QS3_TRY(dpi.alloc(sec->lat->ctx, sizeof(int32_t) * std::max(np, 1)));
    QS3_TRY(dpj.alloc(sec->lat->ctx, sizeof(int32_t) * std::max(np, 1)));
    if (np) {
        QS3_HIP(hipMemcpyAsync(dpi.ptr, hi_.data(), sizeof(int32_t) * np, hipMemcpyHostToDevice, s));
        QS3_HIP(hipMemcpyAsync(dpj.ptr, hj_.data(), sizeof(int32_t) * np, hipMemcpyHostToDevice, s));
    }
    std::vector<double> p, q, pmv;
    QS3_TRY(obs_u1(sec, (const double *)vec, np, dpi.as<int32_t>(), dpj.as<int32_t>(), p, q, pmv, s, hi_.data(),
                   hj_.data()));
    for (int t = 0; t < n_pairs; ++t) {
        if (pi[t] == pj[t]) {
            zz[t] = 0.25;
            pm[2 * t] = 1.0 - p[pi[t]] / n2;  // 1/2 + <s^z_i>
            pm[2 * t + 1] = 0.0;
        }
    }
    for (int t = 0; t < n_pairs; ++t) {
        const int k = which[t];
        if (k < 0) continue;
        const double xi = p[pi[t]] / n2, xj = p[pj[t]] / n2;
        zz[t] = 0.25 - 0.5 * (xi + xj) + q[k] / n2;
        pm[2 * t] = pmv[k] / n2;
        pm[2 * t + 1] = 0.0;
    }
    return QS3_OK;
}

int qs3_sq(qs3_sector *sec, const void *vec, int n_q, const double *qv, double *szz, double *spm,
           double *stot, void *stream) {
    QS3_REQUIRE(sec && vec && qv && szz && spm && stot && n_q >= 0, QS3_EINVAL, "NULL argument");
    hipSetDevice(sec->lat->ctx->device);
    hipStream_t s = (hipStream_t)stream;
    qs3_lattice *lat = sec->lat;
    const int N = lat->N;
    std::vector<double> R(3 * N);
    for (int r = 0; r < N; ++r) position_of(lat, r, &R[3 * r]);
    if (sec->has_k) {
        // S(q) = (1/ns) sum over pair classes (s, t, d) of e^{-i q.(R_(d,t) - R_(0,s))} C(s, t, d)
        // with the translation-averaged C
        std::vector<double> Czz, rho;
        std::vector<std::complex<double>> Cpm;
        QS3_TRY(k_correlations(sec, vec, Czz, Cpm, rho, s));
        const int ns = lat->ns, NT = lat->lx * lat->ly * lat->lz;
        for (int k = 0; k < n_q; ++k) {
            std::complex<double> a = 0, b = 0, c = 0;
            for (int p0 = 0; p0 < ns; ++p0)
                for (int p1 = 0; p1 < ns; ++p1)
                    for (int d = 0; d < NT; ++d) {
                        const int j = p1 + ns * d;  // place p1 of cell d
                        double ph = 0;
                        for (int ax = 0; ax < 3; ++ax) ph += qv[3 * k + ax] * (R[3 * j + ax] - R[3 * p0 + ax]);
                        const std::complex<double> e(std::cos(ph), -std::sin(ph));
                        const size_t i = ((size_t)p0 * ns + p1) * NT + d;
                        a += e * Czz[i];
                        b += e * Cpm[i];
                        // <s^-_(0,p0) s^+_(d,p1)> = <s^+_(d,p1) s^-_(0,p0)> (class (p1, p0, -d));
                        // on one site 1/2 - s^z = rho
                        const std::complex<double> mp =
                            (p0 == p1 && d == 0) ? std::complex<double>(rho[p0]) : Cpm[pair_class(lat, j, p0)];
                        c += e * mp;
                    }
            szz[k] = a.real() / ns;
            spm[k] = b.real() / ns;
            stot[k] = (a.real() + 0.5 * (b.real() + c.real())) / ns;
        }
        return QS3_OK;
    }
    // fixed-N_down: all pairs, then the Fourier sums
    std::vector<int32_t> pi, pj;
    for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
            pi.push_back(i);
            pj.push_back(j);
        }
    std::vector<double> zz(N * N), pm(2 * N * N);
    QS3_TRY(qs3_sisj(sec, vec, N * N, pi.data(), pj.data(), zz.data(), pm.data(), stream));
    for (int k = 0; k < n_q; ++k) {
        std::vector<std::complex<double>> e(N);
        for (int r = 0; r < N; ++r) {
            const double ph = qv[3 * k] * R[3 * r] + qv[3 * k + 1] * R[3 * r + 1] + qv[3 * k + 2] * R[3 * r + 2];
            e[r] = std::complex<double>(std::cos(ph), std::sin(ph));
        }
        double a = 0, b = 0, c = 0;
        for (int r = 0; r < N; ++r)
            for (int rp = 0; rp < N; ++rp) {
                const std::complex<double> w = e[r] * std::conj(e[rp]);
                a += (w * zz[r * N + rp]).real();
                b += (w * std::complex<double>(pm[2 * (r * N + rp)], pm[2 * (r * N + rp) + 1])).real();
                const double mp = (r == rp) ? (1.0 - pm[2 * (r * N + r)]) : pm[2 * (rp * N + r)];
                c += (w * mp).real();
            }
        szz[k] = a / N;
        spm[k] = b / N;
        stot[k] = (a + 0.5 * (b + c)) / N;
    }
    return QS3_OK;
}

int qs3_sq_apply(qs3_sector *from, const void *vec_from, qs3_sector *to, int op, const int32_t *qvec,
                 void *vec_to, void *stream) {
    QS3_REQUIRE(from && to && vec_from && vec_to && qvec, QS3_EINVAL, "NULL argument");
    QS3_REQUIRE(op == QS3_OP_SMINUS || op == QS3_OP_SPLUS || op == QS3_OP_SZ, QS3_EINVAL,
                "unknown spin operator");
    QS3_REQUIRE(from->has_k && to->has_k, QS3_EINVAL, "S^a_q acts between momentum sectors");
    QS3_REQUIRE(from->lat == to->lat && to->K == n_down_after(op, from->K), QS3_EINVAL,
                "target sector must be the same lattice with N_down + 1 (S^-), - 1 (S^+) or + 0 (S^z)");
    qs3_lattice *lat = from->lat;
    const int L[3] = {lat->lx, lat->ly, lat->lz};
    for (int a = 0; a < 3; ++a)
        QS3_REQUIRE(((from->kv[a] + qvec[a]) % L[a] + L[a]) % L[a] == to->kv[a], QS3_EINVAL,
                    "target momentum must be k + q");
    hipSetDevice(lat->ctx->device);
    hipStream_t s = (hipStream_t)stream;
    const int M = from->bat->M;
    int32_t qm[3] = {(int)(((long)((qvec[0] % L[0]) + L[0]) % L[0]) * (M / L[0]) % M),
                     (int)(((long)((qvec[1] % L[1]) + L[1]) % L[1]) * (M / L[1]) % M),
                     (int)(((long)((qvec[2] % L[2]) + L[2]) % L[2]) * (M / L[2]) % M)};
    DevBuf ua, ub, dq;
    QS3_TRY(ua.alloc(lat->ctx, sizeof(double) * 2 * std::max<uint64_t>(from->bat->ks->n_reps, 1)));
    QS3_TRY(ub.alloc(lat->ctx, sizeof(double) * 2 * std::max<uint64_t>(to->bat->ks->n_reps, 1)));
    QS3_TRY(dq.alloc(lat->ctx, sizeof(qm)));
    QS3_HIP(hipMemcpyAsync(dq.ptr, qm, sizeof(qm), hipMemcpyHostToDevice, s));
    DevBuf sp;
    QS3_TRY(sub_phases(lat, 1, qvec, sp, s));
    QS3_TRY(scatter_compact(from, (const double *)vec_from, ua.as<double>(), s));
    QS3_TRY(sq_any(op, from->bat, to->bat, dq.as<int32_t>(), sp.as<double2>(), ua.as<double>(), ub.as<double>(), s));
    QS3_TRY(gather_compact(to, ub.as<double>(), (double *)vec_to, s));
    QS3_HIP(hipStreamSynchronize(s));
    return QS3_OK;
}

}  // extern "C"

namespace qs3 {

struct CfArgs {
    int n_q, n_omega;
    const double *alpha, *beta;  // [x][q]: the Lanczos coefficients of column q
    const double *weight, *triv; // per q: |psi'|^2, weight of the trivial q = 0 pole (or 0)
    const int32_t *m;            // per q: levels taken (0: no weight)
    const double *omega;
    double zshift, eta;          // z = omega + zshift + i eta
};

// Eq. (cfe), one thread per (q, omega): G(z) by the backward recurrence
// g_i = 1 / (z - alpha_i - beta_i^2 g_{i+1}) from the innermost level out,
// S = -Im(weight g_0) / pi, minus the trivial Lorentzian where asked.
__global__ __launch_bounds__(256) void k_cfrac(CfArgs C, double *__restrict__ S) {
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (uint64_t)C.n_q * C.n_omega) return;
    const int q = (int)(t / C.n_omega), k = (int)(t % C.n_omega);
    const double pi = 3.141592653589793;
    const double om = C.omega[k];
    const double tr = C.triv[q] != 0.0 ? C.triv[q] * C.eta / (pi * (om * om + C.eta * C.eta)) : 0.0;
    const int m = C.m[q];
    if (m == 0) {
        S[t] = -tr;
        return;
    }
    const double zr = om + C.zshift, zi = C.eta;
    double gr = 0.0, gi = 0.0;
    for (int i = m - 1; i >= 0; --i) {
        const double b = i < m - 1 ? C.beta[(size_t)i * C.n_q + q] : 0.0;
        const double b2 = b * b;
        const double dr = zr - C.alpha[(size_t)i * C.n_q + q] - b2 * gr;
        const double di = zi - b2 * gi;
        const double inv = 1.0 / (dr * dr + di * di);
        gr = dr * inv;
        gi = -di * inv;
    }
    S[t] = -(C.weight[q] * gi) / pi - tr;
}

}  // namespace qs3

extern "C" {

int qs3_smq(qs3_sector *from, const void *vec_from, qs3_sector *to, const int32_t *qvec, void *vec_to,
            void *stream) {
    return qs3_sq_apply(from, vec_from, to, QS3_OP_SMINUS, qvec, vec_to, stream);
}

int qs3_dsf(qs3_sector *gs, const void *gs_vec, double e0, int n_q, const int32_t *qvecs,
            const qs3_dsf_opts *opts, int n_omega, const double *omega, double *S, double *alpha,
            double *beta, double *weight, void *stream) {
    QS3_REQUIRE(gs && gs_vec && qvecs && opts && n_q > 0 && n_omega >= 0, QS3_EINVAL, "bad argument");
    QS3_REQUIRE(gs->has_k, QS3_EINVAL, "the ground state must be a momentum-sector vector");
    const int op = opts->op;
    QS3_REQUIRE(op == QS3_OP_SMINUS || op == QS3_OP_SPLUS || op == QS3_OP_SZ, QS3_EINVAL,
                "unknown spin operator");
    const int K1 = n_down_after(op, gs->K);
    QS3_REQUIRE(K1 >= 0 && K1 <= 6 && K1 <= gs->lat->N, QS3_EINVAL,
                "the target N_down must lie in 0..6");
    qs3_lattice *lat = gs->lat;
    hipSetDevice(lat->ctx->device);
    hipStream_t s = (hipStream_t)stream;
    const int steps = opts->steps > 0 ? opts->steps : 300;
    const int L[3] = {lat->lx, lat->ly, lat->lz};
    const int M = gs->bat->M;
    // target sectors k0 + q, one batch column each
    std::vector<int32_t> kt(3 * n_q), qm(3 * n_q);
    for (int b = 0; b < n_q; ++b)
        for (int a = 0; a < 3; ++a) {
            const int qa = ((qvecs[3 * b + a] % L[a]) + L[a]) % L[a];
            kt[3 * b + a] = (gs->kv[a] + qa) % L[a];
            qm[3 * b + a] = (int)((long)qa * (M / L[a]) % M);
        }
    qs3_batch *tb = nullptr;
    QS3_TRY(qs3_batch_create(lat, K1, n_q, kt.data(), &tb));
    std::unique_ptr<qs3_batch, int (*)(qs3_batch *)> tb_guard(tb, qs3_batch_destroy);
    DevBuf ua, psi, dq;
    QS3_TRY(ua.alloc(lat->ctx, sizeof(double) * 2 * std::max<uint64_t>(gs->bat->ks->n_reps, 1)));
    QS3_TRY(psi.alloc(lat->ctx, sizeof(double) * 2 * std::max<uint64_t>(tb->ks->n_reps, 1) * n_q));
    QS3_TRY(dq.alloc(lat->ctx, sizeof(int32_t) * 3 * n_q));
    QS3_HIP(hipMemcpyAsync(dq.ptr, qm.data(), sizeof(int32_t) * 3 * n_q, hipMemcpyHostToDevice, s));
    QS3_TRY(scatter_compact(gs, (const double *)gs_vec, ua.as<double>(), s));
    // normalise the ground state on the fly: weights use |gs|^2 = 1
    double g2 = 0;
    QS3_TRY(vec_norm2(gs, gs_vec, &g2, s));
    QS3_REQUIRE(g2 > 0 && std::isfinite(g2), QS3_ENUMERIC, "zero or non-finite ground state");
    DevBuf sp;
    QS3_TRY(sub_phases(lat, n_q, qvecs, sp, s));
    QS3_TRY(sq_any(op, gs->bat, tb, dq.as<int32_t>(), sp.as<double2>(), ua.as<double>(), psi.as<double>(), s));
    // Lanczos from psi'/|psi'| in every target sector (Alg. 10, lines 3-11)
    struct TOp : Operator {
        qs3_batch *b;
        uint64_t rows() const override { return b->ks->n_reps; }
        int cols() const override { return b->B; }
        bool is_complex() const override { return true; }
        int apply(const double *x, double *y, hipStream_t st) override {
            return hv_batch(b, x, QS3_C128, y, QS3_C128, st);
        }
        int apply_f32in(const float *x, double *y, hipStream_t st) override {
            return hv_batch(b, x, QS3_C64, y, QS3_C128, st);
        }
    } top;
    top.b = tb;
    Engine E;
    QS3_REQUIRE(opts->reorth >= QS3_REORTH_NONE && opts->reorth <= QS3_REORTH_PARTIAL, QS3_EINVAL,
                "unknown reorthogonalisation mode");
    QS3_TRY(E.init(lat->ctx, &top, steps + 1, opts->precision, engine_reorth(opts->reorth, false), s));
    std::vector<double> a, bb, n0;
    std::vector<int> done;
    QS3_TRY(run_lanczos(E, psi.as<double>(), steps, a, bb, n0, done));
    // the field moves the poles by the Zeeman change of the operator
    const double shift = op == QS3_OP_SMINUS ? opts->field : (op == QS3_OP_SPLUS ? -opts->field : 0.0);
    const double Mz = 0.5 * lat->N - gs->K;
    std::vector<double> wq(n_q), triv_w(n_q);
    std::vector<int32_t> mq(n_q);
    for (int q = 0; q < n_q; ++q) {
        bool q0 = true;
        for (int a = 0; a < 3; ++a) q0 &= (((qvecs[3 * q + a] % L[a]) + L[a]) % L[a]) == 0;
        const bool trivial = op == QS3_OP_SZ && opts->subtract_trivial && q0;
        wq[q] = n0[q] * n0[q] / g2;
        triv_w[q] = trivial ? Mz * Mz / lat->N : 0.0;
        mq[q] = (wq[q] > 0) ? done[q] : 0;
        if (weight) weight[q] = wq[q];
        if (alpha)
            for (int x = 0; x < steps; ++x) alpha[(size_t)q * steps + x] = a[(size_t)q * steps + x];
        if (beta)
            for (int x = 0; x < steps; ++x) beta[(size_t)q * steps + x] = bb[(size_t)q * steps + x];
    }
    if (n_omega == 0) return QS3_OK;
    // Eq. (cfe) for every (q, omega) on the device, from the coefficient
    // history the Lanczos run left there
    DevBuf par, dom, dS;
    QS3_TRY(par.alloc(lat->ctx, sizeof(double) * 2 * n_q + sizeof(int32_t) * n_q));
    QS3_TRY(dom.alloc(lat->ctx, sizeof(double) * n_omega));
    QS3_TRY(dS.alloc(lat->ctx, sizeof(double) * (size_t)n_q * n_omega));
    std::vector<char> hp(sizeof(double) * 2 * n_q + sizeof(int32_t) * n_q);
    std::memcpy(hp.data(), wq.data(), sizeof(double) * n_q);
    std::memcpy(hp.data() + sizeof(double) * n_q, triv_w.data(), sizeof(double) * n_q);
    std::memcpy(hp.data() + sizeof(double) * 2 * n_q, mq.data(), sizeof(int32_t) * n_q);
    QS3_HIP(hipMemcpyAsync(par.ptr, hp.data(), hp.size(), hipMemcpyHostToDevice, s));
    QS3_HIP(hipMemcpyAsync(dom.ptr, omega, sizeof(double) * n_omega, hipMemcpyHostToDevice, s));
    CfArgs C;
    C.n_q = n_q;
    C.n_omega = n_omega;
    C.alpha = E.ab_hist.as<double>();
    C.beta = E.ab_hist.as<double>() + (size_t)E.slots * n_q;
    C.weight = par.as<double>();
    C.triv = par.as<double>() + n_q;
    C.m = (const int32_t *)(par.as<double>() + 2 * n_q);
    C.omega = dom.as<double>();
    C.zshift = e0 - shift;
    C.eta = opts->eta;
    const uint64_t nt = (uint64_t)n_q * n_omega;
    hipLaunchKernelGGL(k_cfrac, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, C, dS.as<double>());
    QS3_HIP(hipGetLastError());
    QS3_HIP(hipMemcpyAsync(S, dS.ptr, sizeof(double) * nt, hipMemcpyDeviceToHost, s));
    QS3_HIP(hipStreamSynchronize(s));
    return QS3_OK;
}

}  // extern "C"
