// Drives every part of the C-ABI's host code once -- argument validation and
// error paths, sector and structure construction, the solvers' host control
// (restart bookkeeping, the Ritz eigensolver, level selection), observables,
// S(q, omega), batches, point-group sectors and the serving scheduler with
// admission, refusal and cancellation -- so that a build of the library whose
// host code carries AddressSanitizer and UndefinedBehaviorSanitizer (device
// code unchanged) sees all of it.  Results are checked for consistency only
// (status codes, finite values, identities that hold exactly); the numerics
// themselves are the parity tests' business.  Exit status 0 when every check
// holds; a sanitizer report aborts the process.
#include <hip/hip_runtime.h>
#include <sanitizer/lsan_interface.h>
#include <unistd.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "qs3.h"

static int g_fail = 0;

#define CHECK(cond)                                                                   \
    do {                                                                              \
        if (!(cond)) {                                                                \
            std::fprintf(stderr, "check failed at line %d: %s (%s)\n", __LINE__, #cond, \
                         qs3_last_error());                                           \
            ++g_fail;                                                                 \
        }                                                                             \
    } while (0)

#define HIPOK(x) CHECK((x) == hipSuccess)

struct Bonds {
    std::vector<int32_t> bi, bj;
    std::vector<double> jxy, jz;
    void add(int i, int j, double J, double D) {
        bi.push_back(i);
        bj.push_back(j);
        jxy.push_back(J);
        jz.push_back(J * D);
    }
    int n() const { return (int)bi.size(); }
};

// nearest-neighbour bonds of a periodic lx x ly x lz lattice (site x + lx (y + ly z))
static Bonds hyper(int lx, int ly, int lz, double J = 1.0, double D = 1.0) {
    Bonds b;
    for (int z = 0; z < lz; ++z)
        for (int y = 0; y < ly; ++y)
            for (int x = 0; x < lx; ++x) {
                const int s = x + lx * (y + ly * z);
                if (lx > 1) b.add(s, (x + 1) % lx + lx * (y + ly * z), J, D);
                if (ly > 1) b.add(s, x + lx * ((y + 1) % ly + ly * z), J, D);
                if (lz > 1) b.add(s, x + lx * (y + ly * ((z + 1) % lz)), J, D);
            }
    return b;
}

static qs3_lattice *lattice(qs3_ctx *ctx, int lx, int ly, int lz, const Bonds &b) {
    qs3_lattice *lat = nullptr;
    CHECK(qs3_lattice_create(ctx, lx, ly, lz, b.n(), b.bi.data(), b.bj.data(), b.jxy.data(), b.jz.data(),
                             &lat) == QS3_OK);
    return lat;
}

static void *dalloc(size_t bytes) {
    void *p = nullptr;
    HIPOK(hipMalloc(&p, bytes ? bytes : 16));
    return p;
}

static bool all_finite(const double *x, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(x[i])) return false;
    return true;
}

static void check_errors(qs3_ctx *ctx) {
    for (int c = 0; c >= -8; --c) CHECK(qs3_strerror(c) != nullptr);
    CHECK(qs3_version() != nullptr);
    Bonds b = hyper(8, 1, 1);
    qs3_lattice *lat = nullptr;
    // a site out of range, a bond from a site to itself, no bonds array
    Bonds bad = b;
    bad.bj[3] = 99;
    CHECK(qs3_lattice_create(ctx, 8, 1, 1, bad.n(), bad.bi.data(), bad.bj.data(), bad.jxy.data(), bad.jz.data(),
                             &lat) == QS3_EINVAL);
    bad = b;
    bad.bj[2] = bad.bi[2];
    CHECK(qs3_lattice_create(ctx, 8, 1, 1, bad.n(), bad.bi.data(), bad.bj.data(), bad.jxy.data(), bad.jz.data(),
                             &lat) == QS3_EINVAL);
    CHECK(qs3_lattice_create(ctx, 8, 1, 1, b.n(), nullptr, b.bj.data(), b.jxy.data(), b.jz.data(), &lat) ==
          QS3_EINVAL);
    CHECK(qs3_lattice_create(ctx, 0, 1, 1, 0, nullptr, nullptr, nullptr, nullptr, &lat) == QS3_EINVAL);
    lat = lattice(ctx, 8, 1, 1, b);
    qs3_sector *sec = nullptr;
    CHECK(qs3_sector_create(lat, 9, nullptr, &sec) == QS3_EINVAL);
    CHECK(qs3_sector_create(lat, -1, nullptr, &sec) == QS3_EINVAL);
    const int32_t kbad[3] = {8, 0, 0};
    CHECK(qs3_sector_create(lat, 2, kbad, &sec) == QS3_EINVAL);
    // a bond set without translation symmetry refuses momentum sectors
    Bonds dis = b;
    dis.jxy[0] = 0.7;
    dis.jz[0] = 0.7;
    qs3_lattice *ldis = lattice(ctx, 8, 1, 1, dis);
    int n = 0, ti = 1;
    CHECK(qs3_lattice_info(ldis, &n, &ti) == QS3_OK && n == 8 && ti == 0);
    const int32_t k0[3] = {0, 0, 0};
    CHECK(qs3_sector_create(ldis, 2, k0, &sec) == QS3_EINVAL);
    const int32_t kv[3] = {0, 0, 0};
    qs3_batch *bat = nullptr;
    CHECK(qs3_batch_create(ldis, 2, 1, kv, &bat) == QS3_EINVAL);
    qs3_lattice_destroy(ldis);
    qs3_lattice_destroy(lat);
}

static void check_u1(qs3_ctx *ctx, hipStream_t s) {
    Bonds b = hyper(16, 1, 1);
    qs3_lattice *lat = lattice(ctx, 16, 1, 1, b);
    qs3_sector *sec = nullptr;
    CHECK(qs3_sector_create(lat, 3, nullptr, &sec) == QS3_OK);
    uint64_t dim = 0;
    CHECK(qs3_sector_dim(sec, &dim) == QS3_OK && dim == 560);
    double *v = (double *)dalloc(dim * 8), *w = (double *)dalloc(dim * 8);
    CHECK(qs3_sector_start_vector(sec, 1, v, QS3_F64, s) == QS3_OK);
    CHECK(qs3_matvec(sec, v, w, QS3_F64, s) == QS3_OK);
    CHECK(qs3_matvec(sec, v, v, QS3_F64, s) == QS3_EINVAL);  // aliasing
    std::vector<int64_t> cols(64);
    std::vector<double> vals(64);
    double diag = 0;
    int nnz = 0;
    CHECK(qs3_row(sec, 7, 64, cols.data(), vals.data(), &diag, &nnz) == QS3_OK && nnz > 0);
    CHECK(qs3_row(sec, dim, 64, cols.data(), vals.data(), &diag, &nnz) == QS3_EINVAL);
    // thick restart and plain Lanczos
    qs3_eigs_opts o{};
    o.alg = QS3_ALG_TRL;
    o.nev = 4;
    o.seed = 3;
    o.reorth = QS3_REORTH_FULL;
    double ev[4], ev2[4];
    qs3_eigs_info info{};
    double *vecs = (double *)dalloc(dim * 8 * 4);
    CHECK(qs3_eigs(sec, &o, ev, vecs, &info, s) == QS3_OK && info.converged == 1 && all_finite(ev, 4));
    o.alg = QS3_ALG_LANCZOS;
    o.steps = 100;
    CHECK(qs3_eigs(sec, &o, ev2, nullptr, &info, s) == QS3_OK && all_finite(ev2, 4));
    CHECK(std::fabs(ev[0] - ev2[0]) < 1e-9);
    // the restart limit forced from the host: QS3_ENOCONV with the current estimates
    o.alg = QS3_ALG_TRL;
    o.max_restarts = 1;
    o.tol = 1e-15;
    CHECK(qs3_eigs(sec, &o, ev2, nullptr, &info, s) == QS3_ENOCONV && info.converged == 0);
    std::vector<double> al(50), be(50);
    double nrm = 0;
    int done = 0;
    CHECK(qs3_lanczos(sec, nullptr, 50, QS3_PREC_F64, QS3_REORTH_PARTIAL, 5, al.data(), be.data(), &nrm, &done,
                      s) == QS3_OK && done > 0);
    HIPOK(hipMemsetAsync(w, 0, dim * 8, s));
    CHECK(qs3_lanczos(sec, w, 50, QS3_PREC_F64, QS3_REORTH_FULL, 5, al.data(), be.data(), &nrm, &done, s) ==
          QS3_ENUMERIC);
    // observables of the ground state
    std::vector<double> sz(16), zz(16), pm(32), szz(3), spm(3), st(3);
    CHECK(qs3_sz(sec, vecs, sz.data(), s) == QS3_OK && all_finite(sz.data(), 16));
    std::vector<int32_t> pi(16), pj(16);
    for (int i = 0; i < 16; ++i) {
        pi[i] = 0;
        pj[i] = i;
    }
    CHECK(qs3_sisj(sec, vecs, 16, pi.data(), pj.data(), zz.data(), pm.data(), s) == QS3_OK);
    CHECK(std::fabs(zz[0] - 0.25) < 1e-12);
    const double q[9] = {0, 0, 0, M_PI / 8, 0, 0, M_PI, 0, 0};
    CHECK(qs3_sq(sec, vecs, 3, q, szz.data(), spm.data(), st.data(), s) == QS3_OK && all_finite(st.data(), 3));
    // dense block, full diagonalisation and thermal averages
    std::vector<double> all(dim);
    CHECK(qs3_full_diag(sec, all.data(), nullptr, s) == QS3_OK);
    CHECK(std::fabs(all[0] - ev[0]) < 1e-9);
    std::vector<double> Sz(dim, 8.0 - 3.0), beta = {0.0, 0.5, 2.0}, lnZ(3), en(3), heat(3), mag(3), chi(3);
    CHECK(qs3_thermal(dim, all.data(), Sz.data(), 0.5, 3, beta.data(), lnZ.data(), en.data(), heat.data(),
                      mag.data(), chi.data()) == QS3_OK);
    CHECK(std::fabs(lnZ[0] - std::log((double)dim)) < 1e-9);
    HIPOK(hipFree(vecs));
    HIPOK(hipFree(v));
    HIPOK(hipFree(w));
    qs3_sector_destroy(sec);
    qs3_lattice_destroy(lat);
}

static void check_momentum(qs3_ctx *ctx, hipStream_t s) {
    Bonds b = hyper(6, 6, 1);
    qs3_lattice *lat = lattice(ctx, 6, 6, 1, b);
    const int32_t k1[3] = {1, 0, 0}, k0[3] = {0, 0, 0};
    qs3_sector *sec = nullptr, *gs = nullptr;
    CHECK(qs3_sector_create(lat, 3, k1, &sec) == QS3_OK);
    uint64_t dim = 0;
    CHECK(qs3_sector_dim(sec, &dim) == QS3_OK && dim > 0);
    std::vector<uint64_t> ranks(dim);
    std::vector<uint32_t> stab(dim);
    CHECK(qs3_sector_basis(sec, ranks.data(), stab.data()) == QS3_OK);
    for (uint64_t i = 1; i < dim; ++i) CHECK(ranks[i] > ranks[i - 1]);
    double *v = (double *)dalloc(dim * 16), *w = (double *)dalloc(dim * 16), *w2 = (double *)dalloc(dim * 16);
    CHECK(qs3_sector_start_vector(sec, 2, v, QS3_C128, s) == QS3_OK);
    CHECK(qs3_matvec(sec, v, w, QS3_C128, s) == QS3_OK);
    CHECK(qs3_matvec_noalloc(sec, v, w2, QS3_C128, s) == QS3_OK);
    std::vector<double> h1(2 * dim), h2(2 * dim);
    HIPOK(hipMemcpy(h1.data(), w, dim * 16, hipMemcpyDeviceToHost));
    HIPOK(hipMemcpy(h2.data(), w2, dim * 16, hipMemcpyDeviceToHost));
    CHECK(std::memcmp(h1.data(), h2.data(), dim * 16) == 0);
    qs3_eigs_opts o{};
    o.alg = QS3_ALG_TRL;
    o.nev = 3;
    o.seed = 1;
    o.reorth = QS3_REORTH_FULL;
    double ev[3];
    qs3_eigs_info info{};
    CHECK(qs3_eigs(sec, &o, ev, nullptr, &info, s) == QS3_OK && all_finite(ev, 3));
    // S(q, omega) from the k = 0 ground state into N_down = 4
    CHECK(qs3_sector_create(lat, 3, k0, &gs) == QS3_OK);
    uint64_t gdim = 0;
    qs3_sector_dim(gs, &gdim);
    double *g = (double *)dalloc(gdim * 16);
    double e0 = 0;
    o.nev = 1;
    CHECK(qs3_eigs(gs, &o, &e0, g, &info, s) == QS3_OK);
    const int32_t qv[6] = {1, 0, 0, 3, 3, 0};
    qs3_dsf_opts d{};
    d.steps = 40;
    d.eta = 0.1;
    d.field = 4.0;
    d.reorth = QS3_REORTH_FULL;
    std::vector<double> om(64), S(2 * 64), al(2 * 40), be(2 * 40), wt(2);
    for (int i = 0; i < 64; ++i) om[i] = 8.0 * i / 63;
    CHECK(qs3_dsf(gs, g, e0, 2, qv, &d, 64, om.data(), S.data(), al.data(), be.data(), wt.data(), s) == QS3_OK);
    CHECK(all_finite(S.data(), S.size()) && wt[0] > 0);
    d.op = QS3_OP_SZ;
    d.subtract_trivial = 1;
    CHECK(qs3_dsf(gs, g, e0, 2, qv, &d, 64, om.data(), S.data(), al.data(), be.data(), wt.data(), s) == QS3_OK);
    qs3_sector *to = nullptr;
    CHECK(qs3_sector_create(lat, 4, k1, &to) == QS3_OK);
    uint64_t tdim = 0;
    qs3_sector_dim(to, &tdim);
    double *t = (double *)dalloc(tdim * 16);
    const int32_t q1[3] = {1, 0, 0};
    CHECK(qs3_smq(gs, g, to, q1, t, s) == QS3_OK);
    CHECK(qs3_sq_apply(gs, g, to, QS3_OP_SPLUS, q1, t, s) == QS3_EINVAL);  // wrong N_down
    HIPOK(hipFree(t));
    qs3_sector_destroy(to);
    HIPOK(hipFree(g));
    HIPOK(hipFree(v));
    HIPOK(hipFree(w));
    HIPOK(hipFree(w2));
    qs3_sector_destroy(gs);
    qs3_sector_destroy(sec);
    // every momentum in one batch
    std::vector<int32_t> ks;
    for (int y = 0; y < 6; ++y)
        for (int x = 0; x < 6; ++x) {
            ks.push_back(x);
            ks.push_back(y);
            ks.push_back(0);
        }
    qs3_batch *bat = nullptr;
    CHECK(qs3_batch_create(lat, 3, 36, ks.data(), &bat) == QS3_OK);
    uint64_t rows = 0;
    std::vector<uint64_t> dims(36);
    CHECK(qs3_batch_dims(bat, &rows, dims.data()) == QS3_OK);
    double *bv = (double *)dalloc(rows * 36 * 16), *bw = (double *)dalloc(rows * 36 * 16);
    HIPOK(hipMemsetAsync(bv, 0, rows * 36 * 16, s));
    CHECK(qs3_batch_matvec(bat, bv, bw, QS3_C128, s) == QS3_OK);
    std::vector<double> bev(36);
    std::vector<qs3_eigs_info> binfo(36);
    o.nev = 1;
    CHECK(qs3_batch_eigs(bat, &o, bev.data(), binfo.data(), s) == QS3_OK && all_finite(bev.data(), 36));
    int G = 0, bpc = 0;
    CHECK(qs3_batch_schedule(bat, &G, &bpc) == QS3_OK && G > 0);
    {
        int ng = -1, gw = -1;
        CHECK(qs3_batch_groups(bat, &ng, &gw) == QS3_OK && ng >= 1 && gw >= 1);
        CHECK(qs3_batch_groups(nullptr, &ng, &gw) == QS3_EINVAL);
    }
    HIPOK(hipFree(bv));
    HIPOK(hipFree(bw));
    qs3_batch_destroy(bat);
    qs3_lattice_destroy(lat);
}

static void check_point_group(qs3_ctx *ctx, hipStream_t s) {
    // inversion of the periodic 8-site chain (r -> -r) with the even character
    Bonds b = hyper(8, 1, 1);
    qs3_lattice *lat = lattice(ctx, 8, 1, 1, b);
    std::vector<int32_t> perms(16), chars = {1, 1};
    for (int r = 0; r < 8; ++r) {
        perms[r] = r;
        perms[8 + r] = (8 - r) % 8;
    }
    const int32_t k0[3] = {0, 0, 0};
    qs3_pg_sector *pg = nullptr;
    CHECK(qs3_pg_sector_create(lat, 3, k0, 2, perms.data(), chars.data(), &pg) == QS3_OK);
    uint64_t dim = 0;
    CHECK(qs3_pg_sector_dim(pg, &dim) == QS3_OK && dim > 0);
    std::vector<int32_t> badp = perms;
    badp[8] = 1;  // not a permutation
    qs3_pg_sector *pg2 = nullptr;
    CHECK(qs3_pg_sector_create(lat, 3, k0, 2, badp.data(), chars.data(), &pg2) == QS3_EINVAL);
    double *v = (double *)dalloc(dim * 8), *w = (double *)dalloc(dim * 8);
    CHECK(qs3_pg_start_vector(pg, 1, v, s) == QS3_OK);
    CHECK(qs3_pg_matvec(pg, v, w, s) == QS3_OK);
    qs3_eigs_opts o{};
    o.alg = QS3_ALG_TRL;
    o.nev = 1;
    o.seed = 1;
    o.reorth = QS3_REORTH_FULL;
    double ev = 0;
    qs3_eigs_info info{};
    CHECK(qs3_pg_eigs(pg, &o, &ev, v, &info, s) == QS3_OK && std::isfinite(ev));
    qs3_sector *msec = nullptr;
    CHECK(qs3_sector_create(lat, 3, k0, &msec) == QS3_OK);
    uint64_t mdim = 0;
    qs3_sector_dim(msec, &mdim);
    double *m = (double *)dalloc(mdim * 16);
    CHECK(qs3_pg_to_momentum(pg, v, msec, m, s) == QS3_OK);
    HIPOK(hipFree(m));
    qs3_sector_destroy(msec);
    HIPOK(hipFree(v));
    HIPOK(hipFree(w));
    qs3_pg_sector_destroy(pg);
    qs3_lattice_destroy(lat);
}

static void check_server(qs3_ctx *ctx) {
    qs3_server_opts so{};
    so.max_active = 4;
    so.budget_bytes = 2ull << 30;
    qs3_server *srv = nullptr;
    CHECK(qs3_server_create(ctx, &so, &srv) == QS3_OK);
    std::vector<Bonds> keep;
    std::vector<uint64_t> tickets;
    struct Shape {
        int lx, ly, lz, K, use_k;
    };
    const Shape shapes[] = {{16, 1, 1, 2, 0}, {16, 1, 1, 3, 1}, {6, 6, 1, 2, 0}, {6, 6, 1, 3, 1},
                            {4, 4, 4, 2, 1},  {24, 1, 1, 4, 0}, {8, 8, 1, 3, 1}, {20, 1, 1, 1, 0},
                            {10, 10, 10, 4, 0} /* beyond the budget */};
    keep.reserve(16);
    for (const Shape &sh : shapes) {
        keep.push_back(hyper(sh.lx, sh.ly, sh.lz, 1.0, 0.5));
        const Bonds &b = keep.back();
        qs3_request r{};
        r.lx = sh.lx;
        r.ly = sh.ly;
        r.lz = sh.lz;
        r.n_bonds = b.n();
        r.bi = b.bi.data();
        r.bj = b.bj.data();
        r.jxy = b.jxy.data();
        r.jz = b.jz.data();
        r.n_down = sh.K;
        r.use_k = sh.use_k;
        r.nev = 3;
        r.seed = 7;
        uint64_t t = 0;
        CHECK(qs3_submit(srv, &r, &t) == QS3_OK);
        tickets.push_back(t);
    }
    // one more request, cancelled at once
    uint64_t tc = 0;
    {
        const Bonds &b = keep[2];
        qs3_request r{};
        r.lx = 6;
        r.ly = 6;
        r.lz = 1;
        r.n_bonds = b.n();
        r.bi = b.bi.data();
        r.bj = b.bj.data();
        r.jxy = b.jxy.data();
        r.jz = b.jz.data();
        r.n_down = 4;
        r.nev = 3;
        CHECK(qs3_submit(srv, &r, &tc) == QS3_OK);
        const int rc = qs3_cancel(srv, tc);
        CHECK(rc == QS3_OK || rc == QS3_EBUSY);
    }
    qs3_result res{};
    CHECK(qs3_poll(srv, 999999, &res) == QS3_ENOTFOUND);
    for (size_t i = 0; i < tickets.size(); ++i) {
        CHECK(qs3_wait(srv, tickets[i], &res) == QS3_OK);
        if (i + 1 < tickets.size()) {
            CHECK(res.status == QS3_OK && res.n_found >= 1 && all_finite(res.evals, res.n_found));
            CHECK(res.t_done >= res.t_start && res.t_start >= res.t_submit);
        } else {
            CHECK(res.status == QS3_ENOMEM);
        }
    }
    const int rc = qs3_wait(srv, tc, &res);
    CHECK(rc == QS3_OK && (res.status == QS3_ECANCELED || res.status == QS3_OK));
    CHECK(qs3_server_clock(srv) > 0);
    qs3_server_destroy(srv);
}

int main() {
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) {
        std::fprintf(stderr, "no GPU\n");
        return 2;
    }
    qs3_ctx *ctx = nullptr;
    CHECK(qs3_ctx_create(0, 0, &ctx) == QS3_OK);
    hipStream_t s;
    HIPOK(hipStreamCreate(&s));
    std::printf("errors\n");
    std::fflush(stdout);
    check_errors(ctx);
    std::printf("fixed N_down\n");
    std::fflush(stdout);
    check_u1(ctx, s);
    std::printf("momentum\n");
    std::fflush(stdout);
    check_momentum(ctx, s);
    CHECK(qs3_ctx_set_schedule(ctx, 1, 0) == QS3_OK);  // graph replay, fixed schedule
    check_momentum(ctx, s);
    CHECK(qs3_ctx_set_schedule(ctx, 0, 1) == QS3_OK);
    std::printf("point group\n");
    std::fflush(stdout);
    check_point_group(ctx, s);
    std::printf("server\n");
    std::fflush(stdout);
    check_server(ctx);
    HIPOK(hipStreamSynchronize(s));
    HIPOK(hipStreamDestroy(s));
    uint64_t used = 0, budget = 0;
    CHECK(qs3_ctx_memory(ctx, &used, &budget) == QS3_OK);
    CHECK(qs3_ctx_destroy(ctx) == QS3_OK);
    // every handle is destroyed: check for leaks now, then leave without the
    // runtime libraries' exit-time teardown, which the sanitizer's tracking of
    // device allocations does not survive (not this library's code)
    __lsan_do_leak_check();
    std::printf("host ABI check: %s (%d failed checks)\n", g_fail ? "FAILED" : "ok", g_fail);
    std::fflush(stdout);
    std::fflush(stderr);
    _exit(g_fail ? 1 : 0);
}
