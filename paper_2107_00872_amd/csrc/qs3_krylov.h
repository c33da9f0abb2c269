// Krylov engine interface (internal).
#pragma once
#include <algorithm>
#include <memory>
#include <vector>

#include "qs3_impl.h"

namespace qs3 {

struct Engine;
struct ThreeTerm;

// The operator a Lanczos run applies: n rows x B columns, [row][col] layout.
struct Operator {
    virtual ~Operator() = default;
    virtual uint64_t rows() const = 0;
    virtual int cols() const = 0;
    virtual bool is_complex() const = 0;
    virtual int apply(const double *x, double *y, hipStream_t s) = 0;        // float64 in/out
    virtual int apply_f32in(const float *x, double *y, hipStream_t s) = 0;  // float32 in, row sums float32
    // columns with mask[b] == 0 need not be computed (device mask or null)
    virtual void set_mask(const uint8_t *) {}
    // a whole cycle of steps x0..x1-1 in one workgroup; 1 = not supported
    virtual int small_cycle(Engine &, int, int, int) { return 1; }
    // the operator restricted to the listed columns (ascending); 1 = not supported
    virtual int subset(const std::vector<int> &, std::unique_ptr<Operator> *) { return 1; }
};

// Geometry of the deterministic column reductions: a block covers TC columns
// x TR rows, chunks of RC rows, partial sums per (chunk, column).
struct RedGeom {
    uint64_t n;
    int B;
    int TC, TR;
    uint64_t RC;
    int nchunk;
    int ncoltile;
};

// The engine's reorthogonalisation mode for an option value QS3_REORTH_*:
// 0 none, 2 full with the second pass where needed, 3 partial (plain Lanczos
// only; a restarted solve keeps full).
inline int engine_reorth(int opt, bool restarted) {
    if (opt == QS3_REORTH_NONE) return 0;
    return (opt == QS3_REORTH_PARTIAL && !restarted) ? 3 : 2;
}

struct Engine {
    qs3_ctx *ctx = nullptr;
    Operator *op = nullptr;
    hipStream_t st = 0;
    uint64_t n = 0, ne = 0, stride = 0;  // rows, elements (rows*B), doubles per vector
    int B = 1, dpe = 1, slots = 0, precision = 0, reorth = 2;
    bool cplx = false;
    int n_matvec = 0;
    const uint8_t *colmask = nullptr;  // device: columns still iterating (null = all)
    RedGeom rg{};
    DevBuf Psi, W, X32, partial, hvec, alpha, nrm2, ab_hist, act, om;
    ~Engine();
    int init(qs3_ctx *c, Operator *o, int slots, int precision, int reorth, hipStream_t s);
    double *slot(int j);
    int apply(const double *x, double *y);
    // out[j * B + b] = <X_j, Y'> (and |Y'|^2 at j = J when selfdot); re_out,
    // when given, also receives the real parts
    int multidot(const double *X, int J, const double *Y, double2 *out, int selfdot,
                 const uint8_t *mask, const ThreeTerm *f = nullptr, double *re_out = nullptr);
    // dgks_flag (optional): also flag the columns whose first pass cancelled
    // more than half of |W|^2 (dgks_before: |W|^2 before the pass)
    int cgs_update_norm(int J, const double2 *h, const uint8_t *mask, double2 *nrm_out,
                        const ThreeTerm *f = nullptr, const double2 *dgks_before = nullptr,
                        uint8_t *dgks_flag = nullptr);
    int step(int x, int prev);
    // steps x0..x1-1 (step x0's three-term partner is slot prev_first or none)
    int cycle(int x0, int x1, int prev_first);
    // the same, from a graph of the cycle's launches captured on its first
    // call and replayed afterwards (when the context allows graphs and the
    // stream can be captured); the launches of a cycle do not change between
    // the restarts of one engine
    int cycle_replay(int x0, int x1, int prev_first);
    hipGraphExec_t gexec = nullptr;
    int g_x0 = -1, g_x1 = -1, g_pf = -2;
    const uint8_t *g_mask = nullptr;
    int graph_launches = 0;
    int normalize_into_slot0(const double *v0, std::vector<double> *norms0);
    int read_ab(int x0, int x1, std::vector<double> &a, std::vector<double> &b);
    int rotate_dev(int from_slot, int NX, const double *dC, int NY, int to_slot, const uint8_t *act_dev);
    int copy_slot_dev(int from, int to, const uint8_t *act_dev);
    // dst slot to_slot, column j := this engine's slot from_slot, column idx[j]
    int gather_columns_into(Engine &dst, int from_slot, int to_slot, const int32_t *idx_dev);
    void release();
};

// A Lanczos / thick-restart Lanczos solve that advances without blocking:
// begin() enqueues the first cycle, ready() polls its event, advance() does
// the host part (tridiagonal / arrowhead eigensolves, convergence) and
// enqueues the next cycle.  Every column is a separate sector and stops
// changing once it has converged.  When no eigenvectors are wanted and at
// most three quarters of the columns still iterate, a thick restart moves them
// into a narrower engine (the operator restricted to those columns), so the
// slowest sectors no longer pay for the converged ones.
struct SolveRun {
    Engine root;                       // over all the operator's columns
    std::unique_ptr<Engine> narrow;    // after compaction: the columns still iterating
    std::unique_ptr<Operator> narrow_op;
    std::vector<int> cmap;             // column j of the narrow engine is column cmap[j]
    Engine &eng() { return narrow ? *narrow : root; }
    int col(int j) const { return cmap.empty() ? j : cmap[j]; }
    qs3_eigs_opts o{};
    int B = 1;
    bool want_vecs = false;
    int phase = 0;  // 1 first cycle, 2 restart cycle, 3 final rotation, 4 done
    int graph_prev = 0;  // graph replays of the engines before the current one
    bool first = true;
    int restarts = 0;
    double *hab = nullptr, *hC = nullptr;
    uint8_t *hact = nullptr;
    int32_t *hidx = nullptr;
    qs3_ctx *pctx = nullptr;  // the pool the host buffers return to
    size_t cap_hab = 0, cap_hC = 0, cap_hact = 0, cap_hidx = 0;
    DevBuf dC, dact, didx;
    hipEvent_t ev = nullptr;
    std::vector<std::vector<double>> al, be, coup;
    std::vector<uint8_t> active;
    std::vector<std::vector<int>> final_lv;
    std::vector<double> evals;
    std::vector<qs3_eigs_info> info;
    ~SolveRun();
    static int slots_for(const qs3_eigs_opts &o);
    int init(qs3_ctx *ctx, Operator *op, const qs3_eigs_opts &opts, hipStream_t s);
    int begin(const double *v0);
    bool ready() const;
    int wait();
    int advance(bool *done);
    int vec_slot(int col, int y) const;

   private:
    int enqueue_ab_copy(int x0, int x1);
    int compact(const uint8_t *keep, bool *compacted);
};

int solve_blocking(qs3_ctx *ctx, Operator *op, const qs3_eigs_opts &o, const double *v0, hipStream_t s,
                   std::vector<double> &evals, std::vector<qs3_eigs_info> &info, double *vec_out);

void sym_eig(int n, std::vector<double> &A, std::vector<double> &e, std::vector<double> &V);
int run_lanczos(Engine &E, const double *v0, int steps, std::vector<double> &a_out,
                std::vector<double> &b_out, std::vector<double> &norm0, std::vector<int> &done);

// ---- operators for the Krylov engine
int small_cycle_u1(qs3_sector *sec, Engine &E, int x0, int x1, int prev_first);
int small_cycle_batch(qs3_batch *bat, Engine &E, int x0, int x1, int prev_first);

struct U1Op : Operator {
    qs3_sector *sec;
    explicit U1Op(qs3_sector *s) : sec(s) {}
    int small_cycle(Engine &E, int x0, int x1, int pf) override { return small_cycle_u1(sec, E, x0, x1, pf); }
    uint64_t rows() const override { return sec->dim; }
    int cols() const override { return 1; }
    bool is_complex() const override { return false; }
    int apply(const double *x, double *y, hipStream_t s) override {
        return hv_u1(sec, x, QS3_F64, y, QS3_F64, s);
    }
    int apply_f32in(const float *x, double *y, hipStream_t s) override {
        return hv_u1(sec, x, QS3_F32, y, QS3_F64, s);
    }
};

struct BatchOp : Operator {
    qs3_batch *bat;
    explicit BatchOp(qs3_batch *b) : bat(b) {}
    uint64_t rows() const override { return bat->ks->n_reps; }
    int cols() const override { return bat->B; }
    bool is_complex() const override { return true; }
    const uint8_t *mask = nullptr;
    void set_mask(const uint8_t *m) override { mask = m; }
    int small_cycle(Engine &E, int x0, int x1, int pf) override {
        return bat->B == 1 ? small_cycle_batch(bat, E, x0, x1, pf) : 1;
    }
    int apply(const double *x, double *y, hipStream_t s) override {
        bat->active_dev = mask;
        int rc = hv_batch(bat, x, QS3_C128, y, QS3_C128, s);
        bat->active_dev = nullptr;
        return rc;
    }
    int apply_f32in(const float *x, double *y, hipStream_t s) override {
        bat->active_dev = mask;
        int rc = hv_batch(bat, x, QS3_C64, y, QS3_C128, s);
        bat->active_dev = nullptr;
        return rc;
    }
    int subset(const std::vector<int> &cols, std::unique_ptr<Operator> *out) override;
};

// default thick-restart sizes: N_K kept Ritz vectors, N_M Krylov vectors
inline int default_nk(int nev) { return std::max(nev + 5, 8); }
inline int default_nm(int nk) { return std::max(2 * nk, 24); }

inline int fill_opts(qs3_eigs_opts &o, uint64_t min_dim) {
    if (o.nev <= 0) o.nev = 1;
    if (o.nk <= 0) o.nk = default_nk(o.nev);
    if (o.nm <= 0) o.nm = default_nm(o.nk);
    if (o.max_restarts <= 0) o.max_restarts = 2000;
    if (o.steps <= 0) o.steps = 100;
    if (!(o.tol > 0)) o.tol = o.precision == QS3_PREC_F32MV ? 1e-6 : 1e-10;
    QS3_REQUIRE(o.nev <= 16, QS3_EINVAL, "nev must be <= 16");
    QS3_REQUIRE(o.precision == QS3_PREC_F64 || o.precision == QS3_PREC_F32MV, QS3_EINVAL,
                "unknown precision");
    QS3_REQUIRE(o.reorth >= QS3_REORTH_NONE && o.reorth <= QS3_REORTH_PARTIAL, QS3_EINVAL,
                "unknown reorthogonalisation mode");
    if (o.alg == QS3_ALG_TRL) {
        QS3_REQUIRE(o.reorth != QS3_REORTH_NONE, QS3_EINVAL, "thick restart needs reorthogonalisation");
        QS3_REQUIRE(o.nk > o.nev - 1 && o.nm > o.nk, QS3_EINVAL, "need nev <= nk < nm");
        if ((uint64_t)o.nm > min_dim) {
            // the Krylov space would exhaust the sector: plain Lanczos over it
            o.alg = QS3_ALG_LANCZOS;
            o.steps = (int)std::max<uint64_t>(min_dim, 1);
        }
    } else {
        QS3_REQUIRE(o.alg == QS3_ALG_LANCZOS, QS3_EINVAL, "unknown algorithm");
        if ((uint64_t)o.steps > min_dim) o.steps = (int)std::max<uint64_t>(min_dim, 1);
    }
    return QS3_OK;
}


int scatter_compact_f32(qs3_sector *sec, const float *src, float *dst_union, hipStream_t s);
int gather_compact_f32(qs3_sector *sec, const float *src_union, float *dst, hipStream_t s);

}  // namespace qs3
