// Krylov engine interface (internal).
#pragma once
#include <vector>

#include "qs3_impl.h"

namespace qs3 {

// The operator a Lanczos run applies: n rows x B columns, [row][col] layout.
struct Operator {
    virtual ~Operator() = default;
    virtual uint64_t rows() const = 0;
    virtual int cols() const = 0;
    virtual bool is_complex() const = 0;
    virtual int apply(const double *x, double *y, hipStream_t s) = 0;        // float64 in/out
    virtual int apply_f32in(const float *x, double *y, hipStream_t s) = 0;  // float32 in, row sums float32
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

struct Engine {
    qs3_ctx *ctx = nullptr;
    Operator *op = nullptr;
    hipStream_t st = 0;
    uint64_t n = 0, ne = 0, stride = 0;  // rows, elements (rows*B), doubles per vector
    int B = 1, dpe = 1, slots = 0, precision = 0, reorth = 2;
    bool cplx = false;
    int n_matvec = 0;
    RedGeom rg{};
    DevBuf Psi, W, X32, partial, hvec, alpha, nrm2, ab_hist, act;
    ~Engine();
    int init(qs3_ctx *c, Operator *o, int slots, int precision, int reorth, hipStream_t s);
    double *slot(int j);
    int apply(const double *x, double *y);
    int multidot(const double *X, int J, const double *Y, double2 *out, int selfdot,
                 const uint8_t *mask);
    int cgs_update_norm(int J, const double2 *h, const uint8_t *mask, double2 *nrm_out);
    int step(int x, int prev);
    int normalize_into_slot0(const double *v0, std::vector<double> *norms0);
    int read_ab(int x0, int x1, std::vector<double> &a, std::vector<double> &b);
    int rotate(int from_slot, int NX, const std::vector<double> &Cm, int NY, int to_slot,
               const uint8_t *active_host);
    int copy_slot(int from, int to, const uint8_t *active_host);
};

void jacobi_eig(int n, std::vector<double> &A, std::vector<double> &e, std::vector<double> &V);
int run_lanczos(Engine &E, const double *v0, int steps, std::vector<double> &a_out,
                std::vector<double> &b_out, std::vector<double> &norm0, std::vector<int> &done);
int solve_lanczos(Engine &E, const double *v0, const qs3_eigs_opts &o, std::vector<double> &evals,
                  std::vector<qs3_eigs_info> &info, int want_vecs, double *vec_out);
int solve_trl(Engine &E, const double *v0, const qs3_eigs_opts &o, std::vector<double> &evals,
              std::vector<qs3_eigs_info> &info, int want_vecs, double *vec_out);

int scatter_compact_f32(qs3_sector *sec, const float *src, float *dst_union, hipStream_t s);
int gather_compact_f32(qs3_sector *sec, const float *src_union, float *dst, hipStream_t s);

}  // namespace qs3
