// Kernel argument blocks and the per-N_down entry points of the H.v kernels
// (each N_down is instantiated in its own translation unit, hv_inst.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "qs3_impl.h"

namespace qs3 {

// How the batched kernel resolves a hop's target (representative index and
// translation): canonicalisation and a directory search per hop, a lookup in
// the rank -> (representative, translation) table, or the per-representative
// hop lists resolved once when the structure was built.
enum HopMode { HOP_FLY = 0, HOP_TABLE = 1, HOP_LISTS = 2 };

struct BatchArgs {
    LatArgs L;
    uint64_t n_reps;
    const uint64_t *reps;
    const uint16_t *stab;
    const int32_t *nt_of;
    const uint8_t *compat_nt;
    const uint64_t *table;
    const uint64_t *hops;  // [n_reps][hmax] hop lists, or null
    int hmax;
    const uint32_t *dir;
    int dir_shift;
    int B, G;
    int ld;  // row stride of v, w and compat_nt in sectors (B, or the whole batch for a group of its sectors)
    const int32_t *kmul;  // 3*B: K_a * (M / L_a) mod M
    int M;
    double invM;
    const double2 *phase;  // e^{2 pi i P / M}
    const uint8_t *active;  // per sector, or null: rows of inactive sectors are left untouched
    int ph_lds_off;         // byte offset of the phase table in dynamic LDS, or -1 (global)
    // a batch of one sector with uniform couplings: the phase index of e^{ik.t}
    // per cell translation, and the class of every representative in the
    // sector (stabiliser size, 0 outside it; null when every stabiliser is
    // trivial); both null otherwise
    const uint16_t *tP;
    const uint8_t *gcls;
};

struct BuildArgs {
    LatArgs L;
    uint64_t D;
    uint64_t chunk;  // ranks per block
};

struct SmallArgs {
    uint64_t n;         // rows (single column)
    int x0, x1;         // steps x0..x1-1
    int prev_first;     // slot of the three-term partner of step x0, or -1
    double *Psi;        // slots of `stride` doubles
    uint64_t stride;
    double *W;
    double *ab;         // alpha at [x], beta at [slots + x]
    int slots;
    int reorth;         // 0 none, 1 one pass, 2 second pass where needed
};

BatchArgs batch_args(qs3_batch *bat);
// One Lanczos cycle of a small single-column sector in one workgroup (bat =
// null: fixed-N_down sector).  Returns 1 when the size is not supported.
int lanczos_small(qs3_lattice *lat, int K, const BinomTable *bt, qs3_batch *bat, const SmallArgs &S,
                  hipStream_t s);
template <int K>
int lanczos_small_K(qs3_lattice *lat, const BinomTable *bt, qs3_batch *bat, const SmallArgs &S, hipStream_t s);
int grid_for(qs3_ctx *ctx, uint64_t tiles);
int grid_cover(qs3_ctx *ctx, uint64_t tiles);

template <int K>
int hv_u1_K(qs3_sector *sec, const void *v, int vtype, void *w, int wtype, hipStream_t s);
template <int K>
int row_u1_K(qs3_sector *sec, uint64_t row, int cap, int64_t *cols, double *vals, double *diag,
             int *nnz);
template <int K>
int hv_batch_K(qs3_batch *bat, const void *v, int vtype, void *w, int wtype, hipStream_t s);
template <int K>
int row_k_K(qs3_sector *sec, uint64_t u, int cap, int64_t *cols, double *vals, double *diag,
            int *nnz);
template <int K>
int build_kstruct_K(qs3_lattice *lat, const BinomTable &bt, KStructure *ks, hipStream_t s);
// Dense sector blocks, column major, added into A (zero on entry): fixed
// N_down (real) and momentum sectors (complex, u2c: union row -> basis index).
template <int K>
int dense_u1_K(qs3_sector *sec, double *A, hipStream_t s);
template <int K>
int dense_k_K(qs3_sector *sec, const int64_t *u2c, double *A, hipStream_t s);

}  // namespace qs3

namespace qs3 {

// Observables (obs_kernels.h), instantiated per N_down in hv_inst.hip.
// Fixed-N_down sector, real vector phi (device): p_site[i] = sum_{a ∋ i}
// |phi_a|^2; for pairs (pi, pj device, i != j): q[p] = sum_{a ∋ i, j} |phi_a|^2,
// pm[p] = sum_S phi(S+j) phi(S+i).  Host outputs.  hpi, hpj: the same pairs
// on the host with hpi < hpj, or null (then every pair runs its own subset
// loops; with them and at least N pairs, pm comes from one Gram matrix).
template <int K>
int obs_u1_K(qs3_sector *sec, const double *phi, int npairs, const int32_t *pi,
             const int32_t *pj, std::vector<double> &p_site, std::vector<double> &q,
             std::vector<double> &pm, hipStream_t s, const int32_t *hpi = nullptr,
             const int32_t *hpj = nullptr);
// Momentum sector in union layout: per displacement (packed, device) the sums
// zz (pair counts weighted by |phi|^2), nrm = |phi|^2 and pm (complex).
template <int K>
int corr_k_K(qs3_sector *sec, const double *phi_union, int ndisp, const int32_t *disp,
             std::vector<double> &zz, std::vector<double> &nrm, std::vector<double> &pm_re,
             std::vector<double> &pm_im, hipStream_t s);
// S^-_q gather from the source sector (batch of one, union layout) into the
// target batch (union layout [row][sector]); qmul: device, 3 ints per target;
// subph: device, e^{-i q.offset_s} per target and place in a cell.
// S^+_q (source K down spins, targets K - 1) and S^z_q (source and targets
// of one K-down structure), same conventions.
template <int K>
int spq_K(qs3_batch *src, qs3_batch *dst, const int32_t *qmul, const double2 *subph,
          const double *phi_union,
          double *out_union, hipStream_t s);
template <int K>
int szq_K(qs3_batch *src, qs3_batch *dst, const int32_t *qmul, const double2 *subph,
          const double *phi_union,
          double *out_union, hipStream_t s);
template <int K>
int smq_K(qs3_batch *src, qs3_batch *dst, const int32_t *qmul, const double2 *subph,
          const double *phi_union,
          double *out_union, hipStream_t s);

}  // namespace qs3
