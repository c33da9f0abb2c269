// Internal host-side structures of libqs3 (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/qs3.h"

namespace qs3 {

void set_error(const std::string &msg);

struct Status {
    int code;
};

#define QS3_HIP(call)                                                                    \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess) {                                                          \
            ::qs3::set_error(std::string("HIP error ") + hipGetErrorString(e_) + " at " + \
                             __FILE__ + ":" + std::to_string(__LINE__));                 \
            return QS3_EDEVICE;                                                          \
        }                                                                                \
    } while (0)

#define QS3_TRY(call)               \
    do {                            \
        int rc_ = (call);           \
        if (rc_ < 0) return rc_;    \
    } while (0)

#define QS3_REQUIRE(cond, code, msg) \
    do {                             \
        if (!(cond)) {               \
            ::qs3::set_error(msg);   \
            return (code);           \
        }                            \
    } while (0)

constexpr int MAX_K_U1 = 8;   // N_down of fixed-N_down sectors
constexpr int MAX_K_MOM = 6;  // N_down of momentum sectors
constexpr int MAX_SITES = 4096;

// A device allocation accounted against the context budget.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    qs3_ctx *ctx = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf();
    int alloc(qs3_ctx *c, size_t n);
    void release();
    template <typename T>
    T *as() const { return (T *)ptr; }
};

}  // namespace qs3

struct qs3_ctx {
    int device = 0;
    uint64_t budget = 0;
    std::atomic<uint64_t> used{0};
    int n_cu = 256;
    uint64_t table_limit = 16ull << 30;     // largest rank -> (rep, translation) table
    uint64_t hop_list_limit = 64ull << 30;  // largest per-representative hop lists
    std::mutex mu;
    void *blas = nullptr;  // rocBLAS handle, created on first use
    std::mutex blas_mu;    // held while a call is bound to the handle
    int use_graphs = 0;    // replay thick-restart cycles from captured graphs
    int autotune = 1;      // time the batched H.v's schedules once per width class
    // small pinned host buffers kept for reuse (power-of-two capacities): a
    // solve's host staging comes from here, not from hipHostMalloc and
    // hipHostFree per solve (tens of microseconds each)
    std::mutex pin_mu;
    std::multimap<size_t, void *> pin_pool;
    size_t pin_pool_bytes = 0;
    qs3_ctx() = default;
    qs3_ctx(const qs3_ctx &) = delete;
    qs3_ctx &operator=(const qs3_ctx &) = delete;
    ~qs3_ctx();
};

namespace qs3 {

// A pinned host buffer of at least `bytes` from the context's pool (or a new
// one); *cap is its capacity, to be handed back with pinned_put.
int pinned_get(qs3_ctx *c, size_t bytes, void **p, size_t *cap);
// Returns a buffer to the pool (freed instead beyond the pool's limit).  The
// caller must have finished every copy into or out of it.
void pinned_put(qs3_ctx *c, void *p, size_t cap);

// Binomial columns for one (N, K): see Binom<RT> in qs3_device.h.
struct BinomTable {
    int N = 0, K = 0;
    bool wide = false;  // uint64 entries
    uint64_t D = 0;     // C(N, K)
    DevBuf dev;
    std::vector<uint64_t> host;  // full table C(c, m), m = 0..K+1, row-major [c][m]
    uint64_t C(int c, int m) const {
        if (m < 0 || c < m) return 0;
        return host[(size_t)c * (K + 2) + m];
    }
};

// Translation structure of one (lattice, K): the union of representatives of
// every orbit (ascending ranks), stabiliser sizes, a directory for searches
// and optionally the rank -> (union index, translation) table.
struct KStructure {
    int K = 0;
    uint64_t n_reps = 0;
    DevBuf reps;   // uint64 [n_reps]
    DevBuf stab;   // uint16 [n_reps]
    DevBuf dir;    // uint32 [2^dir_bits + 1]
    int dir_shift = 0, dir_bits = 0;
    bool has_table = false;
    DevBuf table;  // uint64 [D]
    // otherwise optionally the resolved hops of every representative row
    bool has_hops = false;
    int hmax = 0;  // N_down * most neighbours of a site
    DevBuf hops;   // uint64 [n_reps * hmax]
    std::vector<uint64_t> h_reps;
    std::vector<uint16_t> h_stab;
    // non-trivial stabilisers: union index and its stabiliser translations
    std::vector<uint32_t> nt_u;
    std::vector<std::vector<int>> nt_trans;  // packed tx | ty<<10 | tz<<20
    DevBuf nt_of;  // int32 [n_reps]: index into nt_u or -1
    // the batched H.v's tuned schedule per (width class, element type, hop
    // store): lanes per row and blocks per CU (see hv_inst.hip)
    std::mutex tune_mu;
    std::map<uint32_t, std::pair<int, int>> tuned;
};

}  // namespace qs3

struct qs3_lattice {
    qs3_ctx *ctx = nullptr;
    int lx = 1, ly = 1, lz = 1, N = 0;
    int ns = 1;  // sites per unit cell: site = s + ns * (x + lx * (y + ly * z))
    std::vector<double> basis;  // ns x 3: place s in its cell, in cell-vector units (default 0)
    int n_bonds = 0;
    std::vector<int> bi, bj;
    std::vector<double> jxy, jz;
    bool translation_invariant = false;
    // adjacency (both directions), CSR over sites
    std::vector<int> h_ptr;
    std::vector<uint16_t> h_nbr;
    int max_degree = 0;    // most neighbours of a site
    bool regular = false;  // every site has max_degree neighbours
    std::vector<double> h_jxy_h, h_jz_h;  // Jxy/2, Jz/2 per directed edge
    bool uniform = false;
    double u_jxy_h = 0, u_jz_h = 0;
    double ez4 = 0;  // sum_b Jz_b / 4
    qs3::DevBuf d_ptr, d_nbr, d_jxy_h, d_jz_h, d_jxy_hf, d_jz_hf, d_jp_h, d_jp_hf, d_coords, d_sqrt;
    std::map<int, std::shared_ptr<qs3::BinomTable>> binoms;
    std::map<int, std::shared_ptr<qs3::KStructure>> kstructs;
    std::mutex mu;
};

namespace qs3 {

int get_binom(qs3_lattice *lat, int K, std::shared_ptr<BinomTable> *out);
int get_kstruct(qs3_lattice *lat, int K, std::shared_ptr<KStructure> *out, hipStream_t s);

// Device view of a lattice handed to kernels by value.
struct LatArgs {
    int N, lx, ly, lz;
    int ns;  // sites per unit cell (translations act on cells)
    const int *ptr;
    const uint16_t *nbr;
    const double *jxy_h, *jz_h;
    const float *jxy_hf, *jz_hf;
    const double2 *jp_h;  // per edge (J_xy/2, J_z/2): one load for both
    const float2 *jp_hf;
    int n_edges;
    int uniform;
    double u_jxy_h, u_jz_h, ez4;
    const uint32_t *coords;
    const double *sqrt_tab;  // sqrt(s), s = 0..N
};
LatArgs lat_args(const qs3_lattice *lat);

}  // namespace qs3

// A batch of momentum sectors of one (lattice, K) in the [row][sector] layout
// over the union of representatives.
struct qs3_batch {
    qs3_lattice *lat = nullptr;
    int K = 0;
    int B = 0;
    std::vector<int> kv;  // 3*B
    std::shared_ptr<qs3::KStructure> ks;
    std::shared_ptr<qs3::BinomTable> bt;
    int M = 1;                    // lcm of the lattice lengths
    qs3::DevBuf kmul;             // int32 [3*B]: K_a * (M / L_a) mod M
    qs3::DevBuf phase;            // double2 [M]: e^{2 pi i P / M}
    qs3::DevBuf compat_nt;        // uint8 [n_nt * B]
    // a batch of one sector on a lattice with one exchange constant: the
    // phase-table index P of e^{ik.t} per cell translation t = tx + lx (ty +
    // ly tz) (uint16 [N_T]), and where the structure has non-trivial
    // stabilisers the class of every representative in this sector (uint8
    // [n_reps]): its stabiliser size s when k is compatible with it (1 for a
    // trivial stabiliser), 0 when it is not in the sector; empty otherwise
    qs3::DevBuf tP, gcls;
    int last_G = 0, last_bpc = 0;  // schedule of the last batched H.v launch
    int last_groups = 0, last_group_width = 0;  // and its split into sector groups
    std::vector<uint8_t> h_compat_nt;
    std::vector<uint64_t> dims;   // per sector
    const uint8_t *active_dev = nullptr;  // device mask set by the solver while it applies H
};

struct qs3_sector {
    qs3_lattice *lat = nullptr;
    int K = 0;
    bool has_k = false;
    int kv[3] = {0, 0, 0};
    uint64_t dim = 0;
    std::shared_ptr<qs3::BinomTable> bt;
    qs3_batch *bat = nullptr;      // B = 1 batch for momentum sectors
    qs3::DevBuf comp2u;            // int64 [dim]: union index of basis state i
    qs3::DevBuf scratch_a, scratch_b;  // union-layout staging for the compact API
};

namespace qs3 {

// ---- kernels' launchers (hv.hip) ----
int hv_u1(qs3_sector *sec, const void *v, int vtype, void *w, int wtype, hipStream_t s);
// The context's rocBLAS handle (a rocblas_handle), created on first use and
// bound to stream s; the caller holds ctx->blas_mu.  Null on failure.
void *blas_on(qs3_ctx *ctx, hipStream_t s);
void blas_release(qs3_ctx *ctx);
int hv_batch(qs3_batch *bat, const void *v, int vtype, void *w, int wtype, hipStream_t s);
int row_u1(qs3_sector *sec, uint64_t row, int cap, int64_t *cols, double *vals, double *diag,
           int *nnz);
int row_k(qs3_sector *sec, uint64_t row, int cap, int64_t *cols, double *vals, double *diag,
          int *nnz);
int build_kstruct(qs3_lattice *lat, int K, KStructure *ks, hipStream_t s);

// ---- helpers (krylov.hip) ----
int start_vector_u1(qs3_sector *sec, uint64_t seed, void *v, int dtype, hipStream_t s);
int start_vector_batch(qs3_batch *bat, const uint64_t *seeds, double *v, hipStream_t s);
int scatter_compact(qs3_sector *sec, const double *src, double *dst_union, hipStream_t s);
// device address of the allocation-free matvec's scratch array on `device`
// (looked up once per device; the device must be current)
int noalloc_init(int device);
int gather_compact(qs3_sector *sec, const double *src_union, double *dst, hipStream_t s);

}  // namespace qs3
