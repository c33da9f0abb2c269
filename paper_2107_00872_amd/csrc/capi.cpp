// C ABI of libqs3: contexts, lattices, sectors, batches, matvec and the
// eigensolver entry points.  Observables are in obs.hip, serving in server.cpp.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <numeric>
#include <unordered_map>

#include "qs3_device.h"
#include "qs3_impl.h"
#include "qs3_krylov.h"

namespace qs3 {

static thread_local std::string g_last_error;
void set_error(const std::string &msg) { g_last_error = msg; }

DevBuf::~DevBuf() { release(); }

// pinned host buffers up to 16 MB are pooled, up to 64 MB in all
static constexpr size_t PIN_POOL_MAX_BUF = 16u << 20, PIN_POOL_MAX = 64u << 20;

int pinned_get(qs3_ctx *c, size_t bytes, void **p, size_t *cap) {
    size_t k = std::max<size_t>(bytes, 1);
    if (k <= PIN_POOL_MAX_BUF) {
        size_t q = 4096;
        while (q < k) q <<= 1;
        k = q;
        std::lock_guard<std::mutex> lk(c->pin_mu);
        auto it = c->pin_pool.find(k);
        if (it != c->pin_pool.end()) {
            *p = it->second;
            *cap = k;
            c->pin_pool_bytes -= k;
            c->pin_pool.erase(it);
            return QS3_OK;
        }
    }
    void *q = nullptr;
    QS3_HIP(hipHostMalloc(&q, k, hipHostMallocDefault));
    *p = q;
    *cap = k;
    return QS3_OK;
}

void pinned_put(qs3_ctx *c, void *p, size_t cap) {
    if (!p) return;
    if (cap <= PIN_POOL_MAX_BUF) {
        std::lock_guard<std::mutex> lk(c->pin_mu);
        if (c->pin_pool_bytes + cap <= PIN_POOL_MAX) {
            c->pin_pool.emplace(cap, p);
            c->pin_pool_bytes += cap;
            return;
        }
    }
    (void)hipHostFree(p);
}

int DevBuf::alloc(qs3_ctx *c, size_t n) {
    release();
    ctx = c;
    if (n == 0) n = 16;
    uint64_t prev = c->used.fetch_add(n);
    if (prev + n > c->budget) {
        c->used.fetch_sub(n);
        set_error("device memory budget exceeded (" + std::to_string(prev + n) + " > " +
                  std::to_string(c->budget) + " bytes)");
        return QS3_ENOMEM;
    }
    hipError_t e = hipMalloc(&ptr, n);
    if (e != hipSuccess) {
        c->used.fetch_sub(n);
        ptr = nullptr;
        set_error(std::string("hipMalloc failed: ") + hipGetErrorString(e));
        return QS3_ENOMEM;
    }
    bytes = n;
    return QS3_OK;
}

void DevBuf::release() {
    if (ptr) {
        (void)hipFree(ptr);
        ctx->used.fetch_sub(bytes);
    }
    ptr = nullptr;
    bytes = 0;
}

struct DeviceGuard {
    explicit DeviceGuard(int dev) { (void)hipSetDevice(dev); }
};

// ---- binomial tables
int get_binom(qs3_lattice *lat, int K, std::shared_ptr<BinomTable> *out) {
    std::lock_guard<std::mutex> lk(lat->mu);
    auto it = lat->binoms.find(K);
    if (it != lat->binoms.end()) {
        *out = it->second;
        return QS3_OK;
    }
    auto bt = std::make_shared<BinomTable>();
    bt->N = lat->N;
    bt->K = K;
    const int N = lat->N;
    bt->host.assign((size_t)(N + 1) * (K + 2), 0);
    for (int c = 0; c <= N; ++c) {
        for (int m = 0; m <= K + 1; ++m) {
            uint64_t v;
            if (m == 0) v = 1;
            else if (c < m) v = 0;
            else {
                uint64_t a = bt->host[(size_t)(c - 1) * (K + 2) + m - 1];
                uint64_t b = bt->host[(size_t)(c - 1) * (K + 2) + m];
                v = a + b;
                if (v < a) v = UINT64_MAX;  // saturate: only reached for m = K+1 beyond range
            }
            bt->host[(size_t)c * (K + 2) + m] = v;
        }
    }
    bt->D = bt->C(N, K);
    QS3_REQUIRE(bt->D < (1ull << 62), QS3_EINVAL, "sector dimension exceeds 2^62");
    bt->wide = bt->D >= (1ull << 32);
    // device columns m = 2..K of C(c, m), c = 0..N, column m at (m - 2) << sh
    const int ncol = std::max(K - 1, 0);
    const size_t esz = bt->wide ? 8 : 4;
    const size_t stride = (size_t)1 << binom_shift(N);
    QS3_TRY(bt->dev.alloc(lat->ctx, std::max<size_t>(esz * ncol * stride, 16)));
    if (ncol) {
        std::vector<unsigned char> buf(esz * ncol * stride, 0);
        for (int m = 2; m <= K; ++m)
            for (int c = 0; c <= N; ++c) {
                uint64_t v = bt->C(c, m);
                if (v > bt->D) v = bt->D;  // only entries above C(N, K) are never looked up usefully
                if (bt->wide) ((uint64_t *)buf.data())[(size_t)(m - 2) * stride + c] = v;
                else ((uint32_t *)buf.data())[(size_t)(m - 2) * stride + c] = (uint32_t)v;
            }
        QS3_HIP(hipMemcpy(bt->dev.ptr, buf.data(), buf.size(), hipMemcpyHostToDevice));
    }
    lat->binoms[K] = bt;
    *out = bt;
    return QS3_OK;
}

// host-side unrank (0-based) used for the few states handled on the host
static void host_unrank(const BinomTable &bt, uint64_t r, int K, int *c) {
    int hi = bt.N - 1;
    for (int m = K; m >= 2; --m) {
        int lo = m - 1, h = hi;
        while (lo < h) {
            int mid = (lo + h + 1) / 2;
            if (bt.C(mid, m) <= r) lo = mid; else h = mid - 1;
        }
        c[m - 1] = lo;
        r -= bt.C(lo, m);
        hi = lo - 1;
    }
    if (K >= 1) c[0] = (int)r;
}

int get_kstruct(qs3_lattice *lat, int K, std::shared_ptr<KStructure> *out, hipStream_t s) {
    {
        std::lock_guard<std::mutex> lk(lat->mu);
        auto it = lat->kstructs.find(K);
        if (it != lat->kstructs.end()) {
            *out = it->second;
            return QS3_OK;
        }
    }
    auto ks = std::make_shared<KStructure>();
    QS3_TRY(build_kstruct(lat, K, ks.get(), s));
    std::shared_ptr<BinomTable> bt;
    QS3_TRY(get_binom(lat, K, &bt));
    // non-trivial stabilisers: enumerate their translations on the host
    std::vector<int32_t> nt_of(ks->n_reps, -1);
    std::vector<int> c(K + 1), img(K + 1);
    for (uint64_t u = 0; u < ks->n_reps; ++u) {
        if (ks->h_stab[u] <= 1) continue;
        nt_of[u] = (int32_t)ks->nt_u.size();
        ks->nt_u.push_back((uint32_t)u);
        host_unrank(*bt, ks->h_reps[u], K, c.data());
        std::vector<int> trans;
        for (int tz = 0; tz < lat->lz; ++tz)
            for (int ty = 0; ty < lat->ly; ++ty)
                for (int tx = 0; tx < lat->lx; ++tx) {
                    for (int m = 0; m < K; ++m) {
                        const int ns = lat->ns, sub = c[m] % ns, cell = c[m] / ns;
                        const int x = cell % lat->lx, y = (cell / lat->lx) % lat->ly, z = cell / (lat->lx * lat->ly);
                        img[m] = sub + ns * ((x + tx) % lat->lx +
                                             lat->lx * (((y + ty) % lat->ly) + lat->ly * ((z + tz) % lat->lz)));
                    }
                    std::sort(img.begin(), img.begin() + K);
                    if (std::equal(img.begin(), img.begin() + K, c.begin()))
                        trans.push_back(tx | (ty << 10) | (tz << 20));
                }
        if ((int)trans.size() != ks->h_stab[u]) {
            set_error("internal: stabiliser size mismatch");
            return QS3_EDEVICE;
        }
        ks->nt_trans.push_back(trans);
    }
    QS3_TRY(ks->nt_of.alloc(lat->ctx, sizeof(int32_t) * std::max<uint64_t>(ks->n_reps, 1)));
    if (ks->n_reps)
        QS3_HIP(hipMemcpy(ks->nt_of.ptr, nt_of.data(), sizeof(int32_t) * ks->n_reps, hipMemcpyHostToDevice));
    std::lock_guard<std::mutex> lk(lat->mu);
    lat->kstructs[K] = ks;
    *out = ks;
    return QS3_OK;
}

}  // namespace qs3

using namespace qs3;

// =====================================================================================
extern "C" {

const char *qs3_version(void) { return "qs3-mi355x 0.1 (gfx950)"; }

const char *qs3_strerror(int code) {
    switch (code) {
        case QS3_OK: return "ok";
        case QS3_EINVAL: return "invalid argument";
        case QS3_ENOMEM: return "out of device memory budget";
        case QS3_ENOCONV: return "not converged";
        case QS3_ENUMERIC: return "numerical failure";
        case QS3_EDEVICE: return "device error";
        case QS3_EBUSY: return "busy";
        case QS3_ENOTFOUND: return "not found";
        case QS3_ECANCELED: return "canceled";
        default: return "unknown error";
    }
}

const char *qs3_last_error(void) { return g_last_error.c_str(); }

int qs3_ctx_create(int device, uint64_t hbm_budget_bytes, qs3_ctx **out) {
    QS3_REQUIRE(out, QS3_EINVAL, "out is NULL");
    int ndev = 0;
    QS3_HIP(hipGetDeviceCount(&ndev));
    QS3_REQUIRE(device >= 0 && device < ndev, QS3_EINVAL, "no such device");
    QS3_HIP(hipSetDevice(device));
    size_t fr = 0, tot = 0;
    QS3_HIP(hipMemGetInfo(&fr, &tot));
    hipDeviceProp_t prop;
    QS3_HIP(hipGetDeviceProperties(&prop, device));
    QS3_TRY(qs3::noalloc_init(device));
    auto *c = new qs3_ctx();
    c->device = device;
    c->budget = hbm_budget_bytes ? hbm_budget_bytes : (uint64_t)(0.9 * fr);
    c->n_cu = prop.multiProcessorCount;
    *out = c;
    return QS3_OK;
}

qs3_ctx::~qs3_ctx() {
    for (auto &e : pin_pool) (void)hipHostFree(e.second);
}

int qs3_ctx_destroy(qs3_ctx *ctx) {
    if (ctx) qs3::blas_release(ctx);
    delete ctx;
    return QS3_OK;
}

int qs3_ctx_set_schedule(qs3_ctx *ctx, int use_graphs, int autotune) {
    QS3_REQUIRE(ctx, QS3_EINVAL, "ctx is NULL");
    ctx->use_graphs = use_graphs ? 1 : 0;
    ctx->autotune = autotune ? 1 : 0;
    return QS3_OK;
}

int qs3_ctx_set_structure_limits(qs3_ctx *ctx, uint64_t table_max_bytes, uint64_t hop_list_max_bytes) {
    QS3_REQUIRE(ctx, QS3_EINVAL, "ctx is NULL");
    ctx->table_limit = table_max_bytes;
    ctx->hop_list_limit = hop_list_max_bytes;
    return QS3_OK;
}

int qs3_ctx_memory(const qs3_ctx *ctx, uint64_t *used, uint64_t *budget) {
    QS3_REQUIRE(ctx, QS3_EINVAL, "ctx is NULL");
    if (used) *used = ctx->used.load();
    if (budget) *budget = ctx->budget;
    return QS3_OK;
}

int qs3_lattice_create(qs3_ctx *ctx, int lx, int ly, int lz, int n_bonds, const int32_t *bi,
                       const int32_t *bj, const double *jxy, const double *jz, qs3_lattice **out) {
    return qs3_lattice_create_cells(ctx, 1, lx, ly, lz, n_bonds, bi, bj, jxy, jz, out);
}

int qs3_lattice_create_cells(qs3_ctx *ctx, int n_sub, int lx, int ly, int lz, int n_bonds, const int32_t *bi,
                             const int32_t *bj, const double *jxy, const double *jz, qs3_lattice **out) {
    QS3_REQUIRE(ctx && out, QS3_EINVAL, "NULL argument");
    QS3_REQUIRE(lx >= 1 && ly >= 1 && lz >= 1 && lx < 1024 && ly < 1024 && lz < 1024, QS3_EINVAL,
                "lattice lengths must be in [1, 1023]");
    QS3_REQUIRE(n_sub >= 1 && n_sub <= 4, QS3_EINVAL, "sites per unit cell must be in [1, 4]");
    const int ns = n_sub;
    const long N = (long)ns * lx * ly * lz;
    QS3_REQUIRE(N <= MAX_SITES, QS3_EINVAL, "at most 4096 sites");
    QS3_REQUIRE(n_bonds >= 0 && (n_bonds == 0 || (bi && bj && jxy && jz)), QS3_EINVAL, "bad bonds");
    DeviceGuard dg(ctx->device);
    auto lat = std::make_unique<qs3_lattice>();
    lat->ctx = ctx;
    lat->lx = lx;
    lat->ly = ly;
    lat->lz = lz;
    lat->ns = ns;
    lat->basis.assign(3 * (size_t)ns, 0.0);
    lat->N = (int)N;
    lat->n_bonds = n_bonds;
    std::vector<std::vector<int>> adj(N);
    for (int b = 0; b < n_bonds; ++b) {
        int i = bi[b], j = bj[b];
        QS3_REQUIRE(i >= 0 && i < N && j >= 0 && j < N, QS3_EINVAL, "bond site out of range");
        QS3_REQUIRE(i != j, QS3_EINVAL, "bond with i == j");
        QS3_REQUIRE(std::isfinite(jxy[b]) && std::isfinite(jz[b]), QS3_EINVAL, "non-finite coupling");
        if (i > j) std::swap(i, j);
        lat->bi.push_back(i);
        lat->bj.push_back(j);
        lat->jxy.push_back(jxy[b]);
        lat->jz.push_back(jz[b]);
        lat->ez4 += jz[b] / 4.0;
    }
    // directed adjacency (both ends), bonds in order
    std::vector<std::vector<std::pair<int, int>>> nb(N);
    for (int b = 0; b < n_bonds; ++b) {
        nb[lat->bi[b]].push_back({lat->bj[b], b});
        nb[lat->bj[b]].push_back({lat->bi[b], b});
    }
    lat->h_ptr.assign(N + 1, 0);
    for (long s = 0; s < N; ++s) {
        lat->h_ptr[s + 1] = lat->h_ptr[s] + (int)nb[s].size();
        lat->max_degree = std::max(lat->max_degree, (int)nb[s].size());
        for (auto &pr : nb[s]) {
            lat->h_nbr.push_back((uint16_t)pr.first);
            lat->h_jxy_h.push_back(lat->jxy[pr.second] / 2.0);
            lat->h_jz_h.push_back(lat->jz[pr.second] / 2.0);
        }
    }
    lat->regular = N > 0;
    for (long s = 0; s < N; ++s)
        if ((int)nb[s].size() != lat->max_degree) lat->regular = false;
    lat->uniform = n_bonds > 0;
    for (int b = 1; b < n_bonds; ++b)
        if (lat->jxy[b] != lat->jxy[0] || lat->jz[b] != lat->jz[0]) lat->uniform = false;
    if (n_bonds > 0) {
        lat->u_jxy_h = lat->jxy[0] / 2.0;
        lat->u_jz_h = lat->jz[0] / 2.0;
    }
    // translation invariance: the bond multiset with couplings is mapped onto
    // itself by the unit translation along every axis
    {
        auto key = [](int i, int j) { return ((uint64_t)std::min(i, j) << 32) | (uint64_t)std::max(i, j); };
        std::unordered_map<uint64_t, std::pair<double, double>> bonds;
        for (int b = 0; b < n_bonds; ++b) {
            auto &v = bonds[key(lat->bi[b], lat->bj[b])];
            v.first += lat->jxy[b];
            v.second += lat->jz[b];
        }
        bool inv = true;
        auto tr = [&](int s, int ax) {
            const int sub = s % ns, cell = s / ns;
            int x = cell % lx, y = (cell / lx) % ly, z = cell / (lx * ly);
            if (ax == 0) x = (x + 1) % lx;
            if (ax == 1) y = (y + 1) % ly;
            if (ax == 2) z = (z + 1) % lz;
            return sub + ns * (x + lx * (y + ly * z));
        };
        for (int ax = 0; ax < 3 && inv; ++ax) {
            for (auto &kv : bonds) {
                int i = (int)(kv.first >> 32), j = (int)(kv.first & 0xffffffffu);
                auto it = bonds.find(key(tr(i, ax), tr(j, ax)));
                if (it == bonds.end() || std::fabs(it->second.first - kv.second.first) > 1e-14 ||
                    std::fabs(it->second.second - kv.second.second) > 1e-14) {
                    inv = false;
                    break;
                }
            }
        }
        lat->translation_invariant = inv;
    }
    std::vector<uint32_t> coords(N);
    for (long s = 0; s < N; ++s) {
        const long cell = s / ns;
        uint32_t x = cell % lx, y = (cell / lx) % ly, z = cell / (lx * ly), sub = (uint32_t)(s % ns);
        coords[s] = x | (y << 10) | (z << 20) | (sub << 30);
    }
    std::vector<double> sq(N + 1);
    for (long s = 0; s <= N; ++s) sq[s] = std::sqrt((double)s);
    std::vector<float> jxyf(lat->h_jxy_h.begin(), lat->h_jxy_h.end()), jzf(lat->h_jz_h.begin(), lat->h_jz_h.end());
    const size_t ne = std::max<size_t>(lat->h_nbr.size(), 1);
    QS3_TRY(lat->d_ptr.alloc(ctx, sizeof(int) * (N + 1)));
    QS3_TRY(lat->d_nbr.alloc(ctx, sizeof(uint16_t) * ne));
    QS3_TRY(lat->d_jxy_h.alloc(ctx, sizeof(double) * ne));
    QS3_TRY(lat->d_jz_h.alloc(ctx, sizeof(double) * ne));
    QS3_TRY(lat->d_jxy_hf.alloc(ctx, sizeof(float) * ne));
    QS3_TRY(lat->d_jp_h.alloc(ctx, sizeof(double) * 2 * ne));
    QS3_TRY(lat->d_jp_hf.alloc(ctx, sizeof(float) * 2 * ne));
    QS3_TRY(lat->d_jz_hf.alloc(ctx, sizeof(float) * ne));
    QS3_TRY(lat->d_coords.alloc(ctx, sizeof(uint32_t) * N));
    QS3_TRY(lat->d_sqrt.alloc(ctx, sizeof(double) * (N + 1)));
    QS3_HIP(hipMemcpy(lat->d_ptr.ptr, lat->h_ptr.data(), sizeof(int) * (N + 1), hipMemcpyHostToDevice));
    if (!lat->h_nbr.empty()) {
        QS3_HIP(hipMemcpy(lat->d_nbr.ptr, lat->h_nbr.data(), sizeof(uint16_t) * lat->h_nbr.size(), hipMemcpyHostToDevice));
        QS3_HIP(hipMemcpy(lat->d_jxy_h.ptr, lat->h_jxy_h.data(), sizeof(double) * lat->h_nbr.size(), hipMemcpyHostToDevice));
        QS3_HIP(hipMemcpy(lat->d_jz_h.ptr, lat->h_jz_h.data(), sizeof(double) * lat->h_nbr.size(), hipMemcpyHostToDevice));
        QS3_HIP(hipMemcpy(lat->d_jxy_hf.ptr, jxyf.data(), sizeof(float) * lat->h_nbr.size(), hipMemcpyHostToDevice));
        std::vector<double> jp(2 * lat->h_nbr.size());
        std::vector<float> jpf(2 * lat->h_nbr.size());
        for (size_t e = 0; e < lat->h_nbr.size(); ++e) {
            jp[2 * e] = lat->h_jxy_h[e];
            jp[2 * e + 1] = lat->h_jz_h[e];
            jpf[2 * e] = jxyf[e];
            jpf[2 * e + 1] = jzf[e];
        }
        QS3_HIP(hipMemcpy(lat->d_jp_h.ptr, jp.data(), sizeof(double) * jp.size(), hipMemcpyHostToDevice));
        QS3_HIP(hipMemcpy(lat->d_jp_hf.ptr, jpf.data(), sizeof(float) * jpf.size(), hipMemcpyHostToDevice));
        QS3_HIP(hipMemcpy(lat->d_jz_hf.ptr, jzf.data(), sizeof(float) * lat->h_nbr.size(), hipMemcpyHostToDevice));
    }
    QS3_HIP(hipMemcpy(lat->d_coords.ptr, coords.data(), sizeof(uint32_t) * N, hipMemcpyHostToDevice));
    QS3_HIP(hipMemcpy(lat->d_sqrt.ptr, sq.data(), sizeof(double) * (N + 1), hipMemcpyHostToDevice));
    *out = lat.release();
    return QS3_OK;
}

int qs3_lattice_destroy(qs3_lattice *lat) {
    if (lat) {
        DeviceGuard dg(lat->ctx->device);
        delete lat;
    }
    return QS3_OK;
}

int qs3_lattice_set_basis(qs3_lattice *lat, const double *offsets) {
    QS3_REQUIRE(lat && offsets, QS3_EINVAL, "NULL argument");
    for (int i = 0; i < 3 * lat->ns; ++i) QS3_REQUIRE(std::isfinite(offsets[i]), QS3_EINVAL, "non-finite offset");
    lat->basis.assign(offsets, offsets + 3 * lat->ns);
    return QS3_OK;
}

int qs3_lattice_info(const qs3_lattice *lat, int *n_sites, int *ti) {
    QS3_REQUIRE(lat, QS3_EINVAL, "lattice is NULL");
    if (n_sites) *n_sites = lat->N;
    if (ti) *ti = lat->translation_invariant ? 1 : 0;
    return QS3_OK;
}

// ---------------------------------------------------------------- batches
static int gcd_i(int a, int b) { return b ? gcd_i(b, a % b) : a; }

int qs3_batch_create(qs3_lattice *lat, int n_down, int n_sectors, const int32_t *kvecs,
                     qs3_batch **out) {
    QS3_REQUIRE(lat && out && kvecs, QS3_EINVAL, "NULL argument");
    QS3_REQUIRE(lat->translation_invariant, QS3_EINVAL,
                "momentum sectors need a translation-invariant bond set");
    QS3_REQUIRE(n_down >= 0 && n_down <= std::min(lat->N, MAX_K_MOM), QS3_EINVAL,
                "n_down out of range for momentum sectors");
    QS3_REQUIRE(n_sectors >= 1 && n_sectors <= 2048, QS3_EINVAL, "1..2048 sectors per batch");
    for (int b = 0; b < n_sectors; ++b) {
        QS3_REQUIRE(kvecs[3 * b] >= 0 && kvecs[3 * b] < lat->lx && kvecs[3 * b + 1] >= 0 &&
                        kvecs[3 * b + 1] < lat->ly && kvecs[3 * b + 2] >= 0 && kvecs[3 * b + 2] < lat->lz,
                    QS3_EINVAL, "momentum index out of range");
    }
    DeviceGuard dg(lat->ctx->device);
    auto bat = std::make_unique<qs3_batch>();
    bat->lat = lat;
    bat->K = n_down;
    bat->B = n_sectors;
    bat->kv.assign(kvecs, kvecs + 3 * n_sectors);
    QS3_TRY(get_binom(lat, n_down, &bat->bt));
    QS3_TRY(get_kstruct(lat, n_down, &bat->ks, 0));
    int M = lat->lx;
    M = M / gcd_i(M, lat->ly) * lat->ly;
    M = M / gcd_i(M, lat->lz) * lat->lz;
    bat->M = M;
    std::vector<int32_t> kmul(3 * n_sectors);
    for (int b = 0; b < n_sectors; ++b) {
        kmul[3 * b] = (int)((long)kvecs[3 * b] * (M / lat->lx) % M);
        kmul[3 * b + 1] = (int)((long)kvecs[3 * b + 1] * (M / lat->ly) % M);
        kmul[3 * b + 2] = (int)((long)kvecs[3 * b + 2] * (M / lat->lz) % M);
    }
    std::vector<double> ph(2 * M);
    for (int p = 0; p < M; ++p) {
        ph[2 * p] = std::cos(2.0 * M_PI * p / M);
        ph[2 * p + 1] = std::sin(2.0 * M_PI * p / M);
    }
    // compatibility of the representatives with non-trivial stabilisers
    const size_t nnt = bat->ks->nt_u.size();
    bat->h_compat_nt.assign(std::max<size_t>(nnt * n_sectors, 1), 1);
    bat->dims.assign(n_sectors, bat->ks->n_reps);
    for (size_t q = 0; q < nnt; ++q) {
        for (int b = 0; b < n_sectors; ++b) {
            bool ok = true;
            for (int t : bat->ks->nt_trans[q]) {
                int tx = t & 1023, ty = (t >> 10) & 1023, tz = (t >> 20) & 1023;
                long P = (long)kmul[3 * b] * tx + (long)kmul[3 * b + 1] * ty + (long)kmul[3 * b + 2] * tz;
                if (P % M != 0) {
                    ok = false;
                    break;
                }
            }
            bat->h_compat_nt[q * n_sectors + b] = ok ? 1 : 0;
            if (!ok) bat->dims[b] -= 1;
        }
    }
    qs3_ctx *ctx = lat->ctx;
    QS3_TRY(bat->kmul.alloc(ctx, sizeof(int32_t) * kmul.size()));
    QS3_TRY(bat->phase.alloc(ctx, sizeof(double) * ph.size()));
    QS3_TRY(bat->compat_nt.alloc(ctx, bat->h_compat_nt.size()));
    QS3_HIP(hipMemcpy(bat->kmul.ptr, kmul.data(), sizeof(int32_t) * kmul.size(), hipMemcpyHostToDevice));
    QS3_HIP(hipMemcpy(bat->phase.ptr, ph.data(), sizeof(double) * ph.size(), hipMemcpyHostToDevice));
    QS3_HIP(hipMemcpy(bat->compat_nt.ptr, bat->h_compat_nt.data(), bat->h_compat_nt.size(), hipMemcpyHostToDevice));
    if (n_sectors == 1 && lat->uniform && M <= 65536) {
        // the single-sector hop-list product reads e^{ik.t} per translation t
        // and the k-dependent stabiliser factors per representative
        const int nt = lat->lx * lat->ly * lat->lz;
        std::vector<uint16_t> tP(nt);
        for (int t = 0; t < nt; ++t) {
            const int tx = t % lat->lx, ty = (t / lat->lx) % lat->ly, tz = t / (lat->lx * lat->ly);
            tP[t] = (uint16_t)(((long)kmul[0] * tx + (long)kmul[1] * ty + (long)kmul[2] * tz) % M);
        }
        QS3_TRY(bat->tP.alloc(ctx, sizeof(uint16_t) * nt));
        QS3_HIP(hipMemcpy(bat->tP.ptr, tP.data(), sizeof(uint16_t) * nt, hipMemcpyHostToDevice));
        if (nnt > 0) {
            // a stabiliser acts freely on the N_down down spins, so s <= N_down
            std::vector<uint8_t> g(bat->ks->n_reps, 1);
            for (size_t q = 0; q < nnt; ++q) {
                const uint32_t u = bat->ks->nt_u[q];
                g[u] = bat->h_compat_nt[q] ? (uint8_t)bat->ks->h_stab[u] : 0;
            }
            QS3_TRY(bat->gcls.alloc(ctx, g.size()));
            QS3_HIP(hipMemcpy(bat->gcls.ptr, g.data(), g.size(), hipMemcpyHostToDevice));
        }
    }
    *out = bat.release();
    return QS3_OK;
}

int qs3_batch_destroy(qs3_batch *bat) {
    if (bat) {
        DeviceGuard dg(bat->lat->ctx->device);
        delete bat;
    }
    return QS3_OK;
}

namespace qs3 {

// A batch operator that owns its batch (the restriction of another one).
struct OwnedBatchOp : BatchOp {
    explicit OwnedBatchOp(qs3_batch *b) : BatchOp(b) {}
    ~OwnedBatchOp() override { qs3_batch_destroy(bat); }
};

int BatchOp::subset(const std::vector<int> &cols, std::unique_ptr<Operator> *out) {
    QS3_REQUIRE(!cols.empty(), QS3_EINVAL, "empty column subset");
    std::vector<int32_t> kv;
    kv.reserve(3 * cols.size());
    for (int c : cols) {
        QS3_REQUIRE(c >= 0 && c < bat->B, QS3_EINVAL, "column out of range");
        kv.insert(kv.end(), bat->kv.begin() + 3 * c, bat->kv.begin() + 3 * c + 3);
    }
    qs3_batch *nb = nullptr;
    QS3_TRY(qs3_batch_create(bat->lat, bat->K, (int)cols.size(), kv.data(), &nb));
    out->reset(new OwnedBatchOp(nb));
    return QS3_OK;
}

}  // namespace qs3

int qs3_batch_dims(const qs3_batch *bat, uint64_t *rows, uint64_t *dims) {
    QS3_REQUIRE(bat, QS3_EINVAL, "batch is NULL");
    if (rows) *rows = bat->ks->n_reps;
    if (dims)
        for (int b = 0; b < bat->B; ++b) dims[b] = bat->dims[b];
    return QS3_OK;
}

int qs3_batch_schedule(const qs3_batch *bat, int *lanes_per_row, int *blocks_per_cu) {
    QS3_REQUIRE(bat, QS3_EINVAL, "batch is NULL");
    if (lanes_per_row) *lanes_per_row = bat->last_G;
    if (blocks_per_cu) *blocks_per_cu = bat->last_bpc;
    return QS3_OK;
}

int qs3_batch_groups(const qs3_batch *bat, int *groups, int *sectors_per_group) {
    QS3_REQUIRE(bat, QS3_EINVAL, "batch is NULL");
    if (groups) *groups = bat->last_groups;
    if (sectors_per_group) *sectors_per_group = bat->last_group_width;
    return QS3_OK;
}

int qs3_batch_matvec(qs3_batch *bat, const void *v, void *w, int dtype, void *stream) {
    QS3_REQUIRE(bat && v && w, QS3_EINVAL, "NULL argument");
    QS3_REQUIRE(v != w, QS3_EINVAL, "v and w must not alias");
    QS3_REQUIRE(dtype == QS3_C128 || dtype == QS3_C64, QS3_EINVAL, "batch vectors are complex");
    DeviceGuard dg(bat->lat->ctx->device);
    return hv_batch(bat, v, dtype, w, dtype, (hipStream_t)stream);
}

int qs3_batch_eigs(qs3_batch *bat, const qs3_eigs_opts *opts, double *evals, qs3_eigs_info *info,
                   void *stream) {
    QS3_REQUIRE(bat && opts && evals, QS3_EINVAL, "NULL argument");
    DeviceGuard dg(bat->lat->ctx->device);
    auto t0 = std::chrono::steady_clock::now();
    qs3_eigs_opts o = *opts;
    uint64_t mind = *std::min_element(bat->dims.begin(), bat->dims.end());
    QS3_TRY(fill_opts(o, mind));
    hipStream_t s = (hipStream_t)stream;
    BatchOp op(bat);
    DevBuf v0, seeds;
    QS3_TRY(v0.alloc(bat->lat->ctx, sizeof(double) * 2 * bat->ks->n_reps * (uint64_t)bat->B));
    std::vector<uint64_t> hs(bat->B);
    for (int b = 0; b < bat->B; ++b) hs[b] = o.seed + (uint64_t)b;
    QS3_TRY(seeds.alloc(bat->lat->ctx, sizeof(uint64_t) * bat->B));
    QS3_HIP(hipMemcpyAsync(seeds.ptr, hs.data(), sizeof(uint64_t) * bat->B, hipMemcpyHostToDevice, s));
    QS3_TRY(start_vector_batch(bat, seeds.as<uint64_t>(), v0.as<double>(), s));
    std::vector<double> ev;
    std::vector<qs3_eigs_info> inf;
    QS3_TRY(solve_blocking(bat->lat->ctx, &op, o, v0.as<double>(), s, ev, inf, nullptr));
    double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    bool allc = true;
    for (int b = 0; b < bat->B; ++b) {
        for (int y = 0; y < opts->nev; ++y) evals[(size_t)b * opts->nev + y] = ev[(size_t)b * o.nev + y];
        inf[b].seconds = secs;
        if (info) info[b] = inf[b];
        allc &= inf[b].converged != 0;
    }
    return allc ? QS3_OK : QS3_ENOCONV;
}

// ---------------------------------------------------------------- sectors
int qs3_sector_create(qs3_lattice *lat, int n_down, const int32_t *kvec, qs3_sector **out) {
    QS3_REQUIRE(lat && out, QS3_EINVAL, "NULL argument");
    QS3_REQUIRE(n_down >= 0 && n_down <= lat->N, QS3_EINVAL, "n_down out of range");
    DeviceGuard dg(lat->ctx->device);
    auto sec = std::make_unique<qs3_sector>();
    sec->lat = lat;
    sec->K = n_down;
    if (!kvec) {
        QS3_REQUIRE(n_down <= MAX_K_U1, QS3_EINVAL, "n_down <= 8 for fixed-N_down sectors");
        QS3_TRY(get_binom(lat, n_down, &sec->bt));
        sec->dim = sec->bt->D;
    } else {
        sec->has_k = true;
        for (int a = 0; a < 3; ++a) sec->kv[a] = kvec[a];
        QS3_TRY(qs3_batch_create(lat, n_down, 1, kvec, &sec->bat));
        sec->bt = sec->bat->bt;
        sec->dim = sec->bat->dims[0];
        std::vector<int64_t> c2u;
        c2u.reserve(sec->dim);
        auto &ks = *sec->bat->ks;
        std::vector<int32_t> ntof(ks.n_reps, -1);
        for (size_t q = 0; q < ks.nt_u.size(); ++q) ntof[ks.nt_u[q]] = (int32_t)q;
        for (uint64_t u = 0; u < ks.n_reps; ++u) {
            if (ks.h_stab[u] > 1 && !sec->bat->h_compat_nt[ntof[u]]) continue;
            c2u.push_back((int64_t)u);
        }
        QS3_TRY(sec->comp2u.alloc(lat->ctx, sizeof(int64_t) * std::max<size_t>(c2u.size(), 1)));
        if (!c2u.empty())
            QS3_HIP(hipMemcpy(sec->comp2u.ptr, c2u.data(), sizeof(int64_t) * c2u.size(), hipMemcpyHostToDevice));
    }
    *out = sec.release();
    return QS3_OK;
}

int qs3_sector_destroy(qs3_sector *sec) {
    if (sec) {
        DeviceGuard dg(sec->lat->ctx->device);
        if (sec->bat) qs3_batch_destroy(sec->bat);
        delete sec;
    }
    return QS3_OK;
}

int qs3_sector_dim(const qs3_sector *sec, uint64_t *dim) {
    QS3_REQUIRE(sec && dim, QS3_EINVAL, "NULL argument");
    *dim = sec->dim;
    return QS3_OK;
}

int qs3_sector_basis(const qs3_sector *sec, uint64_t *ranks, uint32_t *stab) {
    QS3_REQUIRE(sec, QS3_EINVAL, "sector is NULL");
    if (!sec->has_k) {
        for (uint64_t i = 0; i < sec->dim; ++i) {
            if (ranks) ranks[i] = i;
            if (stab) stab[i] = 1;
        }
        return QS3_OK;
    }
    std::vector<int64_t> c2u(sec->dim);
    if (sec->dim)
        QS3_HIP(hipMemcpy(c2u.data(), sec->comp2u.ptr, sizeof(int64_t) * sec->dim, hipMemcpyDeviceToHost));
    auto &ks = *sec->bat->ks;
    for (uint64_t i = 0; i < sec->dim; ++i) {
        if (ranks) ranks[i] = ks.h_reps[c2u[i]];
        if (stab) stab[i] = ks.h_stab[c2u[i]];
    }
    return QS3_OK;
}

int qs3_sector_start_vector(qs3_sector *sec, uint64_t seed, void *v, int dtype, void *stream) {
    QS3_REQUIRE(sec && v, QS3_EINVAL, "NULL argument");
    DeviceGuard dg(sec->lat->ctx->device);
    hipStream_t s = (hipStream_t)stream;
    if (!sec->has_k) return start_vector_u1(sec, seed, v, dtype, s);
    QS3_REQUIRE(dtype == QS3_C128, QS3_EINVAL, "momentum start vectors are QS3_C128");
    qs3_ctx *ctx = sec->lat->ctx;
    DevBuf un, sd;
    QS3_TRY(un.alloc(ctx, sizeof(double) * 2 * sec->bat->ks->n_reps));
    QS3_TRY(sd.alloc(ctx, sizeof(uint64_t)));
    QS3_HIP(hipMemcpyAsync(sd.ptr, &seed, sizeof(uint64_t), hipMemcpyHostToDevice, s));
    QS3_TRY(start_vector_batch(sec->bat, sd.as<uint64_t>(), un.as<double>(), s));
    QS3_TRY(gather_compact(sec, un.as<double>(), (double *)v, s));
    QS3_HIP(hipStreamSynchronize(s));
    return QS3_OK;
}

int qs3_matvec(qs3_sector *sec, const void *v, void *w, int dtype, void *stream) {
    QS3_REQUIRE(sec && v && w, QS3_EINVAL, "NULL argument");
    QS3_REQUIRE(v != w, QS3_EINVAL, "v and w must not alias");
    DeviceGuard dg(sec->lat->ctx->device);
    hipStream_t s = (hipStream_t)stream;
    if (!sec->has_k) {
        QS3_REQUIRE(dtype == QS3_F64 || dtype == QS3_F32, QS3_EINVAL,
                    "fixed-N_down vectors are QS3_F64 or QS3_F32");
        return hv_u1(sec, v, dtype, w, dtype, s);
    }
    QS3_REQUIRE(dtype == QS3_C128 || dtype == QS3_C64, QS3_EINVAL,
                "momentum vectors are QS3_C128 or QS3_C64");
    const uint64_t n = sec->bat->ks->n_reps;
    if (sec->dim == n) return hv_batch(sec->bat, v, dtype, w, dtype, s);  // every rep compatible
    const size_t esz = dtype == QS3_C128 ? 16 : 8;
    if (!sec->scratch_a.ptr) {
        QS3_TRY(sec->scratch_a.alloc(sec->lat->ctx, esz * n * (dtype == QS3_C128 ? 1 : 2)));
        QS3_TRY(sec->scratch_b.alloc(sec->lat->ctx, esz * n * (dtype == QS3_C128 ? 1 : 2)));
    }
    if (dtype == QS3_C128) {
        QS3_TRY(scatter_compact(sec, (const double *)v, sec->scratch_a.as<double>(), s));
        QS3_TRY(hv_batch(sec->bat, sec->scratch_a.ptr, dtype, sec->scratch_b.ptr, dtype, s));
        return gather_compact(sec, sec->scratch_b.as<double>(), (double *)w, s);
    }
    QS3_TRY(scatter_compact_f32(sec, (const float *)v, sec->scratch_a.as<float>(), s));
    QS3_TRY(hv_batch(sec->bat, sec->scratch_a.ptr, dtype, sec->scratch_b.ptr, dtype, s));
    return gather_compact_f32(sec, sec->scratch_b.as<float>(), (float *)w, s);
}

int qs3_row(qs3_sector *sec, uint64_t row, int cap, int64_t *cols, double *vals, double *diag,
            int *nnz) {
    QS3_REQUIRE(sec && cols && vals && diag && nnz && cap >= 0, QS3_EINVAL, "bad argument");
    DeviceGuard dg(sec->lat->ctx->device);
    return sec->has_k ? row_k(sec, row, cap, cols, vals, diag, nnz)
                      : row_u1(sec, row, cap, cols, vals, diag, nnz);
}

// shared driver of qs3_eigs: run the solver on the sector's operator
static int sector_eigs(qs3_sector *sec, qs3_eigs_opts o, std::vector<double> &ev,
                       qs3_eigs_info &inf, void *evecs, hipStream_t s) {
    qs3_ctx *ctx = sec->lat->ctx;
    std::unique_ptr<Operator> op;
    if (sec->has_k) op.reset(new BatchOp(sec->bat));
    else op.reset(new U1Op(sec));
    const uint64_t stride = sec->has_k ? 2 * sec->bat->ks->n_reps : sec->dim;
    DevBuf v0, vo;
    QS3_TRY(v0.alloc(ctx, sizeof(double) * stride));
    if (!sec->has_k) {
        QS3_TRY(start_vector_u1(sec, o.seed, v0.ptr, QS3_F64, s));
    } else {
        DevBuf sd;
        QS3_TRY(sd.alloc(ctx, sizeof(uint64_t)));
        QS3_HIP(hipMemcpyAsync(sd.ptr, &o.seed, sizeof(uint64_t), hipMemcpyHostToDevice, s));
        QS3_TRY(start_vector_batch(sec->bat, sd.as<uint64_t>(), v0.as<double>(), s));
        QS3_HIP(hipStreamSynchronize(s));
    }
    if (evecs) QS3_TRY(vo.alloc(ctx, sizeof(double) * stride * o.nev));
    std::vector<qs3_eigs_info> infs;
    QS3_TRY(solve_blocking(ctx, op.get(), o, v0.as<double>(), s, ev, infs, evecs ? vo.as<double>() : nullptr));
    inf = infs[0];
    if (evecs) {
        for (int y = 0; y < o.nev; ++y) {
            double *src = vo.as<double>() + (size_t)y * stride;
            if (!sec->has_k)
                QS3_HIP(hipMemcpyAsync((double *)evecs + (size_t)y * sec->dim, src,
                                       sizeof(double) * sec->dim, hipMemcpyDeviceToDevice, s));
            else
                QS3_TRY(gather_compact(sec, src, (double *)evecs + (size_t)y * 2 * sec->dim, s));
        }
    }
    QS3_HIP(hipStreamSynchronize(s));
    return QS3_OK;
}

int qs3_eigs(qs3_sector *sec, const qs3_eigs_opts *opts, double *evals, void *evecs,
             qs3_eigs_info *info, void *stream) {
    QS3_REQUIRE(sec && opts && evals, QS3_EINVAL, "NULL argument");
    QS3_REQUIRE(sec->dim > 0, QS3_EINVAL, "empty sector");
    DeviceGuard dg(sec->lat->ctx->device);
    auto t0 = std::chrono::steady_clock::now();
    qs3_eigs_opts o = *opts;
    QS3_TRY(fill_opts(o, sec->dim));
    std::vector<double> ev;
    qs3_eigs_info inf{};
    QS3_TRY(sector_eigs(sec, o, ev, inf, evecs, (hipStream_t)stream));
    for (int y = 0; y < opts->nev; ++y) evals[y] = ev[y];
    inf.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (info) *info = inf;
    return inf.converged ? QS3_OK : QS3_ENOCONV;
}

int qs3_lanczos(qs3_sector *sec, const void *v0, int steps, int precision, int reorth,
                uint64_t seed, double *alpha, double *beta, double *norm0, int *done,
                void *stream) {
    QS3_REQUIRE(sec && alpha && beta && steps > 0, QS3_EINVAL, "bad argument");
    DeviceGuard dg(sec->lat->ctx->device);
    hipStream_t s = (hipStream_t)stream;
    qs3_ctx *ctx = sec->lat->ctx;
    std::unique_ptr<Operator> op;
    if (sec->has_k) op.reset(new BatchOp(sec->bat));
    else op.reset(new U1Op(sec));
    Engine E;
    QS3_REQUIRE(reorth >= QS3_REORTH_NONE && reorth <= QS3_REORTH_PARTIAL, QS3_EINVAL,
                "unknown reorthogonalisation mode");
    QS3_TRY(E.init(ctx, op.get(), steps + 1, precision, engine_reorth(reorth, false), s));
    DevBuf vb;
    QS3_TRY(vb.alloc(ctx, sizeof(double) * E.stride));
    if (v0) {
        if (!sec->has_k)
            QS3_HIP(hipMemcpyAsync(vb.ptr, v0, sizeof(double) * sec->dim, hipMemcpyDeviceToDevice, s));
        else
            QS3_TRY(scatter_compact(sec, (const double *)v0, vb.as<double>(), s));
    } else if (!sec->has_k) {
        QS3_TRY(start_vector_u1(sec, seed, vb.ptr, QS3_F64, s));
    } else {
        DevBuf sd;
        QS3_TRY(sd.alloc(ctx, sizeof(uint64_t)));
        QS3_HIP(hipMemcpyAsync(sd.ptr, &seed, sizeof(uint64_t), hipMemcpyHostToDevice, s));
        QS3_TRY(start_vector_batch(sec->bat, sd.as<uint64_t>(), vb.as<double>(), s));
        QS3_HIP(hipStreamSynchronize(s));
    }
    std::vector<double> a, b, n0;
    std::vector<int> dn;
    QS3_TRY(run_lanczos(E, vb.as<double>(), steps, a, b, n0, dn));
    // a zero or non-finite start vector (or coefficients that turned
    // non-finite) leaves the outputs untouched
    QS3_REQUIRE(std::isfinite(n0[0]) && n0[0] > 0.0, QS3_ENUMERIC, "zero or non-finite start vector");
    for (int x = 0; x < dn[0]; ++x)
        QS3_REQUIRE(std::isfinite(a[x]) && std::isfinite(b[x]), QS3_ENUMERIC, "non-finite Lanczos coefficient");
    for (int x = 0; x < steps; ++x) {
        alpha[x] = a[x];
        beta[x] = b[x];
    }
    if (norm0) *norm0 = n0[0];
    if (done) *done = dn[0];
    return QS3_OK;
}

}  // extern "C"
