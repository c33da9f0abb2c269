// Serving: continuous batching of XXZ solve requests on one device.
//
// A worker thread owns the device work.  Requests wait in a FIFO queue until a
// slot is free and their device footprint (Krylov basis, work vectors and the
// momentum structure they need) fits the server budget; an admitted request
// gets its own stream, lattice, sector and resumable solver (SolveRun).  The
// worker polls every running request's event and, when its restart cycle has
// finished, does the host part and enqueues the next cycle, so the kernels of
// all admitted requests overlap on the device, new requests are admitted as
// soon as memory and slots free up, and finished requests retire
// independently.  A request's arithmetic is the same kernels in the same order
// whatever else runs, so its result does not depend on the mix.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "qs3_impl.h"
#include "qs3_krylov.h"

namespace qs3 {

enum ReqPhase { RQ_QUEUED = 0, RQ_RUNNING = 1, RQ_DONE = 2 };

struct ReqState {
    uint64_t ticket = 0;
    qs3_request req{};
    std::vector<int32_t> bi, bj;
    std::vector<double> jxy, jz;
    int phase = RQ_QUEUED;
    bool canceled = false;
    qs3_result res{};
    uint64_t footprint = 0;
    qs3_eigs_opts opts{};
    qs3_lattice *lat = nullptr;
    qs3_sector *sec = nullptr;
    hipStream_t stream = nullptr;
    std::unique_ptr<Operator> op;
    std::unique_ptr<SolveRun> run;
    DevBuf v0;
};

}  // namespace qs3

struct qs3_server {
    qs3_ctx *ctx = nullptr;
    int max_active = 8;
    uint64_t budget = 0;
    uint64_t reserved = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<qs3::ReqState *> queue;
    std::vector<qs3::ReqState *> running;
    std::unordered_map<uint64_t, std::unique_ptr<qs3::ReqState>> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    std::chrono::steady_clock::time_point t0;
    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace qs3 {

static double binom_d(int n, int k) {
    if (k < 0 || k > n) return 0.0;
    double r = 1.0;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

// Device bytes a request needs: Krylov basis (N_M + 1 + N_K vectors), work
// and start vectors, the float32 copy, reduction scratch, and for momentum
// sectors the representative list, stabilisers, directory and the two hop
// stores the structure build makes when they fit the context's limits: the
// rank -> representative table (8 B per rank) and the per-representative
// hop lists (8 B per representative and hop slot, N_down x the largest
// degree slots).
static uint64_t footprint(const qs3_request &q, const qs3_eigs_opts &o, int max_degree,
                          const qs3_ctx *ctx) {
    const int N = q.lx * q.ly * q.lz;
    const double D = binom_d(N, q.n_down);
    const double rows = q.use_k ? D / N * 1.05 + 64 : D;
    const double elem = q.use_k ? 16.0 : 8.0;
    const double slots = qs3::SolveRun::slots_for(o) + 2 +
                         (o.precision == QS3_PREC_F32MV ? 0.5 : 0.0);
    double bytes = rows * elem * slots + 4.0 * 1024 * 1024;
    if (q.use_k) {
        bytes += rows * (8 + 2 + 4) + 4.0 * (1 << 24);
        if (D * 8 <= (double)ctx->table_limit) bytes += D * 8;
        const double hops = rows * (double)q.n_down * max_degree * 8;
        if (hops <= (double)ctx->hop_list_limit) bytes += hops;
    }
    if (!(bytes < 1.8e19)) return ~0ull;
    return (uint64_t)bytes;
}

static void release_runtime(ReqState *r) {
    if (r->stream) (void)hipStreamSynchronize(r->stream);
    r->run.reset();
    r->op.reset();
    r->v0.release();
    if (r->sec) qs3_sector_destroy(r->sec);
    r->sec = nullptr;
    if (r->lat) qs3_lattice_destroy(r->lat);
    r->lat = nullptr;
    if (r->stream) (void)hipStreamDestroy(r->stream);
    r->stream = nullptr;
}

// called with the lock held
static void finish_locked(qs3_server *S, ReqState *r, int status) {
    r->res.status = status;
    r->res.t_done = S->now();
    r->phase = RQ_DONE;
    S->cv_done.notify_all();
}

// device set-up and the first cycle; no lock held
static int start_request(qs3_server *S, ReqState *r) {
    qs3_ctx *ctx = S->ctx;
    const qs3_request &q = r->req;
    QS3_HIP(hipStreamCreateWithFlags(&r->stream, hipStreamNonBlocking));
    QS3_TRY(qs3_lattice_create(ctx, q.lx, q.ly, q.lz, q.n_bonds, r->bi.data(), r->bj.data(), r->jxy.data(),
                               r->jz.data(), &r->lat));
    QS3_TRY(qs3_sector_create(r->lat, q.n_down, q.use_k ? q.kvec : nullptr, &r->sec));
    QS3_REQUIRE(r->sec->dim > 0, QS3_EINVAL, "empty sector");
    r->res.dim = r->sec->dim;
    QS3_TRY(fill_opts(r->opts, r->sec->dim));
    if (r->sec->has_k) r->op.reset(new BatchOp(r->sec->bat));
    else r->op.reset(new U1Op(r->sec));
    const uint64_t stride = r->sec->has_k ? 2 * r->sec->bat->ks->n_reps : r->sec->dim;
    QS3_TRY(r->v0.alloc(ctx, sizeof(double) * stride));
    if (!r->sec->has_k) {
        QS3_TRY(start_vector_u1(r->sec, r->opts.seed, r->v0.ptr, QS3_F64, r->stream));
    } else {
        DevBuf sd;
        QS3_TRY(sd.alloc(ctx, sizeof(uint64_t)));
        QS3_HIP(hipMemcpyAsync(sd.ptr, &r->opts.seed, sizeof(uint64_t), hipMemcpyHostToDevice, r->stream));
        QS3_TRY(start_vector_batch(r->sec->bat, sd.as<uint64_t>(), r->v0.as<double>(), r->stream));
        QS3_HIP(hipStreamSynchronize(r->stream));
    }
    r->run.reset(new SolveRun());
    QS3_TRY(r->run->init(ctx, r->op.get(), r->opts, r->stream));
    QS3_TRY(r->run->begin(r->v0.as<double>()));
    return QS3_OK;
}

static void worker_main(qs3_server *S) {
    (void)hipSetDevice(S->ctx->device);
    for (;;) {
        std::vector<ReqState *> to_start;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->stop && S->queue.empty() && S->running.empty()) break;
            // admission: FIFO, a slot and the footprint must both be free
            while (!S->queue.empty() && (int)(S->running.size() + to_start.size()) < S->max_active) {
                ReqState *r = S->queue.front();
                if (r->canceled || S->stop) {
                    S->queue.pop_front();
                    finish_locked(S, r, QS3_ECANCELED);
                    continue;
                }
                if (r->footprint > S->budget) {
                    S->queue.pop_front();
                    finish_locked(S, r, QS3_ENOMEM);
                    continue;
                }
                if (S->reserved + r->footprint > S->budget) break;
                S->queue.pop_front();
                S->reserved += r->footprint;
                r->res.t_start = S->now();
                to_start.push_back(r);
            }
        }
        for (ReqState *r : to_start) {
            int rc = start_request(S, r);
            std::lock_guard<std::mutex> lk(S->mu);
            if (rc < 0) {
                release_runtime(r);
                S->reserved -= r->footprint;
                finish_locked(S, r, rc);
            } else {
                r->phase = RQ_RUNNING;
                S->running.push_back(r);
            }
        }
        // progress of the running requests
        bool progressed = !to_start.empty();
        std::vector<ReqState *> snapshot;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            snapshot = S->running;
        }
        for (ReqState *r : snapshot) {
            bool canceled;
            {
                std::lock_guard<std::mutex> lk(S->mu);
                canceled = r->canceled || S->stop;
            }
            int status = 1;  // 1 = still running
            if (canceled) {
                status = QS3_ECANCELED;
            } else if (r->run->ready()) {
                progressed = true;
                bool done = false;
                int rc = r->run->advance(&done);
                if (rc < 0) status = rc;
                else if (done) {
                    (void)r->run->wait();
                    const auto &inf = r->run->info[0];
                    r->res.n_found = inf.n_found;
                    r->res.n_matvec = r->run->eng().n_matvec;
                    for (int y = 0; y < r->opts.nev && y < 16; ++y) r->res.evals[y] = r->run->evals[y];
                    status = inf.converged ? QS3_OK : QS3_ENOCONV;
                }
            }
            if (status != 1) {
                release_runtime(r);
                std::lock_guard<std::mutex> lk(S->mu);
                S->running.erase(std::find(S->running.begin(), S->running.end(), r));
                S->reserved -= r->footprint;
                finish_locked(S, r, status);
                progressed = true;
            }
        }
        if (!progressed) {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->running.empty() && (S->queue.empty() || S->stop)) {
                if (S->stop && S->queue.empty()) break;
                S->cv_work.wait_for(lk, std::chrono::milliseconds(20));
            } else {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(20));
            }
        }
    }
}

}  // namespace qs3

using namespace qs3;

extern "C" {

int qs3_server_create(qs3_ctx *ctx, const qs3_server_opts *opts, qs3_server **out) {
    QS3_REQUIRE(ctx && out, QS3_EINVAL, "NULL argument");
    auto *S = new qs3_server();
    S->ctx = ctx;
    S->max_active = (opts && opts->max_active > 0) ? opts->max_active : 8;
    S->budget = (opts && opts->budget_bytes) ? std::min<uint64_t>(opts->budget_bytes, ctx->budget)
                                             : ctx->budget;
    S->t0 = std::chrono::steady_clock::now();
    S->worker = std::thread(worker_main, S);
    *out = S;
    return QS3_OK;
}

int qs3_server_destroy(qs3_server *S) {
    if (!S) return QS3_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    delete S;
    return QS3_OK;
}

int qs3_submit(qs3_server *S, const qs3_request *q, uint64_t *ticket) {
    QS3_REQUIRE(S && q && ticket, QS3_EINVAL, "NULL argument");
    QS3_REQUIRE(q->lx >= 1 && q->ly >= 1 && q->lz >= 1 && q->n_bonds >= 0, QS3_EINVAL, "bad lattice");
    QS3_REQUIRE(q->nev >= 1 && q->nev <= 16, QS3_EINVAL, "nev must be in [1, 16]");
    auto r = std::make_unique<ReqState>();
    r->req = *q;
    r->bi.assign(q->bi, q->bi + q->n_bonds);
    r->bj.assign(q->bj, q->bj + q->n_bonds);
    r->jxy.assign(q->jxy, q->jxy + q->n_bonds);
    r->jz.assign(q->jz, q->jz + q->n_bonds);
    r->req.bi = r->req.bj = nullptr;
    r->req.jxy = r->req.jz = nullptr;
    r->opts = qs3_eigs_opts{};
    r->opts.alg = QS3_ALG_TRL;
    r->opts.nev = q->nev;
    r->opts.seed = q->seed;
    r->opts.precision = q->precision;
    r->opts.reorth = 1;
    qs3_eigs_opts est = r->opts;
    est.nk = default_nk(est.nev);
    est.nm = default_nm(est.nk);
    std::vector<int> deg((size_t)std::max(q->lx * q->ly * q->lz, 1), 0);
    int max_degree = 0;
    for (size_t b = 0; b < r->bi.size(); ++b) {
        const int i = r->bi[b], j = r->bj[b];
        if (i >= 0 && j >= 0 && i < (int)deg.size() && j < (int)deg.size() && i != j) {
            max_degree = std::max(max_degree, ++deg[i]);
            max_degree = std::max(max_degree, ++deg[j]);
        }
    }
    r->footprint = footprint(r->req, est, max_degree, S->ctx);
    r->res.footprint_bytes = r->footprint;
    std::lock_guard<std::mutex> lk(S->mu);
    r->ticket = S->next_ticket++;
    r->res.t_submit = S->now();
    *ticket = r->ticket;
    S->queue.push_back(r.get());
    S->all[r->ticket] = std::move(r);
    S->cv_work.notify_all();
    return QS3_OK;
}

int qs3_poll(qs3_server *S, uint64_t ticket, qs3_result *out) {
    QS3_REQUIRE(S && out, QS3_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) {
        set_error("unknown ticket");
        return QS3_ENOTFOUND;
    }
    if (it->second->phase != RQ_DONE) return QS3_EBUSY;
    *out = it->second->res;
    return QS3_OK;
}

int qs3_wait(qs3_server *S, uint64_t ticket, qs3_result *out) {
    QS3_REQUIRE(S && out, QS3_EINVAL, "NULL argument");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) {
        set_error("unknown ticket");
        return QS3_ENOTFOUND;
    }
    ReqState *r = it->second.get();
    S->cv_done.wait(lk, [&] { return r->phase == RQ_DONE; });
    *out = r->res;
    return QS3_OK;
}

int qs3_cancel(qs3_server *S, uint64_t ticket) {
    QS3_REQUIRE(S, QS3_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) {
        set_error("unknown ticket");
        return QS3_ENOTFOUND;
    }
    it->second->canceled = true;
    S->cv_work.notify_all();
    return QS3_OK;
}

double qs3_server_clock(qs3_server *S) { return S ? S->now() : 0.0; }

}  // extern "C"
