// serve.hip -- request server of the CGGM library: continuous batching of
// many regularisation-path solves on one device.
//
// Worker threads (one HIP stream each) take requests from a queue when the
// device pool has a free block for the request's workspace; a request keeps
// its block (Sigma, the factor, the maintained products, the parameters)
// resident over its whole penalty path and gives it back when done.  Kernels
// of different requests overlap on the device through their streams.
#include <math.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "admission.hpp"
#include "solver.hpp"

namespace cggm {
namespace {

constexpr size_t POOL_ALIGN = 256;
constexpr int MAX_SLOTS = 64;

struct Job {
    int64_t ticket = 0;
    cggm_request req{};
    std::vector<double> lamL, lamT;
    cggm_options opt{};
    size_t footprint = 0, offset = 0;
    double t_submit = 0.0, t_admit = 0.0, t_done = 0.0;
    int slot = -1, status = CGGM_OK, iters_total = 0;
    std::vector<double> f;
    std::vector<int> iters;
    std::string error;
    bool done = false;
};

size_t round_up(size_t b) { return (b + POOL_ALIGN - 1) & ~(POOL_ALIGN - 1); }

}  // namespace

struct Server {
    std::mutex m;
    std::condition_variable cv_work, cv_done;
    std::deque<Job *> queue;
    std::unordered_map<int64_t, std::unique_ptr<Job>> jobs;
    Pool pool;
    void *base = nullptr;
    int slots = 1, max_bypass = 0, head_bypassed = 0, running = 0;
    size_t in_use = 0;
    cggm_server_stats st{};
    bool stopping = false;
    int64_t next_ticket = 1;
    int device = 0;
    std::vector<std::thread> workers;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();

    double now_ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
            .count();
    }

    Job *admit_locked() { return admit_next(queue, pool, head_bypassed, max_bypass); }

    void run_job(Job &j, hipStream_t s) {
        const cggm_request &r = j.req;
        int iters_total = 0;
        j.status = guarded([&] {
            Solver sv(r.n, r.p, r.q, &j.opt, s, r.dtype);
            if (round_up(sv.footprint()) != j.footprint)
                fail(CGGM_EHIP, "workspace size changed between submit and admission");
            sv.bind((char *)base + j.offset);
            sv.load(r.X, r.Y);
            sv.start();
            int status = CGGM_OK;
            for (int k = 0; k < r.npath; ++k) {
                const SolveOutcome o = sv.run(j.lamL[k], j.lamT[k], r.tol);
                j.f[k] = o.f;
                j.iters[k] = o.iters;
                iters_total += o.iters;
                status = combine_status(status, o.status);
                sv.copy_dense(r.Lambda_out ? r.Lambda_out + (int64_t)k * r.q * r.q : nullptr,
                              r.Theta_out ? r.Theta_out + (int64_t)k * r.p * r.q : nullptr);
            }
            CGGM_HIP(hipStreamSynchronize(s));
            return status;
        });
        if (j.status < 0 && j.status != CGGM_ELINESEARCH) {
            j.error = last_error_text();
            // Leave the stream idle before the block goes back to the pool.
            (void)hipStreamSynchronize(s);
        }
        j.iters_total = iters_total;
    }

    void worker(int slot) {
        hipStream_t s = nullptr;
        const bool ok = hipSetDevice(device) == hipSuccess &&
                        hipStreamCreateWithFlags(&s, hipStreamNonBlocking) == hipSuccess;
        for (;;) {
            Job *j = nullptr;
            {
                std::unique_lock<std::mutex> lk(m);
                cv_work.wait(lk, [&] {
                    j = admit_locked();
                    return j != nullptr || (stopping && queue.empty());
                });
                if (!j) break;
                j->slot = slot;
                j->t_admit = now_ms();
                ++running;
                in_use += j->footprint;
                st.max_running = std::max(st.max_running, running);
                st.peak_bytes_in_use = std::max(st.peak_bytes_in_use, in_use);
            }
            if (ok) {
                run_job(*j, s);
            } else {
                j->status = CGGM_EHIP;
                j->error = "the worker could not create its HIP stream";
            }
            {
                std::lock_guard<std::mutex> lk(m);
                pool.give(j->offset, j->footprint);
                in_use -= j->footprint;
                --running;
                j->t_done = now_ms();
                j->done = true;
                ++st.completed;
            }
            cv_done.notify_all();
            cv_work.notify_all();
        }
        if (s) (void)hipStreamDestroy(s);
    }
};

namespace {

Job *make_job(const cggm_request *req) {
    if (!req) fail(CGGM_EINVAL, "NULL request");
    const cggm_request &r = *req;
    if (!r.X || !r.Y || !r.lamL || !r.lamT) fail(CGGM_EINVAL, "NULL pointer in the request");
    if (r.npath < 1) fail(CGGM_EINVAL, "npath must be >= 1");
    if (!(r.tol >= 0.0) || !isfinite(r.tol)) fail(CGGM_EINVAL, "tol must be finite and >= 0");
    if (r.max_iter < 0 || r.lambda_passes < 0) fail(CGGM_EINVAL, "invalid iteration limits");
    for (int k = 0; k < r.npath; ++k)
        if (!(r.lamL[k] >= 0.0) || !(r.lamT[k] >= 0.0) || !isfinite(r.lamL[k]) ||
            !isfinite(r.lamT[k]))
            fail(CGGM_EINVAL, "penalties must be finite and >= 0");
    auto j = std::make_unique<Job>();
    j->req = r;
    j->lamL.assign(r.lamL, r.lamL + r.npath);
    j->lamT.assign(r.lamT, r.lamT + r.npath);
    j->req.lamL = nullptr;     // the copies above are what the worker reads
    j->req.lamT = nullptr;
    cggm_default_options(&j->opt);
    j->opt.precision = r.precision;
    j->opt.graphs = 1;       // replay each sweep's launches: small requests are launch-bound
    if (r.tile > 0) j->opt.tile = r.tile;
    if (r.max_iter > 0) j->opt.max_iter = r.max_iter;
    if (r.lambda_passes > 0) j->opt.lambda_passes = r.lambda_passes;
    if (r.mixed_min_q >= 0) j->opt.mixed_min_q = r.mixed_min_q;
    j->footprint = round_up(solve_footprint(r.n, r.p, r.q, &j->opt, r.dtype));   // validates
    j->f.assign(r.npath, 0.0);
    j->iters.assign(r.npath, 0);
    return j.release();
}

}  // namespace
}  // namespace cggm

using namespace cggm;

extern "C" {

int cggm_server_create(int slots, size_t pool_bytes, int max_bypass, cggm_server **out) {
    return guarded([&] {
        if (!out) fail(CGGM_EINVAL, "NULL output pointer");
        if (slots < 1 || slots > MAX_SLOTS) fail(CGGM_EINVAL, "slots must be in [1, 64]");
        if (max_bypass < 0) fail(CGGM_EINVAL, "max_bypass must be >= 0");
        pool_bytes &= ~(POOL_ALIGN - 1);
        if (pool_bytes == 0) fail(CGGM_EINVAL, "pool_bytes must be >= 256");
        auto srv = std::make_unique<Server>();
        CGGM_HIP(hipGetDevice(&srv->device));
        if (hipMalloc(&srv->base, pool_bytes) != hipSuccess) {
            (void)hipGetLastError();
            srv->base = nullptr;
            fail(CGGM_ENOMEM, "hipMalloc of the " + std::to_string(pool_bytes) +
                                  "-byte pool failed");
        }
        srv->pool.init(pool_bytes);
        srv->st.pool_bytes = pool_bytes;
        srv->slots = slots;
        srv->max_bypass = max_bypass;
        Server *raw = srv.get();
        try {
            for (int k = 0; k < slots; ++k) srv->workers.emplace_back([raw, k] { raw->worker(k); });
        } catch (...) {
            {
                std::lock_guard<std::mutex> lk(raw->m);
                raw->stopping = true;
            }
            raw->cv_work.notify_all();
            for (auto &t : raw->workers) t.join();
            (void)hipFree(raw->base);
            throw;
        }
        *out = reinterpret_cast<cggm_server *>(srv.release());
        return CGGM_OK;
    });
}

int cggm_server_submit(cggm_server *srv_, const cggm_request *req, int64_t *ticket) {
    return guarded([&] {
        auto *srv = reinterpret_cast<Server *>(srv_);
        if (!srv || !ticket) fail(CGGM_EINVAL, "NULL pointer argument");
        std::unique_ptr<Job> j(make_job(req));
        std::lock_guard<std::mutex> lk(srv->m);
        if (srv->stopping) fail(CGGM_EINVAL, "the server is shutting down");
        if (j->footprint > srv->pool.size) {
            ++srv->st.rejected;
            fail(CGGM_ECAPACITY, "the request needs " + std::to_string(j->footprint) +
                                     " bytes, the pool has " + std::to_string(srv->pool.size));
        }
        j->ticket = srv->next_ticket++;
        j->t_submit = srv->now_ms();
        *ticket = j->ticket;
        srv->queue.push_back(j.get());
        srv->jobs.emplace(j->ticket, std::move(j));
        ++srv->st.submitted;
        srv->cv_work.notify_all();
        return CGGM_OK;
    });
}

int cggm_server_wait(cggm_server *srv_, int64_t ticket, cggm_request_info *info, double *f,
                     int *iters) {
    return guarded([&] {
        auto *srv = reinterpret_cast<Server *>(srv_);
        if (!srv) fail(CGGM_EINVAL, "NULL server");
        std::unique_ptr<Job> j;
        {
            std::unique_lock<std::mutex> lk(srv->m);
            auto it = srv->jobs.find(ticket);
            if (it == srv->jobs.end()) fail(CGGM_EINVAL, "unknown ticket");
            Job *raw = it->second.get();
            srv->cv_done.wait(lk, [&] { return raw->done; });
            j = std::move(it->second);
            srv->jobs.erase(it);
        }
        if (info) {
            info->status = j->status;
            info->slot = j->slot;
            info->iters_total = j->iters_total;
            info->_pad = 0;
            info->t_submit_ms = j->t_submit;
            info->t_admit_ms = j->t_admit;
            info->t_done_ms = j->t_done;
            info->footprint = j->footprint;
        }
        if (f) std::copy(j->f.begin(), j->f.end(), f);
        if (iters) std::copy(j->iters.begin(), j->iters.end(), iters);
        if (j->status < 0 && !j->error.empty()) fail(j->status, j->error);
        return j->status;
    });
}

int cggm_server_stats_get(cggm_server *srv_, cggm_server_stats *st) {
    return guarded([&] {
        auto *srv = reinterpret_cast<Server *>(srv_);
        if (!srv || !st) fail(CGGM_EINVAL, "NULL pointer argument");
        std::lock_guard<std::mutex> lk(srv->m);
        *st = srv->st;
        return CGGM_OK;
    });
}

void cggm_server_destroy(cggm_server *srv_) {
    auto *srv = reinterpret_cast<Server *>(srv_);
    if (!srv) return;
    {
        std::lock_guard<std::mutex> lk(srv->m);
        srv->stopping = true;
    }
    srv->cv_work.notify_all();
    for (auto &t : srv->workers) t.join();
    if (srv->base) (void)hipFree(srv->base);
    delete srv;
}

}  // extern "C"
