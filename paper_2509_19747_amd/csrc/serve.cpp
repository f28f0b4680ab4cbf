// rr_serve: continuous-batching server for independent kernel ridge solves.
//
// One host loop polls next() for arrivals, queues them in FIFO order and admits
// the head of the queue as soon as a slot is free and its device-memory estimate
// fits in the remaining HBM budget (a request larger than the whole budget is
// rejected).  Each slot is a worker thread with its own HIP stream: it uploads
// the request, builds the request's C-RandRAND preconditioner, keeps it resident
// while it solves all its right-hand sides, copies X back to the host, frees
// everything and calls deliver().  Builds of different requests overlap on their
// streams.  The PCG iteration batches run in the grouped engine (group.cpp): every
// request waiting for its next batch joins one replay of grouped persistent
// kernels, so the iterations of all resident requests share each launch; with
// grouping off each request replays its own captured hipGraph.  A request's
// arithmetic depends only on the request (own handle, own work items, fixed-order
// reductions), so its result is the same alone and in the mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "batch.hpp"
#include "ctx.hpp"
#include "group.hpp"

using namespace rr;

namespace {

double wall_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// Device bytes one request holds at its peak (build temporaries included).
size_t request_bytes(const rr_request& r, bool grouped) {
    const double n = (double)r.n, l = (double)r.l, d = (double)r.d, m = (double)std::max(r.nrhs, 1);
    double b = n * l * (4 + 2 + 8 + 4 + 8 + 16);        // Omega f32/bf16, Q, Y, W, Theta
    b += n * d * 4 + n * 4;                              // points, |x|^2
    b += l * l * 8 * 26 + 4.0 * (2 * l) * (2 * l) * 8;   // l x l factors, GEMM workspace
    const int nr = (int)std::min<double>(m, 8.0);
    b += 8.0 * (double)std::max(rr::kernel_matvec_ws_doubles(r.n, r.d, nr),   // matvec slot partials
                                rr::kernel_matvec_ws_doubles(r.n, r.d, 2));
    b += n * 8 * (8 + 8 * m);                            // CG vectors, batched PCG blocks, B and X
    if (grouped) {
        // slot partials per (padded) column, Q^T R partials and D per column
        const int64_t cols = std::max<int64_t>(r.nrhs, 1) + 3;
        b += 8.0 * (double)cols * (double)rr::kernel_mma_ws_doubles(r.n, 1);
        b += 8.0 * m * l * (rr::gemv_t_chunks(r.n, std::max<int64_t>(r.l, 1)) + 1);
    }
    b += 64.0 * 1024 * 1024;                             // fixed slack
    return (size_t)b;
}

struct Job {
    rr_request req;
    size_t bytes;
};

struct Shared {
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Job> admitted;
    bool stop = false;
    size_t used = 0, peak = 0;
    int active = 0, max_active = 0;
    std::vector<double> lat_ms;          // OK requests only
    int64_t served = 0, rejected = 0, ok = 0, failed = 0, graph_fallbacks = 0;
    GroupEngine* engine = nullptr;   // grouped PCG batches (nullptr: a graph per request)
    std::mutex deliver_mu;
    rr_status first_err = RR_OK;
    std::string first_err_msg;   // the library's message for the first failed request
};

void run_job(const rr_serve_config& cfg, Job& job, hipStream_t st, double t0, rr_deliver_fn deliver,
             void* user, Shared& sh) {
    rr_request& r = job.req;
    rr_solve_info info{};
    info.status = RR_OK;
    rr_precond* P = nullptr;
    float* pts = nullptr;
    double *b = nullptr, *x = nullptr;
    const int64_t n = r.n;
    const int64_t nr = std::max<int32_t>(r.nrhs, 1);
    std::string err_msg;
    auto fail = [&](rr_status s) {
        info.status = s;
        if (err_msg.empty()) err_msg = rr_last_error();   // this worker thread's message
    };
    // request buffers: the caller's allocator when the config has one, else the
    // device's stream-ordered pool on this worker's stream
    const rr_allocator* ua = cfg.alloc;
    auto dalloc = [&](size_t bytes) -> void* {
        if (ua) return ua->alloc(ua->ctx, bytes, (void*)st);
        void* q = nullptr;
        if (hipMallocAsync(&q, bytes, st) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return q;
    };
    auto dfree = [&](void* q) {
        if (!q) return;
        if (ua) ua->free(ua->ctx, q, (void*)st);
        else (void)hipFreeAsync(q, st);
    };
    do {
        pts = (float*)dalloc((size_t)r.d * n * sizeof(float));
        b = (double*)dalloc((size_t)n * nr * sizeof(double));
        x = (double*)dalloc((size_t)n * nr * sizeof(double));
        if (!pts || !b || !x) {
            fail(RR_ENOMEM);
            break;
        }
        if (hipMemcpyAsync(pts, r.pts, (size_t)r.d * n * sizeof(float), hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemcpyAsync(b, r.B, (size_t)n * nr * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess ||
            hipMemsetAsync(x, 0, (size_t)n * nr * sizeof(double), st) != hipSuccess) {
            fail(RR_EDEVICE);
            break;
        }
        rr_operator op{};
        op.kind = r.kind;
        op.n = n;
        op.pts = pts;
        op.d = r.d;
        op.kconst = r.kconst;
        op.scale = r.scale;
        rr_build_opts bo = cfg.build;
        bo.l = r.l;
        bo.seed = r.seed;
        const double mu = r.mu;
        // the library's own allocation path: the worker's stream keeps its freed
        // blocks, so the next request on this slot reuses them without pool calls
        rr_status s = rr_build_precond(&op, &mu, 1, &bo, ua, st, &P);
        if (s != RR_OK) { fail(s); break; }
        // every right-hand side of the request in one fused batched PCG, its
        // iteration batches replayed as a hipGraph
        rr_solve_opts so = cfg.solve;
        if (cfg.graph_iters > 0) {
            so.use_graph = 1;
            so.check_every = cfg.graph_iters;
        }
        so.relres_history = nullptr;
        so.history_cap = 0;
        std::vector<int32_t> mu_idx((size_t)nr, 0);
        std::vector<rr_solve_info> infos((size_t)nr);
        struct EngineRunner final : BatchRunner {
            GroupEngine* e;
            explicit EngineRunner(GroupEngine* eng) : e(eng) {}
            rr_status run(Batch& bt, double* X, int64_t ldx) override { return e->run(bt, X, ldx); }
        } runner(sh.engine);
        s = solve_batch_with(P, mu_idx.data(), b, n, (int32_t)nr, x, n, &so, infos.data(), st,
                             sh.engine ? &runner : nullptr);
        int iters = 0;
        double worst = 0.0, worst64 = 0.0;
        for (const rr_solve_info& si : infos) {
            iters = std::max(iters, si.iters);
            worst = std::max(worst, si.relres_work);
            if (std::isfinite(si.relres_fp64)) worst64 = std::max(worst64, si.relres_fp64);
            info.tau = si.tau; info.normE = si.normE; info.lamhat = si.lamhat; info.orth_err = si.orth_err;
            info.ms_build = si.ms_build;
            info.ms_solve = si.ms_solve;
            info.restarts = std::max(info.restarts, si.restarts);
            info.graph_fallbacks = std::max(info.graph_fallbacks, si.graph_fallbacks);
        }
        if (hipMemcpyAsync(r.X, x, (size_t)n * nr * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            s = RR_EDEVICE;
        }
        info.iters = iters;
        info.relres_work = worst;
        info.relres_fp64 = worst64;
        if (s != RR_OK) fail(s);
    } while (false);
    (void)hipStreamSynchronize(st);
    // the handle's work is complete (every call returned after it); its blocks stay
    // in this worker stream's cache for the next request on the slot.  No device-wide
    // synchronisation anywhere on this path: other workers may be capturing graphs.
    if (P) rr_precond_release(P, true);
    dfree(pts);
    dfree(b);
    dfree(x);
    (void)hipStreamSynchronize(st);
    const double t_done = wall_s() - t0;
    {
        std::lock_guard<std::mutex> lk(sh.deliver_mu);
        deliver(user, &r, &info, t_done);
    }
    std::lock_guard<std::mutex> lk(sh.mu);
    sh.used -= job.bytes;
    sh.active -= 1;
    sh.served += 1;
    if (info.status == RR_OK) {
        sh.ok += 1;
        sh.lat_ms.push_back(1e3 * (t_done - r.t_arrival));
    } else {
        sh.failed += 1;
    }
    sh.graph_fallbacks += info.graph_fallbacks ? 1 : 0;
    if (info.status != RR_OK && sh.first_err == RR_OK) {
        sh.first_err = (rr_status)info.status;
        sh.first_err_msg = err_msg;
    }
    sh.cv_done.notify_all();
}

}  // namespace

extern "C" rr_status rr_serve(const rr_serve_config* cfg, rr_next_fn next, rr_deliver_fn deliver,
                              void* user, rr_serve_stats* stats) {
    return guarded([&]() -> rr_status {
        RR_REQUIRE(cfg != nullptr, "config is null");
        RR_REQUIRE(next != nullptr && deliver != nullptr, "callbacks are null");
        RR_REQUIRE(cfg->max_slots >= 1 && cfg->max_slots <= 64, "max_slots must be in [1, 64]");
        RR_REQUIRE(cfg->hbm_budget > 0, "hbm_budget must be > 0");
        RR_REQUIRE(cfg->graph_iters >= 0 && cfg->graph_iters <= 4096, "graph_iters must be in [0, 4096]");
        if (cfg->alloc) RR_REQUIRE(cfg->alloc->alloc && cfg->alloc->free, "allocator callbacks are null");
        RR_REQUIRE(cfg->grouped >= 0 && cfg->grouped <= 8, "grouped must be in [0, 8]");
        RR_REQUIRE(cfg->grouped == 0 || (cfg->graph_iters > 0 && cfg->graph_iters <= 256),
                   "grouped batches need graph_iters in [1, 256]");
        require_device();
        int dev = 0;
        RR_HIP(hipGetDevice(&dev));
        Shared sh;
        std::unique_ptr<GroupEngine> engine;
        if (cfg->grouped) {
            engine.reset(new GroupEngine(cfg->graph_iters, cfg->max_slots, cfg->grouped));
            engine->init();
            sh.engine = engine.get();
        }
        const double t0 = wall_s();
        std::vector<std::thread> workers;
        for (int w = 0; w < cfg->max_slots; ++w) {
            workers.emplace_back([&, w]() {
                (void)w;
                (void)hipSetDevice(dev);
                hipStream_t st = nullptr;
                if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) st = nullptr;
                while (true) {
                    Job job;
                    {
                        std::unique_lock<std::mutex> lk(sh.mu);
                        sh.cv_work.wait(lk, [&] { return sh.stop || !sh.admitted.empty(); });
                        if (sh.admitted.empty()) break;
                        job = sh.admitted.front();
                        sh.admitted.pop_front();
                    }
                    run_job(*cfg, job, st, t0, deliver, user, sh);
                }
                if (st) {
                    (void)hipStreamSynchronize(st);
                    release_stream_blocks(st);
                    (void)hipStreamSynchronize(st);
                    (void)hipStreamDestroy(st);
                }
            });
        }
        std::deque<Job> pending;
        bool ended = false;
        rr_status loop_err = RR_OK;
        while (true) {
            const double now = wall_s() - t0;
            if (!ended) {
                while (true) {
                    rr_request r{};
                    const int32_t got = next(user, now, &r);
                    if (got < 0) { ended = true; break; }
                    if (got == 0) break;
                    const bool valid = r.n >= 1 && r.d >= 1 && r.d <= 32 && r.pts && r.B && r.X &&
                                       r.nrhs >= 1 && r.l >= 0 && r.l <= r.n && std::isfinite(r.mu) &&
                                       r.mu >= 0.0 && (r.kind == RR_OP_RBF || r.kind == RR_OP_MATERN32);
                    Job j{r, request_bytes(r, cfg->grouped != 0)};
                    if (!valid || j.bytes > cfg->hbm_budget) {
                        rr_solve_info inf{};
                        inf.status = valid ? RR_ENOMEM : RR_EINVAL;
                        {
                            std::lock_guard<std::mutex> lk(sh.deliver_mu);
                            deliver(user, &r, &inf, wall_s() - t0);
                        }
                        std::lock_guard<std::mutex> lk(sh.mu);
                        sh.rejected += 1;
                        continue;
                    }
                    pending.push_back(j);
                }
            }
            {
                std::unique_lock<std::mutex> lk(sh.mu);
                while (!pending.empty() && sh.active < cfg->max_slots &&
                       sh.used + pending.front().bytes <= cfg->hbm_budget) {
                    Job j = pending.front();
                    pending.pop_front();
                    sh.used += j.bytes;
                    sh.peak = std::max(sh.peak, sh.used);
                    sh.active += 1;
                    sh.max_active = std::max(sh.max_active, sh.active);
                    sh.admitted.push_back(j);
                    sh.cv_work.notify_one();
                }
                if (ended && pending.empty() && sh.active == 0 && sh.admitted.empty()) break;
                sh.cv_done.wait_for(lk, std::chrono::microseconds(200));
            }
        }
        {
            std::lock_guard<std::mutex> lk(sh.mu);
            sh.stop = true;
        }
        sh.cv_work.notify_all();
        for (auto& t : workers) t.join();
        const double wall = wall_s() - t0;
        GroupStats gst{};
        if (engine) {
            gst = engine->stats();
            engine.reset();
        }
        if (stats) {
            std::memset(stats, 0, sizeof(*stats));
            std::vector<double> v = sh.lat_ms;
            std::sort(v.begin(), v.end());
            auto pct = [&](double p) {
                if (v.empty()) return 0.0;
                const size_t k = (size_t)std::min<double>(v.size() - 1, std::floor(p * (v.size() - 1) + 0.5));
                return v[k];
            };
            stats->p50_ms = pct(0.50);
            stats->p99_ms = pct(0.99);
            double s = 0.0;
            for (double q : v) s += q;
            stats->mean_ms = v.empty() ? 0.0 : s / v.size();
            stats->served = sh.served;
            stats->rejected = sh.rejected;
            stats->ok = sh.ok;
            stats->failed = sh.failed;
            stats->graph_fallbacks = sh.graph_fallbacks;
            stats->solves_per_s = wall > 0 ? sh.ok / wall : 0.0;
            stats->hbm_peak = sh.peak;
            stats->max_active = sh.max_active;
            stats->group_replays = gst.replays;
            stats->group_mean = gst.replays > 0 ? (double)gst.jobs / (double)gst.replays : 0.0;
            stats->group_max = (int32_t)gst.max_jobs;
            stats->group_busy_s = gst.busy_s;
            stats->group_wait_s = gst.wait_s;
        }
        (void)loop_err;
        if (sh.first_err != RR_OK) {
            set_error("at least one request failed (see its deliver status); first: " + sh.first_err_msg);
            return sh.first_err;
        }
        return RR_OK;
    });
}
