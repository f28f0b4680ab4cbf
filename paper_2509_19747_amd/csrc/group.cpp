// The serving loop's grouped PCG engine (see group.hpp for the kernels).
//
// Worker threads own their requests (build, restarts with the true residual,
// stopping rules and delivery, exactly as rr_solve_batch).  When a request needs
// its next batch of iterations, its worker calls GroupEngine::run, which queues it
// and waits.  An idle lane of the engine takes every queued request, writes their
// work units and the list headers to the device, and replays one hipGraph of `iters`
// grouped iterations (persistent kernels over the unit lists, work counters zeroed by
// the graph's first node) for all of them at once, then wakes their workers.  Lanes
// run on their own streams, so replays of different groups overlap on the device.
// Each lane captures one graph per set of non-empty lists and keeps it for the
// engine's lifetime; the unit arrays change between replays, the graph does not.
#include "group.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "batch.hpp"
#include "ctx.hpp"
#include "kentry.hpp"
#include "prof.hpp"

namespace rr {

int group_rec_class(int dm) { return dm <= 4 ? 0 : dm <= 8 ? 1 : dm <= 16 ? 2 : 3; }
int group_width_class(int nr) { return nr >= 8 ? 3 : nr >= 4 ? 2 : nr >= 2 ? 1 : 0; }

int group_list_blocks(int list) {
    if (list < GL_FIN) return GROUP_MAT_BLOCKS;
    if (list == GL_FIN) return GROUP_FIN_BLOCKS;
    if (list == GL_BXR || list == GL_BP) return GROUP_VEC_BLOCKS;
    if (list >= GL_QD && list < GL_QD + 4) return GROUP_QD_BLOCKS;
    return GROUP_PROJ_BLOCKS;
}

void launch_group_list(int list, int blocks, const GTable* tab, const GPair* pairs, const GVec* vecs,
                       const GProj* projs, int32_t* ctr, hipStream_t st) {
    if (list < GL_FIN) launch_group_mat(list, blocks, tab, pairs, ctr, st);
    else if (list == GL_FIN) launch_group_fin(blocks, tab, pairs, ctr, st);
    else if (list == GL_BXR) launch_group_vec(false, blocks, tab, vecs, ctr, st);
    else if (list == GL_BP) launch_group_vec(true, blocks, tab, vecs, ctr, st);
    else launch_group_proj(list, blocks, tab, projs, ctr, st);
}

namespace {

// Device image of one replay: the list headers, then the three unit arrays.
struct Layout {
    size_t pairs, vecs, projs, bytes;
    Layout(int mp, int mv, int mj) {
        auto up = [](size_t b) { return (b + 255) & ~(size_t)255; };
        pairs = up(sizeof(GTable));
        vecs = pairs + up((size_t)mp * sizeof(GPair));
        projs = vecs + up((size_t)mv * sizeof(GVec));
        bytes = projs + up((size_t)mj * sizeof(GProj));
    }
};

}  // namespace

struct GroupEngine::Impl {
    struct Job {
        Batch* bt;
        double* X;
        int64_t ldx;
        rr_status status = RR_OK;
        bool done = false;
    };
    // One replay lane: its own stream, device and pinned host images of the unit lists,
    // work counters, graphs and thread.  Lanes take queued batches independently, so
    // a batch that arrives while one replay runs starts on an idle lane at once.
    struct Lane {
        hipStream_t gs = nullptr;
        void* dtab = nullptr;       // device image
        char* htab = nullptr;       // pinned host image
        int32_t* ctr = nullptr;     // iters x GL_COUNT work counters
        std::map<uint64_t, hipGraphExec_t> graphs;
        std::thread th;
    };
    int iters, max_jobs, cap_pairs, cap_vecs, cap_projs;
    Layout lay;
    int dev = 0;
    std::vector<Lane> lanes;
    std::mutex mu;
    std::condition_variable cv_in, cv_out;
    std::deque<Job*> queue;
    bool stop = false;
    GroupStats stats{};

    Impl(int it, int jobs, int nlanes)
        : iters(it), max_jobs(jobs), cap_pairs(jobs * (int)KMULTI_MAX), cap_vecs(jobs),
          cap_projs(jobs * (int)KMULTI_MAX), lay(cap_pairs, cap_vecs, cap_projs), lanes(nlanes) {}

    rr_status init() {
        RR_HIP(hipGetDevice(&dev));
        for (Lane& ln : lanes) {
            RR_HIP(hipStreamCreateWithFlags(&ln.gs, hipStreamNonBlocking));
            RR_HIP(hipMalloc(&ln.dtab, lay.bytes));
            RR_HIP(hipHostMalloc((void**)&ln.htab, lay.bytes, hipHostMallocDefault));
            RR_HIP(hipMalloc((void**)&ln.ctr, (size_t)iters * GL_COUNT * sizeof(int32_t)));
        }
        for (Lane& ln : lanes) ln.th = std::thread([this, &ln]() { loop(ln); });
        return RR_OK;
    }

    ~Impl() {
        {
            std::lock_guard<std::mutex> lk(mu);
            stop = true;
        }
        cv_in.notify_all();
        for (Lane& ln : lanes)
            if (ln.th.joinable()) ln.th.join();
        for (Lane& ln : lanes) {
            for (auto& g : ln.graphs) (void)hipGraphExecDestroy(g.second);
            if (ln.gs) (void)hipStreamSynchronize(ln.gs);
            if (ln.ctr) (void)hipFree(ln.ctr);
            if (ln.dtab) (void)hipFree(ln.dtab);
            if (ln.htab) (void)hipHostFree(ln.htab);
            if (ln.gs) (void)hipStreamDestroy(ln.gs);
        }
    }

    rr_status run(Batch& bt, double* X, int64_t ldx) {
        RR_HIP(hipStreamSynchronize(bt.st));   // the request's own work precedes the replay
        Job job{&bt, X, ldx};
        const double t0 = now_ms();
        std::unique_lock<std::mutex> lk(mu);
        RR_REQUIRE(!stop, "the grouped engine has stopped");
        queue.push_back(&job);
        cv_in.notify_one();
        cv_out.wait(lk, [&] { return job.done; });
        stats.wait_s += 1e-3 * (now_ms() - t0);
        if (job.status != RR_OK) set_error("grouped PCG replay failed on the device");
        return job.status;
    }

    // Work units of the taken jobs, written into the host image; returns the mask of
    // non-empty lists.
    uint64_t describe(const std::vector<Job*>& jobs, char* htab) {
        GTable& tab = *reinterpret_cast<GTable*>(htab);
        std::memset(&tab, 0, sizeof(tab));
        GPair* pairs = reinterpret_cast<GPair*>(htab + lay.pairs);
        GVec* vecs = reinterpret_cast<GVec*>(htab + lay.vecs);
        GProj* projs = reinterpret_cast<GProj*>(htab + lay.projs);
        // column blocks, sorted by product list (kind, record class, width); finish over all
        int np = 0, wf = 0;
        for (int L = GL_MAT; L < GL_FIN; ++L) {
            tab.list[L].off = np;
            int w = 0;
            for (Job* j : jobs) {
                Batch& b = *j->bt;
                const KernelOp k = kernel_op_of(b.P);
                const KmmaPlanInfo pl = kernel_mma_plan_info(b.n);
                const int nfb = kernel_matvec_blocks(b.n);
                for (int64_t c0 = 0; c0 < b.m;) {
                    const int nr = Batch::mat_width(b.m, c0, k.dm);
                    if (L == group_mat_list(k.kind, k.dm, nr)) {
                        GPair& g = pairs[np++];
                        g.xa = k.xa;
                        g.sqn = k.sqn;
                        g.u = b.Pm.as<double>() + c0 * b.n;
                        g.part = b.gpart.as<double>() + (size_t)c0 * b.gpart_doubles;
                        g.y = b.W.as<double>() + c0 * b.n;
                        g.dot = b.kdot.as<double>() + c0 * nfb;
                        g.st = b.state.as<BState>() + c0;
                        g.n = b.n;
                        g.scale = k.scale;
                        g.mu = b.mu1;
                        g.c = kernel_c32(k.kind, k.kconst);
                        g.nr = nr;
                        g.ncols = (int32_t)std::min<int64_t>(nr, b.m - c0);
                        g.nb = pl.nb;
                        g.m = pl.m;
                        g.S = pl.S;
                        g.nfb = nfb;
                        g.w_mat = w;
                        g.w_fin = wf;
                        w += (int)pl.items;
                        wf += nfb;
                    }
                    c0 += nr;
                }
            }
            tab.list[L].count = np - tab.list[L].off;
            tab.list[L].total = w;
        }
        tab.list[GL_FIN] = GList{0, np, wf, 0};
        // requests
        int nv = 0, wv = 0;
        for (Job* j : jobs) {
            Batch& b = *j->bt;
            GVec& v = vecs[nv++];
            const int nfb = kernel_matvec_blocks(b.n), nbq = qd_blocks(b.n);
            v.n = b.n;
            v.ldx = j->ldx;
            v.X = j->X;
            v.R = b.R.as<double>();
            v.P = b.Pm.as<double>();
            v.W = b.W.as<double>();
            v.Z = b.Z.as<double>();
            v.st = b.state.as<BState>();
            v.pw = ColParts{b.kdot.as<double>(), nfb, 1, nfb};
            v.rz = ColParts{b.rzp.as<double>(), nbq, 1, nbq};
            v.rr_part = b.rrp.as<double>();
            v.cnt = b.cnt.as<int32_t>();
            v.m = (int32_t)b.m;
            v.nbx = bxr_blocks(b.n);
            v.w0 = wv;
            wv += v.nbx * v.m;
        }
        tab.list[GL_BXR] = GList{0, nv, wv, 0};
        tab.list[GL_BP] = GList{0, nv, wv, 0};
        // projection groups, sorted by width; the core list runs over all of them
        int nj = 0, wc = 0;
        for (int wcls = 0; wcls < 4; ++wcls) {
            const int LG = GL_GEMV + wcls, LQ = GL_QD + wcls;
            tab.list[LG].off = tab.list[LQ].off = nj;
            int wg = 0, wq = 0;
            for (Job* j : jobs) {
                Batch& b = *j->bt;
                const double* Kc = b.P.per[b.mus_used[0]].Kc.as<double>();
                const int nbq = qd_blocks(b.n);
                const int64_t rpc = gemv_t_rows_per_chunk_of(b.n, b.kb);
                for (int64_t c0 = 0; c0 < b.m;) {
                    const int nr = b.group_width(c0);
                    if (group_width_class(nr) == wcls) {
                        GProj& g = projs[nj++];
                        g.n = b.n;
                        g.k = b.kb;
                        g.Q = b.P.Qb.as<double>();
                        g.Kc = Kc;
                        g.R = b.R.as<double>() + c0 * b.n;
                        g.cpart = b.gcpart.as<double>() + (size_t)c0 * b.gch * b.kb;
                        g.D = b.gdcols.as<double>() + (size_t)c0 * b.kb;
                        g.Z = b.Z.as<double>() + c0 * b.n;
                        g.rz = b.rzp.as<double>() + c0 * nbq;
                        g.st = b.state.as<BState>() + c0;
                        g.rpc = rpc;
                        g.nr = nr;
                        g.nch = b.gch;
                        g.cblk = (int32_t)((b.kb + 3) / 4);
                        g.nbq = nbq;
                        g.w_gemv = wg;
                        g.w_qd = wq;
                        g.w_core = wc;
                        wg += g.cblk * g.nch;
                        wq += nbq;
                        wc += (int32_t)((b.kb + 3) / 4) * nr;
                    }
                    c0 += nr;
                }
            }
            tab.list[LG].count = tab.list[LQ].count = nj - tab.list[LG].off;
            tab.list[LG].total = wg;
            tab.list[LQ].total = wq;
        }
        tab.list[GL_CORE] = GList{0, nj, wc, 0};
        uint64_t mask = 0;
        for (int L = 0; L < GL_COUNT; ++L)
            if (tab.list[L].total > 0) mask |= 1ull << L;
        return mask;
    }

    static int prof_slot(int list) {
        if (list < GL_FIN) return PROF_GROUP_PRODUCT;
        if (list == GL_FIN) return PROF_GROUP_FINISH;
        if (list == GL_BXR || list == GL_BP) return PROF_GROUP_UPDATE;
        return PROF_GROUP_PROJECT;
    }

    // The launches of one replay on the engine stream: counter reset, then per
    // iteration the products (widest blocks first), their finish, the x and r update,
    // the projection and the p update.  timed: one event span per iteration and class.
    void launch_lists(Lane& ln, uint64_t mask, bool timed, bool sized) {
        const GTable& htb = *reinterpret_cast<const GTable*>(ln.htab);
        const GTable* tab = reinterpret_cast<const GTable*>(ln.dtab);
        const GPair* pairs = reinterpret_cast<const GPair*>((char*)ln.dtab + lay.pairs);
        const GVec* vecs = reinterpret_cast<const GVec*>((char*)ln.dtab + lay.vecs);
        const GProj* projs = reinterpret_cast<const GProj*>((char*)ln.dtab + lay.projs);
        hipStream_t gs = ln.gs;
        int32_t* ctr = ln.ctr;
        launch_group_reset(ctr, iters * GL_COUNT, gs);
        for (int k = 0; k < iters; ++k) {
            int L = 0;
            while (L < GL_COUNT) {
                const int slot = prof_slot(L < GL_FIN ? GL_FIN - 1 - L : L);
                ProfScope ps(timed ? slot : -1, gs);
                for (; L < GL_COUNT; ++L) {
                    const int list = L < GL_FIN ? GL_FIN - 1 - L : L;
                    if (prof_slot(list) != slot) break;
                    if (!(mask & (1ull << list))) continue;
                    // sized: as many blocks as the list has work items, up to the cap
                    const int cap = group_list_blocks(list);
                    const int blocks = sized ? std::max(1, std::min(cap, htb.list[list].total)) : cap;
                    launch_group_list(list, blocks, tab, pairs, vecs, projs, ctr + k * GL_COUNT + list, gs);
                }
            }
        }
    }

    // The replay graph for the lists in mask (captured on first use).
    hipGraphExec_t graph_for(Lane& ln, uint64_t mask) {
        auto it = ln.graphs.find(mask);
        if (it != ln.graphs.end()) return it->second;
        hipGraph_t g = nullptr;
        hipGraphExec_t e = nullptr;
        // relaxed: other threads allocate and launch while the engine captures
        if (hipStreamBeginCapture(ln.gs, hipStreamCaptureModeRelaxed) != hipSuccess) return nullptr;
        launch_lists(ln, mask, false, false);
        const hipError_t ce = hipStreamEndCapture(ln.gs, &g);
        if (ce != hipSuccess || !g) {
            (void)hipGetLastError();
            if (g) (void)hipGraphDestroy(g);
            return nullptr;
        }
        const hipError_t ie = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ie != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        ln.graphs[mask] = e;
        return e;
    }

    void loop(Lane& ln) {
        (void)hipSetDevice(dev);
        while (true) {
            std::vector<Job*> jobs;
            {
                std::unique_lock<std::mutex> lk(mu);
                cv_in.wait(lk, [&] { return stop || !queue.empty(); });
                if (queue.empty()) break;
                while (!queue.empty() && (int)jobs.size() < max_jobs) {
                    jobs.push_back(queue.front());
                    queue.pop_front();
                }
            }
            rr_status s = RR_OK;
            const double t0 = now_ms();
            const uint64_t mask = describe(jobs, ln.htab);
            hipGraphExec_t e = nullptr;
            bool ok = hipMemcpyAsync(ln.dtab, ln.htab, lay.bytes, hipMemcpyHostToDevice, ln.gs) == hipSuccess;
            if (ok && prof_enabled()) {
                // kernel timing: the same kernels as plain launches, grids sized to the
                // work, one timed span per iteration and class
                launch_lists(ln, mask, true, true);
                ok = hipGetLastError() == hipSuccess;
            } else if (ok) {
                ok = (e = graph_for(ln, mask)) != nullptr && hipGraphLaunch(e, ln.gs) == hipSuccess;
            }
            if (!ok || hipStreamSynchronize(ln.gs) != hipSuccess) {
                (void)hipGetLastError();
                s = RR_EDEVICE;
            }
            const double t1 = now_ms();
            std::lock_guard<std::mutex> lk(mu);
            stats.busy_s += 1e-3 * (t1 - t0);
            stats.replays += 1;
            stats.jobs += (int64_t)jobs.size();
            stats.max_jobs = std::max<int64_t>(stats.max_jobs, (int64_t)jobs.size());
            for (Job* j : jobs) {
                j->status = s;
                j->done = true;
            }
            cv_out.notify_all();
        }
    }
};

GroupEngine::GroupEngine(int iters, int max_jobs, int lanes) : impl_(new Impl(iters, max_jobs, lanes)) {}
GroupEngine::~GroupEngine() { delete impl_; }
rr_status GroupEngine::init() { return impl_->init(); }
rr_status GroupEngine::run(Batch& bt, double* X, int64_t ldx) { return impl_->run(bt, X, ldx); }
GroupStats GroupEngine::stats() {
    std::lock_guard<std::mutex> lk(impl_->mu);
    return impl_->stats;
}

}  // namespace rr
