// Serving loop: admission by device footprint, a pool of worker slots (one
// host thread and one HIP stream each) running the two-phase driver, and a
// first-fit allocator over the caller's device arena.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <vector>

#include "swe.h"
#include "swe_internal.h"

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// First-fit allocator over [0, size) in 256-byte granules.
class Arena {
public:
    explicit Arena(size_t size) { free_.push_back({0, size}); }
    bool alloc(size_t bytes, size_t &off)
    {
        bytes = align256(bytes);
        for (size_t k = 0; k < free_.size(); ++k) {
            if (free_[k].second >= bytes) {
                off = free_[k].first;
                free_[k].first += bytes;
                free_[k].second -= bytes;
                if (free_[k].second == 0) free_.erase(free_.begin() + k);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes)
    {
        bytes = align256(bytes);
        free_.push_back({off, bytes});
        std::sort(free_.begin(), free_.end());
        std::vector<std::pair<size_t, size_t>> merged;
        for (auto &f : free_) {
            if (!merged.empty() && merged.back().first + merged.back().second == f.first)
                merged.back().second += f.second;
            else
                merged.push_back(f);
        }
        free_.swap(merged);
    }

private:
    std::vector<std::pair<size_t, size_t>> free_;   // (offset, size), sorted by offset
};

// Device layout of one request inside its arena block.
struct ReqLayout {
    size_t B, eta0, frames, q[3], flag_acc, maxip, ws, ws_bytes, total;
};

bool layout(const swe_request *r, ReqLayout *L)
{
    const swe_grid &g = r->grid;
    if (g.nx < 2 || g.ny < 1 || g.pitch != g.nx || r->K < 1) return false;
    int ncomp = g.ny > 1 ? 3 : 2;
    size_t plane = (size_t)g.nx * g.ny * sizeof(double);
    size_t off = 0;
    L->B = off; off = align256(off + plane);
    L->eta0 = off; off = align256(off + plane);
    L->frames = off; off = align256(off + plane * (size_t)(r->K + 1) * ncomp);
    for (int c = 0; c < 3; ++c) {
        L->q[c] = off;
        if (c < ncomp) off = align256(off + plane);
    }
    L->flag_acc = off; off = align256(off + (size_t)g.nx * g.ny);
    L->maxip = off; off = align256(off + plane);
    swe_problem pb;
    std::memset(&pb, 0, sizeof pb);
    pb.grid = g;
    pb.params = r->params;
    pb.B = pb.eta0 = pb.frames = (double *)(uintptr_t)256;
    pb.q_out.f0 = pb.q_out.f1 = pb.q_out.f2 = (double *)(uintptr_t)256;
    pb.target_R = r->target_R;
    pb.target_shape = r->target_shape;
    pb.K = r->K;
    pb.t0 = r->t0; pb.ts = r->ts; pb.tf = r->tf; pb.tol = r->tol;
    pb.flag_every = r->flag_every;
    size_t ws = swe_run_workspace_bytes(&pb);
    if (ws == 0) return false;
    L->ws = off;
    L->ws_bytes = ws;
    off = align256(off + ws);
    L->total = off;
    return true;
}

double now_s(std::chrono::steady_clock::time_point t0)
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// Run one request on `stream` inside its block.
swe_status run_one(const swe_request *r, char *base, const ReqLayout &L, hipStream_t s, swe_request_stats *st)
{
    const swe_grid &g = r->grid;
    int ncomp = g.ny > 1 ? 3 : 2;
    size_t n = (size_t)g.nx * g.ny;
    double *B = (double *)(base + L.B), *E = (double *)(base + L.eta0);
    int8_t *acc = (int8_t *)(base + L.flag_acc);
    double *macc = (double *)(base + L.maxip);
#define SERVE_HIP(x)                                                                       \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) return swe::fail(SWE_E_HIP, "%s: %s", #x, hipGetErrorString(e_)); \
    } while (0)
    SERVE_HIP(hipMemcpyAsync(B, r->B_host, n * sizeof(double), hipMemcpyHostToDevice, s));
    SERVE_HIP(hipMemcpyAsync(E, r->eta0_host, n * sizeof(double), hipMemcpyHostToDevice, s));
    SERVE_HIP(hipMemsetAsync(acc, 0, n, s));
    SERVE_HIP(hipMemsetAsync(macc, 0, n * sizeof(double), s));
    swe_problem pb;
    std::memset(&pb, 0, sizeof pb);
    pb.grid = g;
    pb.params = r->params;
    pb.B = B;
    pb.eta0 = E;
    pb.target_xc = r->target_xc; pb.target_yc = r->target_yc; pb.target_R = r->target_R;
    pb.target_shape = r->target_shape;
    pb.K = r->K;
    pb.t0 = r->t0; pb.ts = r->ts; pb.tf = r->tf; pb.tol = r->tol;
    pb.flag_every = r->flag_every;
    pb.frames = (double *)(base + L.frames);
    pb.q_out.f0 = (double *)(base + L.q[0]);
    pb.q_out.f1 = (double *)(base + L.q[1]);
    pb.q_out.f2 = ncomp == 3 ? (double *)(base + L.q[2]) : nullptr;
    pb.flags_at = nullptr;
    pb.flag_acc = acc;
    pb.maxip_acc = macc;
    swe_result res;
    swe_status rs = swe_run(&pb, base + L.ws, L.ws_bytes, &res, s);
    if (rs != SWE_OK) return rs;
    st->n_adj_steps = res.n_adj_steps;
    st->n_fwd_steps = res.n_fwd_steps;
    if (r->flag_acc_host) SERVE_HIP(hipMemcpyAsync(r->flag_acc_host, acc, n, hipMemcpyDeviceToHost, s));
    if (r->maxip_acc_host)
        SERVE_HIP(hipMemcpyAsync(r->maxip_acc_host, macc, n * sizeof(double), hipMemcpyDeviceToHost, s));
    double *qd[3] = {pb.q_out.f0, pb.q_out.f1, pb.q_out.f2};
    for (int c = 0; c < ncomp; ++c)
        if (r->q_host[c]) SERVE_HIP(hipMemcpyAsync(r->q_host[c], qd[c], n * sizeof(double), hipMemcpyDeviceToHost, s));
    SERVE_HIP(hipStreamSynchronize(s));
#undef SERVE_HIP
    return SWE_OK;
}

} // namespace

extern "C" {

size_t swe_serve_footprint(const swe_request *req)
{
    ReqLayout L;
    if (!req || !layout(req, &L)) return 0;
    return L.total;
}

swe_status swe_serve(const swe_request *req, int32_t n, const swe_serve_config *cfg, swe_request_stats *stats)
{
    using swe::fail;
    if (!req || n < 1 || !cfg || !stats) return fail(SWE_E_INVAL, "null argument or n < 1");
    if (!cfg->arena || ((uintptr_t)cfg->arena & 255) || cfg->arena_bytes == 0 || cfg->max_active < 1)
        return fail(SWE_E_INVAL, "need a 256-byte aligned arena and max_active >= 1");
    std::vector<ReqLayout> lay(n);
    for (int k = 0; k < n; ++k) {
        if (!req[k].B_host || !req[k].eta0_host || !layout(&req[k], &lay[k]))
            return fail(SWE_E_INVAL, "request %d: bad grid, inputs or problem", k);
        if (k > 0 && req[k].arrival < req[k - 1].arrival)
            return fail(SWE_E_INVAL, "requests must be ordered by arrival");
        std::memset(&stats[k], 0, sizeof stats[k]);
        stats[k].bytes = lay[k].total;
        stats[k].slot = -1;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return fail(SWE_E_HIP, "no current device");

    const int W = cfg->max_active;
    Arena arena(cfg->arena_bytes);
    std::mutex mu;
    std::condition_variable cv;
    std::deque<int> ready_slots;
    struct Job { int req = -1; size_t off = 0; bool stop = false; };
    std::vector<Job> job(W);
    std::vector<std::condition_variable> slot_cv(W);
    int done_count = 0;
    swe_status first_err = SWE_OK;
    auto t0 = std::chrono::steady_clock::now();

    std::vector<std::thread> workers;
    std::vector<hipStream_t> streams(W, nullptr);
    for (int w = 0; w < W; ++w) {
        if (hipSetDevice(dev) != hipSuccess || hipStreamCreateWithFlags(&streams[w], hipStreamNonBlocking) != hipSuccess) {
            for (int v = 0; v < w; ++v) (void)hipStreamDestroy(streams[v]);
            return fail(SWE_E_HIP, "stream creation failed");
        }
        ready_slots.push_back(w);
    }
    for (int w = 0; w < W; ++w) {
        workers.emplace_back([&, w] {
            (void)hipSetDevice(dev);
            for (;;) {
                Job jb;
                {
                    std::unique_lock<std::mutex> lk(mu);
                    slot_cv[w].wait(lk, [&] { return job[w].req >= 0 || job[w].stop; });
                    if (job[w].stop && job[w].req < 0) return;
                    jb = job[w];
                }
                swe_request_stats st;
                std::memset(&st, 0, sizeof st);
                swe_status rs = run_one(&req[jb.req], (char *)cfg->arena + jb.off, lay[jb.req], streams[w], &st);
                // a failed run may leave work in flight on the block: drain it before the block is reused
                if (rs != SWE_OK) (void)hipStreamSynchronize(streams[w]);
                double fin = now_s(t0);
                swe_request_stats done;
                {
                    std::lock_guard<std::mutex> lk(mu);
                    stats[jb.req].status = rs;
                    stats[jb.req].n_adj_steps = st.n_adj_steps;
                    stats[jb.req].n_fwd_steps = st.n_fwd_steps;
                    stats[jb.req].finished = fin;
                    stats[jb.req].latency = fin - (cfg->realtime ? req[jb.req].arrival : 0.0);
                    done = stats[jb.req];
                    if (rs != SWE_OK && first_err == SWE_OK) first_err = rs;
                    arena.release(jb.off, lay[jb.req].total);
                    job[w].req = -1;
                    ready_slots.push_back(w);
                    ++done_count;
                    cv.notify_all();
                }
                if (cfg->on_done) cfg->on_done(jb.req, &done, cfg->user);
            }
        });
    }

    // admission loop: first come first served; a request too large for the
    // arena is refused, one that does not fit now waits for memory
    int next = 0;
    {
        std::unique_lock<std::mutex> lk(mu);
        while (done_count < n) {
            double now = now_s(t0);
            while (next < n) {
                const swe_request &r = req[next];
                if (lay[next].total > cfg->arena_bytes) {
                    stats[next].status = SWE_E_NOMEM;
                    stats[next].finished = stats[next].admitted = now;
                    if (first_err == SWE_OK) first_err = SWE_E_NOMEM;
                    ++done_count;
                    ++next;
                    continue;
                }
                if (cfg->realtime && r.arrival > now) break;
                if (ready_slots.empty()) break;
                size_t off;
                if (!arena.alloc(lay[next].total, off)) break;
                int w = ready_slots.front();
                ready_slots.pop_front();
                stats[next].admitted = now;
                stats[next].slot = w;
                job[w].req = next;
                job[w].off = off;
                slot_cv[w].notify_one();
                ++next;
            }
            if (done_count >= n) break;
            if (next < n && cfg->realtime && req[next].arrival > now) {
                auto wake = t0 + std::chrono::duration_cast<std::chrono::steady_clock::duration>(
                                     std::chrono::duration<double>(req[next].arrival));
                cv.wait_until(lk, wake);
            } else {
                cv.wait(lk);
            }
        }
        for (int w = 0; w < W; ++w) {
            job[w].stop = true;
            slot_cv[w].notify_one();
        }
    }
    for (auto &t : workers) t.join();
    for (int w = 0; w < W; ++w) (void)hipStreamDestroy(streams[w]);
    if (first_err != SWE_OK) return fail(first_err, "at least one request failed (see stats)");
    return SWE_OK;
}

} // extern "C"
