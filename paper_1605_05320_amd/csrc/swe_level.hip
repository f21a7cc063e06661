// Batched AMR level: schedule construction (host) and the advance entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "swe.h"
#include "swe_device.h"
#include "swe_internal.h"

namespace {

// A strip of a patch: columns c0 .. c0 + ncols - 1 (at most STRIP of them),
// occupying ncols + 4 lanes (two ghost columns each side).
struct Seg {
    int patch, c0, ncols, ny;
    int width() const { return ncols + 2 * swe::HALO; }
};

struct Pass {
    std::vector<Seg> segs;
    int used = 0;
    int rows = 0;
    int row0 = 0;
};

// The current device's CU count and co-resident persistent workgroups,
// queried once per device (the occupancy query costs host time on every
// call, which a timed persistent advance would otherwise include).
bool persistent_sizes(int &cus, int &cap)
{
    static std::mutex m;
    static std::map<int, std::pair<int, int>> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    std::lock_guard<std::mutex> lock(m);
    auto it = cache.find(dev);
    if (it == cache.end()) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1)
            return false;
        const int k = swe::level_persistent_capacity();
        if (k < 1) return false;
        it = cache.emplace(dev, std::make_pair(c, k)).first;
    }
    cus = it->second.first;
    cap = it->second.second;
    return true;
}

long long lane_code(int patch, int role, int col)
{
    return ((long long)patch << 32) | ((long long)role << 16) | (long long)(col + 32768);
}

void fill_lanes(const Pass &p, long long *out)
{
    for (int l = 0; l < swe::WAVE; ++l) out[l] = -1;
    int l = 0;
    for (const Seg &s : p.segs) {
        for (int o = 0; o < s.width(); ++o, ++l) {
            int col = s.c0 + o - swe::HALO;
            int role = 0;
            if (o >= swe::HALO && o < swe::HALO + s.ncols) role |= 1;
            if (o >= swe::HALO && o <= swe::HALO + s.ncols) role |= 2;
            out[l] = lane_code(s.patch, role, col);
        }
    }
}

} // namespace

extern "C" {

int32_t swe_level_schedule(const swe_patch *patches, int32_t n, int32_t kind, int32_t chunk_rows, int64_t *lanes,
                           int32_t *pass_rows, int32_t *pass_row0, int32_t *job_pass, int32_t *n_jobs_out)
{
    using swe::fail;
    if (!patches || n < 1 || !n_jobs_out) return fail(SWE_E_INVAL, "need patches, n >= 1 and n_jobs");
    if (kind != SWE_SCHED_STRIP && kind != SWE_SCHED_PACKED) return fail(SWE_E_INVAL, "unknown schedule kind");
    if (chunk_rows < 0) return fail(SWE_E_INVAL, "chunk_rows must be >= 0");
    for (int p = 0; p < n; ++p)
        if (patches[p].nx < 2 || patches[p].ny < 2 || patches[p].offset < 0 || !(patches[p].dx > 0.0) ||
            !(patches[p].dy > 0.0))
            return fail(SWE_E_INVAL, "patch %d: need nx, ny >= 2, offset >= 0, dx, dy > 0", p);
    for (int p = 0; p < n; ++p)
        for (int k = 0; k < 4; ++k)
            if (patches[p].bc[k] != SWE_BC_WALL && patches[p].bc[k] != SWE_BC_EXTRAP)
                return fail(SWE_E_INVAL, "patch %d: bc[%d] = %d is not a boundary condition", p, k, patches[p].bc[k]);

    // jobs: lists of passes; a patch never spans two jobs
    std::vector<std::vector<Pass>> jobs;
    std::vector<Seg> small;   // single-strip patches (packable)
    for (int p = 0; p < n; ++p) {
        const swe_patch &pt = patches[p];
        int nstrip = (pt.nx + swe::STRIP - 1) / swe::STRIP;
        if (nstrip == 1 && kind == SWE_SCHED_PACKED) {
            small.push_back({p, 0, pt.nx, pt.ny});
            continue;
        }
        std::vector<Pass> job;
        for (int k = 0; k < nstrip; ++k) {
            Pass ps;
            Seg s{p, k * swe::STRIP, std::min(swe::STRIP, pt.nx - k * swe::STRIP), pt.ny};
            ps.segs.push_back(s);
            ps.used = s.width();
            ps.rows = pt.ny;
            job.push_back(ps);
        }
        jobs.push_back(job);
    }
    if (kind == SWE_SCHED_PACKED) {
        // first-fit decreasing by width within groups of equal row count
        std::sort(small.begin(), small.end(), [](const Seg &a, const Seg &b) {
            if (a.ny != b.ny) return a.ny > b.ny;
            if (a.ncols != b.ncols) return a.ncols > b.ncols;
            return a.patch < b.patch;
        });
        size_t i = 0;
        while (i < small.size()) {
            size_t j = i;
            while (j < small.size() && small[j].ny == small[i].ny) ++j;
            std::vector<Pass> open;
            for (size_t k = i; k < j; ++k) {
                const Seg &s = small[k];
                bool placed = false;
                for (Pass &ps : open)
                    if (ps.used + s.width() <= swe::WAVE) {
                        ps.segs.push_back(s);
                        ps.used += s.width();
                        placed = true;
                        break;
                    }
                if (!placed) {
                    Pass ps;
                    ps.segs.push_back(s);
                    ps.used = s.width();
                    ps.rows = s.ny;
                    open.push_back(ps);
                }
            }
            for (Pass &ps : open) jobs.push_back({ps});
            i = j;
        }
        // longest jobs first (cost: marched rows plus the warm-up of each pass)
        std::stable_sort(jobs.begin(), jobs.end(), [](const std::vector<Pass> &a, const std::vector<Pass> &b) {
            double ca = 0, cb = 0;
            for (const Pass &p : a) ca += p.rows + 2.5;
            for (const Pass &p : b) cb += p.rows + 2.5;
            return ca > cb;
        });
    }
    if (chunk_rows > 0) {
        // cut tall passes into row chunks, each chunk a job of its own
        std::vector<std::vector<Pass>> cut;
        for (auto &j : jobs)
            for (const Pass &ps : j) {
                if (ps.rows <= chunk_rows) {
                    cut.push_back({ps});
                    continue;
                }
                for (int r0 = 0; r0 < ps.rows; r0 += chunk_rows) {
                    Pass c = ps;
                    c.row0 = r0;
                    c.rows = std::min(chunk_rows, ps.rows - r0);
                    cut.push_back({c});
                }
            }
        std::stable_sort(cut.begin(), cut.end(), [](const std::vector<Pass> &a, const std::vector<Pass> &b) {
            return a[0].rows > b[0].rows;
        });
        jobs.swap(cut);
    }
    int npass = 0;
    for (auto &j : jobs) npass += (int)j.size();
    *n_jobs_out = (int32_t)jobs.size();
    if (!lanes && !pass_rows && !pass_row0 && !job_pass) return npass;
    if (!lanes || !pass_rows || !pass_row0 || !job_pass)
        return fail(SWE_E_INVAL, "lanes, pass_rows, pass_row0 and job_pass go together");
    int q = 0;
    for (size_t j = 0; j < jobs.size(); ++j) {
        job_pass[j] = q;
        for (const Pass &ps : jobs[j]) {
            fill_lanes(ps, (long long *)lanes + (size_t)q * swe::WAVE);
            pass_rows[q] = ps.rows;
            pass_row0[q] = ps.row0;
            ++q;
        }
    }
    job_pass[jobs.size()] = q;
    return npass;
}

swe_status swe_level_advance(const swe_level *L, const swe_params *prm, const double *B, swe_fields a,
                             swe_fields b, swe_ctl *ctl, int32_t n_steps, int32_t persistent, void *stream)
{
    using swe::fail;
    if (!L || !prm || !B || !ctl) return fail(SWE_E_INVAL, "level, params, B or ctl is NULL");
    if (!L->patches || !L->lanes || !L->pass_rows || !L->job_pass) return fail(SWE_E_INVAL, "level tables missing");
    if (L->n_patches < 1 || L->n_passes < 1 || L->n_jobs < 1 || n_steps < 0) return fail(SWE_E_INVAL, "bad level sizes");
    if (!a.f0 || !a.f1 || !a.f2 || !b.f0 || !b.f1 || !b.f2) return fail(SWE_E_INVAL, "null state plane");
    if (a.f0 == b.f0 || a.f1 == b.f1 || a.f2 == b.f2) return fail(SWE_E_INVAL, "a and b alias");
    if (prm->model != SWE_NONLINEAR || (prm->order != 1 && prm->order != 2) ||
        (prm->transverse != 0 && prm->transverse != 1) || !(prm->cfl_desired > 0.0) ||
        !(prm->cfl_max >= prm->cfl_desired))
        return fail(SWE_E_INVAL, "bad parameters (nonlinear model, order, transverse, 0 < cfl_desired <= cfl_max)");
    if (!swe::params_in_range(prm))
        return fail(SWE_E_INVAL, "g = %g and dry_tol = %g must lie in [1e-100, 1e100]", prm->g, prm->dry_tol);
    if (persistent && !L->sync) return fail(SWE_E_INVAL, "persistent mode needs the sync words");
    if (n_steps == 0) return SWE_OK;

    swe::KParams k;
    std::memset(&k, 0, sizeof k);
    k.order = prm->order;
    k.transverse = prm->transverse;
    k.g = prm->g;
    k.sea_level = prm->sea_level;
    k.dry_tol = prm->dry_tol;
    k.B = B;
    k.in0 = a.f0; k.in1 = a.f1; k.in2 = a.f2;
    k.out0 = b.f0; k.out1 = b.f1; k.out2 = b.f2;
    k.ctl = ctl;
    k.cfl_desired = prm->cfl_desired;
    k.cfl_max = prm->cfl_max;
    k.n_clamped = &ctl->n_clamped;
    k.n_nonfinite = &ctl->n_nonfinite;
    swe::LevelArgs la;
    la.n_passes = L->n_passes;
    la.patches = L->patches;
    la.lanes = (const long long *)L->lanes;
    la.pass_rows = L->pass_rows;
    la.sync = L->sync;
    la.pass_row0 = L->pass_row0;
    hipStream_t s = (hipStream_t)stream;
    if (!persistent) {
        for (int n = 0; n < n_steps; ++n) {
            k.attempt = n;
            hipError_t e = swe::launch_level_step(k, la, s);
            if (e != hipSuccess) return fail(SWE_E_HIP, "level step launch: %s", hipGetErrorString(e));
        }
        hipError_t e = swe::launch_ctl_finish(ctl, n_steps, prm->cfl_desired, prm->cfl_max, s);
        if (e != hipSuccess) return fail(SWE_E_HIP, "control launch: %s", hipGetErrorString(e));
        return SWE_OK;
    }
    int cus = 0, cap = 0;
    if (!persistent_sizes(cus, cap)) return fail(SWE_E_HIP, "cannot size the persistent launch");
    // Eight passes per workgroup, but at least one workgroup per CU while
    // there are passes for them: a level of few passes packed into few
    // workgroups would put up to eight marches on the four SIMDs of one CU
    // (measured, 20 steps: four 80-128-cell patches in 16-row chunks 67.8 ->
    // 45.9 us per step, 256 patches 71.3 -> 57.3; 3000 patches unchanged).
    int nw = std::min(cap, std::max((L->n_passes + swe::LVL_WAVES - 1) / swe::LVL_WAVES, std::min(L->n_passes, cus)));
    hipError_t e = swe::launch_level_persistent(k, la, n_steps, nw, s);
    if (e != hipSuccess) return fail(SWE_E_HIP, "persistent level launch: %s", hipGetErrorString(e));
    return SWE_OK;
}

swe_status swe_level_tune(const swe_level *const *levels, int32_t n_levels, const swe_params *prm, const double *B,
                          swe_fields init, swe_fields work_a, swe_fields work_b, swe_fields ref, swe_ctl *ctl,
                          int32_t *mismatch, double dt, int32_t n_trial, int64_t n_cells, swe_tune_entry *out,
                          int32_t *best, void *stream)
{
    using swe::fail;
    if (!levels || n_levels < 1 || !prm || !B || !ctl || !mismatch || !out || !best)
        return fail(SWE_E_INVAL, "null argument");
    if (!(dt > 0.0) || n_trial < 1 || n_cells < 1) return fail(SWE_E_INVAL, "need dt > 0, n_trial >= 1, n_cells >= 1");
    if (!init.f0 || !init.f1 || !init.f2 || !ref.f0 || !ref.f1 || !ref.f2) return fail(SWE_E_INVAL, "null plane");
    hipStream_t s = (hipStream_t)stream;
    size_t bytes = (size_t)n_cells * sizeof(double);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return fail(SWE_E_HIP, "event creation failed");
    }
#define TUNE_HIP(expr)                                                                  \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) return fail(SWE_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)
    double best_us = 1e300;
    int nout = 0;
    bool have_ref = false;
    auto run_candidate = [&](int k, int pers) -> swe_status {
        swe_status st;
        const double *src[3] = {init.f0, init.f1, init.f2};
        double *dst[3] = {work_a.f0, work_a.f1, work_a.f2};
        // one untimed attempt first, so that one-time costs of a launch form
        // (loading its kernel, sizing the cooperative launch) are not timed
        for (int c = 0; c < 3; ++c) TUNE_HIP(hipMemcpyAsync(dst[c], src[c], bytes, hipMemcpyDeviceToDevice, s));
        if ((st = swe_ctl_set(ctl, 0.0, dt, 1.0e300, 0, stream)) != SWE_OK) return st;
        if ((st = swe_level_advance(levels[k], prm, B, work_a, work_b, ctl, 1, pers, stream)) != SWE_OK) return st;
        for (int c = 0; c < 3; ++c) TUNE_HIP(hipMemcpyAsync(dst[c], src[c], bytes, hipMemcpyDeviceToDevice, s));
        if ((st = swe_ctl_set(ctl, 0.0, dt, 1.0e300, 0, stream)) != SWE_OK) return st;
        TUNE_HIP(hipStreamSynchronize(s));
        TUNE_HIP(hipEventRecord(e0, s));
        if ((st = swe_level_advance(levels[k], prm, B, work_a, work_b, ctl, n_trial, pers, stream)) != SWE_OK)
            return st;
        TUNE_HIP(hipEventRecord(e1, s));
        TUNE_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        TUNE_HIP(hipEventElapsedTime(&ms, e0, e1));
        swe_ctl hc;
        uint32_t syncw[4] = {0, 0, 0, 0};
        TUNE_HIP(hipMemcpy(&hc, ctl, sizeof hc, hipMemcpyDeviceToHost));
        if (levels[k]->sync) TUNE_HIP(hipMemcpy(syncw, levels[k]->sync, sizeof syncw, hipMemcpyDeviceToHost));
        if (syncw[2]) return fail(SWE_E_HIP, "persistent level barrier timed out");
        swe_fields cur = hc.s.cur ? work_b : work_a;
        double *cp[3] = {cur.f0, cur.f1, cur.f2};
        double *rp[3] = {ref.f0, ref.f1, ref.f2};
        if (!have_ref) {
            for (int c = 0; c < 3; ++c) TUNE_HIP(hipMemcpyAsync(rp[c], cp[c], bytes, hipMemcpyDeviceToDevice, s));
            TUNE_HIP(hipStreamSynchronize(s));
            have_ref = true;
        } else {
            TUNE_HIP(hipMemsetAsync(mismatch, 0, sizeof(int32_t), s));
            for (int c = 0; c < 3; ++c) TUNE_HIP(swe::launch_count_diff(cp[c], rp[c], n_cells, mismatch, s));
            int32_t hm = 0;
            TUNE_HIP(hipMemcpyAsync(&hm, mismatch, sizeof hm, hipMemcpyDeviceToHost, s));
            TUNE_HIP(hipStreamSynchronize(s));
            if (hm != 0)
                return fail(SWE_E_HIP, "schedule %d (persistent %d) differs from the first in %d values", k, pers, hm);
        }
        double us = ms * 1e3 / n_trial;
        out[nout].level = k;
        out[nout].persistent = pers;
        out[nout].us_per_attempt = us;
        if (us < best_us) {
            best_us = us;
            *best = nout;
        }
        ++nout;
        return SWE_OK;
    };
#undef TUNE_HIP
    swe_status st = SWE_OK;
    for (int k = 0; k < n_levels && st == SWE_OK; ++k)
        for (int pers = 0; pers < 2 && st == SWE_OK; ++pers) st = run_candidate(k, pers);
    hipError_t es = hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st == SWE_OK && es != hipSuccess) st = fail(SWE_E_HIP, "synchronisation failed: %s", hipGetErrorString(es));
    return st;
}

} // extern "C"
