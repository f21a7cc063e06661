// Batched AMR level: schedule construction (host) and the advance entry point.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
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
};

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

int32_t swe_level_schedule(const swe_patch *patches, int32_t n, int32_t kind, int64_t *lanes,
                           int32_t *pass_rows, int32_t *job_pass, int32_t *n_jobs_out)
{
    using swe::fail;
    if (!patches || n < 1 || !n_jobs_out) return fail(SWE_E_INVAL, "need patches, n >= 1 and n_jobs");
    if (kind != SWE_SCHED_STRIP && kind != SWE_SCHED_PACKED) return fail(SWE_E_INVAL, "unknown schedule kind");
    for (int p = 0; p < n; ++p)
        if (patches[p].nx < 2 || patches[p].ny < 2 || patches[p].offset < 0 || !(patches[p].dx > 0.0) ||
            !(patches[p].dy > 0.0))
            return fail(SWE_E_INVAL, "patch %d: need nx, ny >= 2, offset >= 0, dx, dy > 0", p);

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
    int npass = 0;
    for (auto &j : jobs) npass += (int)j.size();
    *n_jobs_out = (int32_t)jobs.size();
    if (!lanes && !pass_rows && !job_pass) return npass;
    if (!lanes || !pass_rows || !job_pass) return fail(SWE_E_INVAL, "lanes, pass_rows and job_pass go together");
    int q = 0;
    for (size_t j = 0; j < jobs.size(); ++j) {
        job_pass[j] = q;
        for (const Pass &ps : jobs[j]) {
            fill_lanes(ps, (long long *)lanes + (size_t)q * swe::WAVE);
            pass_rows[q] = ps.rows;
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
    la.n_jobs = L->n_jobs;
    la.patches = L->patches;
    la.lanes = (const long long *)L->lanes;
    la.pass_rows = L->pass_rows;
    la.job_pass = L->job_pass;
    la.sync = L->sync;
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
    int cap = swe::level_persistent_capacity();
    if (cap < 1) return fail(SWE_E_HIP, "cannot size the persistent launch");
    int nw = std::min(cap, L->n_jobs);
    hipError_t e = swe::launch_level_persistent(k, la, n_steps, nw, s);
    if (e != hipSuccess) return fail(SWE_E_HIP, "persistent level launch: %s", hipGetErrorString(e));
    return SWE_OK;
}

} // extern "C"
