// C ABI entry points declared in include/swe.h: argument validation, launch
// of the kernels, and the two-phase driver.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>

#include "swe.h"
#include "swe_device.h"
#include "swe_internal.h"

namespace {
thread_local char g_err[512] = "";
}

namespace swe {
swe_status fail(swe_status st, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return st;
}
} // namespace swe

namespace {
using swe::fail;

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(SWE_E_HIP, "%s: %s", #expr, hipGetErrorString(e_));           \
    } while (0)

// Wavefront slots of the step kernel on the current device: 4 SIMDs per CU,
// 2 resident wavefronts per SIMD (register-limited).
int wave_slots()
{
    static const int slots = [] {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
        return cus * 4 * 2;
    }();
    return slots;
}

// Rows marched per wavefront: ly, and ly + 1 for the first lyr chunks of a
// strip; heights differ by at most one row.  A march's time is its rows plus
// a warm-up of about 2.5 rows, and a wavefront alone on its SIMD runs faster
// than each of a pair (measured on 1024^2 with 103 marches of 10 rows per
// strip: alone 30 us, a pair 30 and 47 us).  Busy steps, graph replays:
//  * grids small enough for one-row marches with one wavefront per SIMD take
//    them (96^2 to 224^2: 7.8-8.5 us against 10.0-10.8 us at 2 rows);
//  * otherwise the most chunks of at least 2 rows that fill the resident
//    slots, two wavefronts per SIMD (11.5 us at 2 rows against 24.6 us at 8
//    on 256^2, 20.0 against 25.7 us at 3 and 8 rows on 512^2) -
//  * - unless that leaves between one and one and a half wavefronts per SIMD,
//    where some SIMDs hold pairs that set the launch's time while the others
//    idle: then one wavefront per SIMD with taller marches (352^2 to 416^2:
//    13.5-13.9 us at 3 rows against 14.5-15.0 us at 2);
//  * a launch whose single wave of wavefronts would need marches of more than
//    56 rows takes marches of 23-24 rows instead, in several waves (2048^2
//    with waves on every edge: 36 rows in one wave 135 us, 24 rows 151 us;
//    2560^2: 54-55 rows 205 us, 24 rows 230 us; 24 rows best of 16 to 138 on
//    4096^2, and equal to 78 rows on 3072^2).
// SWE_MARCH_ROWS forces ly rows for every chunk, SWE_MARCH_CHUNKS the number
// of balanced chunks per strip (tuning sweeps).
void march_rows(int nx, int ny, int &ly, int &lyr)
{
    static const int forced = [] {
        const char *e = std::getenv("SWE_MARCH_ROWS");
        int v = e ? std::atoi(e) : 0;
        return (v >= 1 && v <= 4096) ? v : 0;
    }();
    static const int forced_chunks = [] {
        const char *e = std::getenv("SWE_MARCH_CHUNKS");
        int v = e ? std::atoi(e) : 0;
        return (v >= 1 && v <= (1 << 20)) ? v : 0;
    }();
    lyr = 0;
    if (forced > 0) { ly = forced; return; }
    const long long strips = (nx + swe::STRIP - 1) / swe::STRIP;
    const long long slots = wave_slots(), simds = slots / 2;
    long long c;
    if (forced_chunks > 0) {
        c = std::min<long long>(forced_chunks, ny);
    } else if (strips * ny <= simds) {
        c = ny;
    } else {
        c = std::min<long long>(slots / strips, ny / 2);
        if (c >= 1 && strips * c > simds && 2 * strips * c < 3 * simds) c = simds / strips;
        if (c < 1 || (ny + c - 1) / c > 56) c = (ny + 23) / 24;
    }
    ly = (int)(ny / c);
    lyr = (int)(ny % c);
}

// Chunks of a strip for march heights ly, lyr.
int march_chunks(int ny, int ly, int lyr)
{
    return lyr > 0 ? (ny - lyr) / ly : (ny + ly - 1) / ly;
}

// XCD-aware tile placement pays when all wavefronts of the launch are
// resident together (halo rows then come from the shared L2); for larger
// launches it concentrates each XCD on a narrow band of memory and is off.
// SWE_XCD_REMAP=0/1 forces it.
int xcd_remap_for(int nx, int nchunks)
{
    static const int forced = [] {
        const char *e = std::getenv("SWE_XCD_REMAP");
        return e ? (std::atoi(e) != 0 ? 1 : 0) : -1;
    }();
    if (forced >= 0) return forced;
    long long waves = (long long)((nx + swe::STRIP - 1) / swe::STRIP) * nchunks;
    return waves <= wave_slots() ? 1 : 0;
}

swe_status check_grid(const swe_grid *g)
{
    if (!g) return fail(SWE_E_INVAL, "grid is NULL");
    if (g->nx < 2) return fail(SWE_E_INVAL, "nx = %d < 2", g->nx);
    if (g->ny < 1) return fail(SWE_E_INVAL, "ny = %d < 1", g->ny);
    if (g->pitch < g->nx) return fail(SWE_E_INVAL, "pitch %d < nx %d", g->pitch, g->nx);
    // a row's bytes must fit the 32-bit range of the step kernel's row stores
    if (g->nx > SWE_MAX_NX) return fail(SWE_E_INVAL, "nx = %d > %d", g->nx, SWE_MAX_NX);
    if ((long long)g->ny * g->pitch > (1LL << 40)) return fail(SWE_E_INVAL, "grid too large");
    if (!(g->dx > 0.0) || !std::isfinite(g->dx)) return fail(SWE_E_INVAL, "dx must be > 0");
    if (g->ny > 1 && (!(g->dy > 0.0) || !std::isfinite(g->dy))) return fail(SWE_E_INVAL, "dy must be > 0");
    for (int k = 0; k < 4; ++k)
        if (g->bc[k] != SWE_BC_WALL && g->bc[k] != SWE_BC_EXTRAP)
            return fail(SWE_E_INVAL, "bc[%d] = %d is not a boundary condition", k, g->bc[k]);
    return SWE_OK;
}

swe_status check_params(const swe_params *p)
{
    if (!p) return fail(SWE_E_INVAL, "params is NULL");
    if (p->order != 1 && p->order != 2) return fail(SWE_E_INVAL, "order must be 1 or 2");
    if (p->transverse != 0 && p->transverse != 1) return fail(SWE_E_INVAL, "transverse must be 0 or 1");
    if (!swe::params_in_range(p))
        return fail(SWE_E_INVAL, "g = %g and dry_tol = %g must lie in [1e-100, 1e100]", p->g, p->dry_tol);
    if (!std::isfinite(p->sea_level)) return fail(SWE_E_INVAL, "sea_level must be finite");
    if (p->model != SWE_NONLINEAR && p->model != SWE_LINEAR) return fail(SWE_E_INVAL, "unknown model");
    return SWE_OK;
}

swe_status check_fields(const swe_grid *g, swe_fields f, const char *what)
{
    if (!f.f0 || !f.f1) return fail(SWE_E_INVAL, "%s: null plane", what);
    if (g->ny > 1 && !f.f2) return fail(SWE_E_INVAL, "%s: null plane f2 in 2D", what);
    return SWE_OK;
}

bool overlaps(const void *a, const void *b, size_t bytes)
{
    const char *pa = (const char *)a, *pb = (const char *)b;
    return pa < pb + bytes && pb < pa + bytes;
}

swe_status check_alias(const swe_grid *g, swe_fields in, swe_fields out)
{
    size_t bytes = (size_t)g->ny * g->pitch * sizeof(double);
    const double *ins[3] = {in.f0, in.f1, g->ny > 1 ? in.f2 : nullptr};
    const double *outs[3] = {out.f0, out.f1, g->ny > 1 ? out.f2 : nullptr};
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (ins[a] && outs[b] && overlaps(ins[a], outs[b], bytes))
                return fail(SWE_E_INVAL, "input plane %d overlaps output plane %d", a, b);
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b)
            if (outs[a] && outs[b] && overlaps(outs[a], outs[b], bytes))
                return fail(SWE_E_INVAL, "output planes %d and %d overlap", a, b);
    return SWE_OK;
}

swe::KParams make_kparams(const swe_grid *g, const swe_params *p, const double *B, swe_fields in,
                          swe_fields out, double dt, swe_scalars *sc)
{
    swe::KParams k;
    std::memset(&k, 0, sizeof k);
    k.nx = g->nx; k.ny = g->ny; k.pitch = g->pitch;
    march_rows(g->nx, g->ny, k.ly, k.lyr);
    k.xcd_remap = xcd_remap_for(g->nx, march_chunks(g->ny, k.ly, k.lyr));
    for (int c = 0; c < 4; ++c) k.bc[c] = g->bc[c];
    k.order = p->order; k.transverse = p->transverse;
    k.dx = g->dx; k.dy = g->ny > 1 ? g->dy : 1.0; k.dt = dt;
    k.g = p->g; k.sea_level = p->sea_level; k.dry_tol = p->dry_tol;
    k.B = B;
    k.in0 = in.f0; k.in1 = in.f1; k.in2 = in.f2;
    k.out0 = out.f0; k.out1 = out.f1; k.out2 = out.f2;
    if (sc) {
        k.cfl_bits = (unsigned long long *)&sc->cfl_bits;
        k.cfl_spread = 1;
        k.cfl_stride = 1;
        k.n_clamped = &sc->n_clamped;
        k.n_nonfinite = &sc->n_nonfinite;
    }
    return k;
}

swe::CellParams make_cparams(const swe_grid *g, const swe_params *p, const double *B, swe_fields o)
{
    swe::CellParams c;
    std::memset(&c, 0, sizeof c);
    c.nx = g->nx; c.ny = g->ny; c.pitch = g->pitch;
    c.dx = g->dx; c.dy = g->ny > 1 ? g->dy : 1.0; c.x_lo = g->x_lo; c.y_lo = g->y_lo;
    c.g = p->g; c.sea_level = p->sea_level; c.dry_tol = p->dry_tol;
    c.B = B;
    c.o0 = o.f0; c.o1 = o.f1; c.o2 = g->ny > 1 ? o.f2 : nullptr;
    return c;
}

swe_status step_common(int model, const swe_grid *grid, const swe_params *prm, const double *B,
                       swe_fields in, swe_fields out, double dt, swe_scalars *scal, void *stream)
{
    swe_status st;
    if ((st = check_grid(grid)) != SWE_OK) return st;
    if ((st = check_params(prm)) != SWE_OK) return st;
    if (!B) return fail(SWE_E_INVAL, "B is NULL");
    if ((st = check_fields(grid, in, "in")) != SWE_OK) return st;
    if ((st = check_fields(grid, out, "out")) != SWE_OK) return st;
    if ((st = check_alias(grid, in, out)) != SWE_OK) return st;
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SWE_E_INVAL, "dt must be finite and > 0");
    if (model == swe::MODEL_NL && grid->ny < 2)
        return fail(SWE_E_INVAL, "the nonlinear model is two-dimensional (ny >= 2)");
    swe::KParams k = make_kparams(grid, prm, B, in, out, dt, scal);
    HIP_TRY(swe::launch_step(model, k, (hipStream_t)stream));
    return SWE_OK;
}

} // namespace

extern "C" {

const char *swe_last_error(void) { return g_err; }

swe_status swe_step(const swe_grid *grid, const swe_params *prm, const double *B, swe_fields in,
                    swe_fields out, double dt, swe_scalars *scal, void *stream)
{
    if (!prm) return fail(SWE_E_INVAL, "params is NULL");
    int model = prm->model == SWE_NONLINEAR ? swe::MODEL_NL : swe::MODEL_LIN;
    return step_common(model, grid, prm, B, in, out, dt, scal, stream);
}

swe_status adj_step(const swe_grid *grid, const swe_params *prm, const double *B, swe_fields in,
                    swe_fields out, double dt, swe_scalars *scal, void *stream)
{
    return step_common(swe::MODEL_ADJ, grid, prm, B, in, out, dt, scal, stream);
}

swe_status adj_target(const swe_grid *grid, const swe_params *prm, const double *B, double xc,
                      double yc, double R, int32_t shape, swe_fields phi, void *stream)
{
    swe_status st;
    if ((st = check_grid(grid)) != SWE_OK) return st;
    if ((st = check_params(prm)) != SWE_OK) return st;
    if (!B) return fail(SWE_E_INVAL, "B is NULL");
    if ((st = check_fields(grid, phi, "phi")) != SWE_OK) return st;
    if (!(R > 0.0) || !std::isfinite(R)) return fail(SWE_E_INVAL, "target radius must be > 0");
    if (shape != SWE_TARGET_GAUSS && shape != SWE_TARGET_DISK) return fail(SWE_E_INVAL, "unknown target shape");
    HIP_TRY(swe::launch_target(make_cparams(grid, prm, B, phi), xc, yc, R, shape, (hipStream_t)stream));
    return SWE_OK;
}

swe_status swe_init(const swe_grid *grid, const swe_params *prm, const double *B, const double *eta0,
                    swe_fields q, void *stream)
{
    swe_status st;
    if ((st = check_grid(grid)) != SWE_OK) return st;
    if ((st = check_params(prm)) != SWE_OK) return st;
    if (!B || !eta0) return fail(SWE_E_INVAL, "B or eta0 is NULL");
    if ((st = check_fields(grid, q, "q")) != SWE_OK) return st;
    HIP_TRY(swe::launch_init(make_cparams(grid, prm, B, q), eta0, prm->model == SWE_NONLINEAR,
                             (hipStream_t)stream));
    return SWE_OK;
}

swe_status swe_max_speed(const swe_grid *grid, const swe_params *prm, const double *B, swe_fields q,
                         int32_t adjoint, uint64_t *out_bits, void *stream)
{
    swe_status st;
    if ((st = check_grid(grid)) != SWE_OK) return st;
    if ((st = check_params(prm)) != SWE_OK) return st;
    if (!B || !out_bits) return fail(SWE_E_INVAL, "B or out is NULL");
    int mode = (adjoint || prm->model == SWE_LINEAR) ? 1 : 0;
    if (mode == 0 && (st = check_fields(grid, q, "q")) != SWE_OK) return st;
    swe_fields none = {nullptr, nullptr, nullptr};
    HIP_TRY(swe::launch_max_speed(make_cparams(grid, prm, B, none), q.f0, q.f1, q.f2, mode,
                                  (unsigned long long *)out_bits, (hipStream_t)stream));
    return SWE_OK;
}

static double snap(double r)
{
    double rr = std::nearbyint(r);
    return std::fabs(r - rr) <= 1e-9 ? rr : r;
}

swe_status swe_ctl_set(swe_ctl *ctl, double t, double dt, double t_out, int32_t cur, void *stream)
{
    if (!ctl) return fail(SWE_E_INVAL, "ctl is NULL");
    if (!std::isfinite(t) || !std::isfinite(t_out) || !(t_out >= t)) return fail(SWE_E_INVAL, "need finite t <= t_out");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(SWE_E_INVAL, "dt must be finite and > 0");
    if (cur != 0 && cur != 1) return fail(SWE_E_INVAL, "cur must be 0 or 1");
    HIP_TRY(swe::launch_ctl_set(ctl, t, dt, t_out, cur, (hipStream_t)stream));
    return SWE_OK;
}

swe_status swe_ctl_retarget(swe_ctl *ctl, double t_out, void *stream)
{
    if (!ctl) return fail(SWE_E_INVAL, "ctl is NULL");
    if (!std::isfinite(t_out)) return fail(SWE_E_INVAL, "t_out must be finite");
    HIP_TRY(swe::launch_ctl_retarget(ctl, t_out, (hipStream_t)stream));
    return SWE_OK;
}

static swe_status setup_interp(swe::FlagParams &f, const swe_grid *grid, const swe_grid *ag, const double *aB);

static swe_status advance_impl(const swe_grid *grid, const swe_params *prm, const double *B, swe_fields a,
                               swe_fields b, swe_ctl *ctl, int32_t n_attempts, const swe_flagging *fl,
                               void *stream)
{
    swe_status st;
    if ((st = check_grid(grid)) != SWE_OK) return st;
    if ((st = check_params(prm)) != SWE_OK) return st;
    if (!B || !ctl) return fail(SWE_E_INVAL, "B or ctl is NULL");
    if ((st = check_fields(grid, a, "a")) != SWE_OK) return st;
    if ((st = check_fields(grid, b, "b")) != SWE_OK) return st;
    if ((st = check_alias(grid, a, b)) != SWE_OK) return st;
    if (n_attempts < 0) return fail(SWE_E_INVAL, "n_attempts must be >= 0");
    if (!(prm->cfl_desired > 0.0) || !(prm->cfl_max >= prm->cfl_desired))
        return fail(SWE_E_INVAL, "need 0 < cfl_desired <= cfl_max");
    int model = prm->model == SWE_NONLINEAR ? swe::MODEL_NL : swe::MODEL_LIN;
    if (model == swe::MODEL_NL && grid->ny < 2) return fail(SWE_E_INVAL, "the nonlinear model needs ny >= 2");
    swe::FlagParams fp;
    swe::FlagCtl fc;
    if (fl) {
        if (!fl->frames || fl->K < 1 || fl->flag_every < 1 || !(fl->tf > fl->t0))
            return fail(SWE_E_INVAL, "flagging: need frames, K >= 1, flag_every >= 1, tf > t0");
        if (!fl->flags_final && !fl->flag_acc && !fl->maxip_acc)
            return fail(SWE_E_INVAL, "flagging: no output");
        std::memset(&fp, 0, sizeof fp);
        fp.nx = grid->nx; fp.ny = grid->ny; fp.pitch = grid->pitch;
        fp.twod = grid->ny > 1; fp.ncomp = fp.twod ? 3 : 2;
        fp.nonlinear = prm->model == SWE_NONLINEAR;
        fp.sea_level = prm->sea_level; fp.dry_tol = prm->dry_tol; fp.tol = fl->tol;
        fp.B = B; fp.frames = fl->frames;
        fp.flag_acc = fl->flag_acc; fp.maxip_acc = fl->maxip_acc;
        fp.bounds = fl->bounds;
        if (fl->adj_grid && (st = setup_interp(fp, grid, fl->adj_grid, fl->adj_B)) != SWE_OK) return st;
        std::memset(&fc, 0, sizeof fc);
        fc.ctl = ctl; fc.K = fl->K; fc.flag_every = fl->flag_every;
        fc.cfl_desired = prm->cfl_desired; fc.cfl_max = prm->cfl_max;
        fc.t0 = fl->t0; fc.ts = fl->ts; fc.tf = fl->tf;
        fc.a0 = a.f0; fc.a1 = a.f1; fc.a2 = a.f2; fc.b0 = b.f0; fc.b1 = b.f1; fc.b2 = b.f2;
        fc.flags_final = fl->flags_final;
    }
    swe::KParams k = make_kparams(grid, prm, B, a, b, 1.0, nullptr);
    k.ctl = ctl;
    k.cfl_desired = prm->cfl_desired;
    k.cfl_max = prm->cfl_max;
    k.n_clamped = &ctl->n_clamped;
    k.n_nonfinite = &ctl->n_nonfinite;
    hipStream_t s = (hipStream_t)stream;
    for (int n = 0; n < n_attempts; ++n) {
        k.attempt = n;
        HIP_TRY(swe::launch_step(model, k, s));
        if (fl) {
            fc.attempt = n;
            HIP_TRY(swe::launch_flag_ctl(fp, fc, s));
        }
    }
    if (n_attempts > 0) HIP_TRY(swe::launch_ctl_finish(ctl, n_attempts, prm->cfl_desired, prm->cfl_max, s));
    return SWE_OK;
}

swe_status swe_advance(const swe_grid *grid, const swe_params *prm, const double *B, swe_fields a,
                       swe_fields b, swe_ctl *ctl, int32_t n_attempts, void *stream)
{
    return advance_impl(grid, prm, B, a, b, ctl, n_attempts, nullptr, stream);
}

swe_status swe_advance_flagged(const swe_grid *grid, const swe_params *prm, const double *B, swe_fields a,
                               swe_fields b, swe_ctl *ctl, int32_t n_attempts, const swe_flagging *fl,
                               void *stream)
{
    if (!fl) return fail(SWE_E_INVAL, "flagging is NULL");
    return advance_impl(grid, prm, B, a, b, ctl, n_attempts, fl, stream);
}

swe_status adj_window(double t, double t0, double ts, double tf, int32_t K, int32_t *k_lo, int32_t *k_hi)
{
    if (!k_lo || !k_hi) return fail(SWE_E_INVAL, "null output");
    if (K < 1) return fail(SWE_E_INVAL, "K must be >= 1");
    if (!(tf > t0)) return fail(SWE_E_INVAL, "tf must exceed t0");
    if (!std::isfinite(t) || !std::isfinite(ts)) return fail(SWE_E_INVAL, "t and ts must be finite");
    double ds = (tf - t0) / K;
    double T = std::fmin(t + (tf - ts), tf);
    double sa = tf - T, sb = tf - t;
    if (sb < 0.0) {
        *k_lo = 1;
        *k_hi = 0;
        return SWE_OK;
    }
    double lo = std::floor(snap(sa / ds)), hi = std::ceil(snap(sb / ds));
    if (lo < 0.0) lo = 0.0;
    if (hi > K) hi = K;
    *k_lo = (int32_t)lo;
    *k_hi = (int32_t)hi;
    return SWE_OK;
}

// Snapshots on a grid of their own: validate it and record its geometry.
static swe_status setup_interp(swe::FlagParams &f, const swe_grid *grid, const swe_grid *ag, const double *aB)
{
    swe_status st;
    if ((st = check_grid(ag)) != SWE_OK) return st;
    if ((ag->ny > 1) != (grid->ny > 1)) return fail(SWE_E_INVAL, "adjoint grid of another dimension");
    if (!aB) return fail(SWE_E_INVAL, "adjoint grid without its bottom");
    f.interp = 1;
    f.x_lo = grid->x_lo; f.y_lo = grid->y_lo; f.dx = grid->dx; f.dy = grid->dy;
    f.anx = ag->nx; f.any = ag->ny; f.apitch = ag->pitch;
    f.ax_lo = ag->x_lo; f.ay_lo = ag->y_lo; f.adx = ag->dx; f.ady = ag->dy;
    f.aB = aB;
    return SWE_OK;
}

static swe_status flag_common(const swe_grid *grid, const swe_params *prm, const double *B, swe_fields q,
                              const swe_grid *ag, const double *aB, const double *frames, int32_t K, int32_t k_lo,
                              int32_t k_hi, double tol, int8_t *flags, double *maxip, int8_t *flag_acc,
                              double *maxip_acc, const int32_t *bounds, void *stream)
{
    swe_status st;
    if ((st = check_grid(grid)) != SWE_OK) return st;
    if ((st = check_params(prm)) != SWE_OK) return st;
    if (!B || !frames) return fail(SWE_E_INVAL, "B or frames is NULL");
    if ((st = check_fields(grid, q, "q")) != SWE_OK) return st;
    if (K < 0) return fail(SWE_E_INVAL, "K must be >= 0");
    if (k_lo <= k_hi && (k_lo < 0 || k_hi > K)) return fail(SWE_E_INVAL, "window [%d, %d] outside [0, %d]", k_lo, k_hi, K);
    if (!flags && !maxip && !flag_acc && !maxip_acc) return fail(SWE_E_INVAL, "no output requested");
    if (!std::isfinite(tol)) return fail(SWE_E_INVAL, "tol must be finite");
    if (prm->model == SWE_NONLINEAR && grid->ny < 2) return fail(SWE_E_INVAL, "nonlinear model needs ny >= 2");
    swe::FlagParams f;
    std::memset(&f, 0, sizeof f);
    f.nx = grid->nx; f.ny = grid->ny; f.pitch = grid->pitch;
    f.twod = grid->ny > 1; f.ncomp = f.twod ? 3 : 2;
    f.nonlinear = prm->model == SWE_NONLINEAR;
    f.k_lo = k_lo; f.k_hi = k_hi;
    f.sea_level = prm->sea_level; f.dry_tol = prm->dry_tol; f.tol = tol;
    f.B = B; f.q0 = q.f0; f.q1 = q.f1; f.q2 = q.f2; f.frames = frames;
    f.flags = flags; f.maxip = maxip; f.flag_acc = flag_acc; f.maxip_acc = maxip_acc;
    f.bounds = bounds;
    if (ag && (st = setup_interp(f, grid, ag, aB)) != SWE_OK) return st;
    HIP_TRY(swe::launch_flag(f, (hipStream_t)stream));
    return SWE_OK;
}

swe_status adj_flag(const swe_grid *grid, const swe_params *prm, const double *B, swe_fields q,
                    const double *frames, int32_t K, int32_t k_lo, int32_t k_hi, double tol,
                    int8_t *flags, double *maxip, int8_t *flag_acc, double *maxip_acc, const int32_t *bounds,
                    void *stream)
{
    return flag_common(grid, prm, B, q, nullptr, nullptr, frames, K, k_lo, k_hi, tol, flags, maxip, flag_acc,
                       maxip_acc, bounds, stream);
}

swe_status adj_frame_bounds(const swe_grid *grid, const double *frames, int32_t K, int32_t *bounds, void *stream)
{
    swe_status st;
    if ((st = check_grid(grid)) != SWE_OK) return st;
    if (!frames || !bounds) return fail(SWE_E_INVAL, "frames or bounds is NULL");
    if (K < 0) return fail(SWE_E_INVAL, "K must be >= 0");
    HIP_TRY(swe::launch_frame_bounds(frames, grid->nx, grid->ny, grid->pitch, grid->ny > 1 ? 3 : 2, K, bounds,
                                     (hipStream_t)stream));
    return SWE_OK;
}

swe_status adj_flag_interp(const swe_grid *grid, const swe_params *prm, const double *B, swe_fields q,
                           const swe_grid *adj_grid, const double *adj_B, const double *frames, int32_t K,
                           int32_t k_lo, int32_t k_hi, double tol, int8_t *flags, double *maxip, int8_t *flag_acc,
                           double *maxip_acc, const int32_t *bounds, void *stream)
{
    if (!adj_grid) return fail(SWE_E_INVAL, "adj_grid is NULL");
    return flag_common(grid, prm, B, q, adj_grid, adj_B, frames, K, k_lo, k_hi, tol, flags, maxip, flag_acc,
                       maxip_acc, bounds, stream);
}

swe_status swe_surface_flag(const swe_grid *grid, const swe_params *prm, const double *B, swe_fields q, double tol,
                            int8_t *flags, int8_t *flag_acc, void *stream)
{
    swe_status st;
    if ((st = check_grid(grid)) != SWE_OK) return st;
    if ((st = check_params(prm)) != SWE_OK) return st;
    if (!B || !q.f0) return fail(SWE_E_INVAL, "B or q.f0 is NULL");
    if (!flags && !flag_acc) return fail(SWE_E_INVAL, "no output requested");
    if (!std::isfinite(tol)) return fail(SWE_E_INVAL, "tol must be finite");
    swe_fields none = {nullptr, nullptr, nullptr};
    HIP_TRY(swe::launch_surface_flag(make_cparams(grid, prm, B, none), q.f0, tol, prm->model == SWE_NONLINEAR,
                                     flags, flag_acc, (hipStream_t)stream));
    return SWE_OK;
}

// ---------------------------------------------------------------------------
// two-phase driver
// ---------------------------------------------------------------------------
struct Workspace {
    double *a[3], *b[3];      // adjoint ping-pong is done in the frame buffer; these are the forward second set
    int8_t *flags;
    swe_scalars *sc;
    unsigned long long *speed;
    swe_ctl *ctl;
    int32_t *bounds;          // non-zero boxes of the snapshots
    // 1D runs in one workgroup: the recorded states of a forward launch, their
    // times and end-of-segment marks, their count, and m per record and cell
    double *hist, *hist_t, *hist_m;
    int *hist_done, *n_rec;
    size_t bytes;
};

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static swe_status check_problem(const swe_problem *pb)
{
    if (!pb) return fail(SWE_E_INVAL, "problem is NULL");
    swe_status st;
    if ((st = check_grid(&pb->grid)) != SWE_OK) return st;
    if ((st = check_params(&pb->params)) != SWE_OK) return st;
    if (!pb->B || !pb->eta0 || !pb->frames) return fail(SWE_E_INVAL, "B, eta0 or frames is NULL");
    if ((st = check_fields(&pb->grid, pb->q_out, "q_out")) != SWE_OK) return st;
    if (pb->K < 1) return fail(SWE_E_INVAL, "K must be >= 1");
    if (!(pb->tf > pb->t0) || !std::isfinite(pb->tf) || !std::isfinite(pb->t0))
        return fail(SWE_E_INVAL, "need finite t0 < tf");
    if (!(pb->ts >= pb->t0 && pb->ts <= pb->tf)) return fail(SWE_E_INVAL, "need t0 <= ts <= tf");
    if (pb->flag_every < 1) return fail(SWE_E_INVAL, "flag_every must be >= 1");
    if (pb->full_frames != 0 && pb->full_frames != 1) return fail(SWE_E_INVAL, "full_frames must be 0 or 1");
    if (pb->launch_per_step != 0 && pb->launch_per_step != 1)
        return fail(SWE_E_INVAL, "launch_per_step must be 0 or 1");
    if (!(pb->target_R > 0.0)) return fail(SWE_E_INVAL, "target radius must be > 0");
    if (pb->adj_grid.nx != 0) {
        if ((st = check_grid(&pb->adj_grid)) != SWE_OK) return st;
        if ((pb->adj_grid.ny > 1) != (pb->grid.ny > 1)) return fail(SWE_E_INVAL, "adjoint grid of another dimension");
        if (!pb->adj_B) return fail(SWE_E_INVAL, "adjoint grid without its bottom adj_B");
    }
    bool twod = pb->grid.ny > 1;
    if (!twod && pb->params.model != SWE_LINEAR) return fail(SWE_E_INVAL, "1D runs use the linear model");
    return SWE_OK;
}

static size_t ws_layout(const swe_problem *pb, Workspace *w, char *base)
{
    // the two state sets serve the adjoint sub-steps (on the adjoint grid) and the forward run
    size_t plane = (size_t)pb->grid.ny * pb->grid.pitch * sizeof(double);
    if (pb->adj_grid.nx != 0)
        plane = std::max(plane, (size_t)pb->adj_grid.ny * pb->adj_grid.pitch * sizeof(double));
    size_t off = 0;
    for (int c = 0; c < 3; ++c) {
        if (w) w->a[c] = (double *)(base + off);
        off = align256(off + plane);
    }
    for (int c = 0; c < 3; ++c) {
        if (w) w->b[c] = (double *)(base + off);
        off = align256(off + plane);
    }
    if (w) w->flags = (int8_t *)(base + off);
    off = align256(off + (size_t)pb->grid.ny * pb->grid.pitch);
    if (w) w->sc = (swe_scalars *)(base + off);
    off = align256(off + sizeof(swe_scalars));
    if (w) w->speed = (unsigned long long *)(base + off);
    off = align256(off + sizeof(unsigned long long));
    if (w) w->ctl = (swe_ctl *)(base + off);
    off = align256(off + sizeof(swe_ctl));
    if (w) w->bounds = (int32_t *)(base + off);
    off = align256(off + (size_t)4 * (pb->K + 1) * sizeof(int32_t));
    if (w) { w->hist = w->hist_t = w->hist_m = nullptr; w->hist_done = w->n_rec = nullptr; }
    if (pb->grid.ny == 1 && pb->grid.nx <= swe::RUN1D_MAX_NX && !pb->launch_per_step) {
        const size_t nx = (size_t)pb->grid.nx, R = swe::RUN1D_RECORDS;
        if (w) w->hist = (double *)(base + off);
        off = align256(off + R * 2 * nx * sizeof(double));
        if (w) w->hist_m = (double *)(base + off);
        off = align256(off + R * nx * sizeof(double));
        if (w) w->hist_t = (double *)(base + off);
        off = align256(off + R * sizeof(double));
        if (w) w->hist_done = (int *)(base + off);
        off = align256(off + R * sizeof(int));
        if (w) w->n_rec = (int *)(base + off);
        off = align256(off + sizeof(int));
    }
    if (w) w->bytes = off;
    return off;
}

size_t swe_run_workspace_bytes(const swe_problem *pb)
{
    if (check_problem(pb) != SWE_OK) return 0;
    return ws_layout(pb, nullptr, nullptr);
}

static double bits_to_double(unsigned long long b)
{
    double d;
    std::memcpy(&d, &b, sizeof d);
    return d;
}

swe_status swe_run(const swe_problem *pb, void *workspace, size_t workspace_bytes, swe_result *res,
                   void *stream)
{
    swe_status st;
    if ((st = check_problem(pb)) != SWE_OK) return st;
    if (!res) return fail(SWE_E_INVAL, "result is NULL");
    if (!workspace) return fail(SWE_E_INVAL, "workspace is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(SWE_E_INVAL, "workspace must be 256-byte aligned");
    size_t need = ws_layout(pb, nullptr, nullptr);
    if (workspace_bytes < need) return fail(SWE_E_NOMEM, "workspace %zu bytes < %zu needed", workspace_bytes, need);
    Workspace w;
    ws_layout(pb, &w, (char *)workspace);
    hipStream_t s = (hipStream_t)stream;
    std::memset(res, 0, sizeof *res);

    const swe_grid *G = &pb->grid;
    const swe_params *P = &pb->params;
    const bool twod = G->ny > 1;
    const int ncomp = twod ? 3 : 2;
    const size_t plane = (size_t)G->ny * G->pitch;
    const int K = pb->K;
    // the adjoint's grid and bottom (the forward's unless a grid of its own is given)
    const bool interp = pb->adj_grid.nx != 0;
    const swe_grid *AG = interp ? &pb->adj_grid : G;
    const double *AB = interp ? pb->adj_B : pb->B;
    const size_t aplane = (size_t)AG->ny * AG->pitch;
    auto frame = [&](int k) {
        swe_fields f;
        f.f0 = pb->frames + ((size_t)k * ncomp + 0) * aplane;
        f.f1 = pb->frames + ((size_t)k * ncomp + 1) * aplane;
        f.f2 = twod ? pb->frames + ((size_t)k * ncomp + 2) * aplane : nullptr;
        return f;
    };
    swe_fields A = {w.a[0], w.a[1], twod ? w.a[2] : nullptr};
    swe_fields Bf = {w.b[0], w.b[1], twod ? w.b[2] : nullptr};

    // ---- phase A: adjoint snapshots
    HIP_TRY(hipMemsetAsync(w.speed, 0, sizeof(unsigned long long), s));
    if ((st = swe_max_speed(AG, P, AB, A, 1, (uint64_t *)w.speed, stream)) != SWE_OK) return st;
    unsigned long long spb = 0;
    HIP_TRY(hipMemcpyAsync(&spb, w.speed, sizeof spb, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    // speed = max over wet cells of max(c/dx, c/dy) = max(cmax/dx, cmax/dy)
    double smax = bits_to_double(spb);
    double ds = (pb->tf - pb->t0) / K;
    if (!(smax > 0.0)) return fail(SWE_E_INVAL, "no wet cell for the adjoint");
    double dt_cfl = P->cfl_desired / smax;
    int nsub = (int)std::ceil(ds / dt_cfl);
    if (nsub < 1) nsub = 1;
    double dt_adj = ds / nsub;
    res->n_sub = nsub;
    res->dt_adj = dt_adj;
    if ((st = adj_target(AG, P, AB, pb->target_xc, pb->target_yc, pb->target_R, pb->target_shape,
                         frame(0), stream)) != SWE_OK)
        return st;
    // a 1D adjoint grid that fits one workgroup: the whole phase in one launch
    if (!twod && !pb->launch_per_step && swe::run1d_lds_bytes(AG->nx)) {
        swe::Run1dArgs ra;
        std::memset(&ra, 0, sizeof ra);
        ra.P = make_kparams(AG, P, AB, frame(0), frame(0), dt_adj, nullptr);
        ra.frames = pb->frames;
        ra.fplane = aplane;
        ra.K = K;
        ra.nsub = nsub;
        HIP_TRY(swe::launch_adj_run1d(ra, s));
        res->n_adj_steps = K * nsub;
    } else {
        for (int k = 1; k <= K; ++k) {
            swe_fields src = frame(k - 1);
            for (int sstep = 0; sstep < nsub; ++sstep) {
                bool last = sstep == nsub - 1;
                swe_fields dst = last ? frame(k) : ((sstep & 1) ? Bf : A);
                if ((st = adj_step(AG, P, AB, src, dst, dt_adj, nullptr, stream)) != SWE_OK) return st;
                res->n_adj_steps++;
                src = dst;
            }
        }
    }

    // the snapshots' non-zero boxes: outside them the flag passes have nothing to read
    const int32_t *bounds = nullptr;
    if (!pb->full_frames) {
        if ((st = adj_frame_bounds(AG, pb->frames, K, w.bounds, stream)) != SWE_OK) return st;
        bounds = w.bounds;
    }

    // ---- phase B: forward with flagging, stepped and flagged on the device;
    // the host only waits once per output segment
    swe_fields cur = A, nxt = Bf;
    if ((st = swe_init(G, P, pb->B, pb->eta0, cur, stream)) != SWE_OK) return st;
    {
        int32_t lo, hi;
        if ((st = adj_window(pb->t0, pb->t0, pb->ts, pb->tf, K, &lo, &hi)) != SWE_OK) return st;
        int8_t *fl0 = pb->flags_at ? pb->flags_at : w.flags;
        if ((st = flag_common(G, P, pb->B, cur, interp ? AG : nullptr, AB, pb->frames, K, lo, hi, pb->tol, fl0,
                              nullptr, pb->flag_acc, pb->maxip_acc, bounds, stream)) != SWE_OK)
            return st;
        if (pb->surface_flags_at &&
            (st = swe_surface_flag(G, P, pb->B, cur, pb->surface_tol, pb->surface_flags_at, nullptr, stream)) !=
                SWE_OK)
            return st;
    }
    HIP_TRY(hipMemsetAsync(w.speed, 0, sizeof(unsigned long long), s));
    if ((st = swe_max_speed(G, P, pb->B, cur, 0, (uint64_t *)w.speed, stream)) != SWE_OK) return st;
    HIP_TRY(hipMemcpyAsync(&spb, w.speed, sizeof spb, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    smax = bits_to_double(spb);
    if (!(smax > 0.0)) return fail(SWE_E_INVAL, "no wet cell for the forward problem");
    double dt0 = P->cfl_desired / smax;
    swe_flagging fl;
    fl.frames = pb->frames;
    fl.K = K;
    fl.flag_every = pb->flag_every;
    fl.t0 = pb->t0; fl.ts = pb->ts; fl.tf = pb->tf; fl.tol = pb->tol;
    fl.flag_acc = pb->flag_acc;
    fl.maxip_acc = pb->maxip_acc;
    fl.adj_grid = interp ? AG : nullptr;
    fl.adj_B = interp ? AB : nullptr;
    fl.bounds = bounds;
    // a 1D forward grid that fits one workgroup: each round of attempts in one
    // launch, its flagged states flagged afterwards in two
    const bool run1d = !twod && w.hist && swe::run1d_lds_bytes(G->nx);
    swe::Run1dArgs ra;
    swe::FlagParams hf;
    swe::HistArgs ha;
    if (run1d) {
        std::memset(&ra, 0, sizeof ra);
        ra.P = make_kparams(G, P, pb->B, A, Bf, 1.0, nullptr);
        ra.P.ctl = w.ctl;
        ra.P.cfl_desired = P->cfl_desired;
        ra.P.cfl_max = P->cfl_max;
        ra.flag_every = pb->flag_every;
        ra.hist = w.hist;
        ra.hist_t = w.hist_t;
        ra.hist_done = w.hist_done;
        ra.n_rec = w.n_rec;
        std::memset(&hf, 0, sizeof hf);
        hf.nx = G->nx; hf.ny = 1; hf.pitch = G->pitch; hf.ncomp = 2;
        hf.twod = 0; hf.nonlinear = 0;
        hf.sea_level = P->sea_level; hf.dry_tol = P->dry_tol; hf.tol = pb->tol;
        hf.B = pb->B; hf.frames = pb->frames;
        hf.flag_acc = pb->flag_acc; hf.maxip_acc = pb->maxip_acc;
        hf.bounds = bounds;
        if (interp && (st = setup_interp(hf, G, AG, AB)) != SWE_OK) return st;
        std::memset(&ha, 0, sizeof ha);
        ha.hist = w.hist; ha.hist_t = w.hist_t; ha.hist_done = w.hist_done; ha.n_rec = w.n_rec;
        ha.m = w.hist_m;
        ha.t0 = pb->t0; ha.ts = pb->ts; ha.tf = pb->tf; ha.K = K;
    }
    swe_ctl hc;
    for (int j = 1; j <= K; ++j) {
        double tout = (j == K) ? pb->tf : pb->t0 + j * ds;
        if (j == 1) {
            if ((st = swe_ctl_set(w.ctl, pb->t0, dt0, tout, 0, stream)) != SWE_OK) return st;
            HIP_TRY(hipMemcpyAsync(&hc, w.ctl, sizeof hc, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
        } else {
            // the host's copy of the control block is the state at the last
            // output time, which the retarget leaves as it is but for the new
            // output time (and dt clamped to it): the attempt count below
            // comes out the same from either dt, so no read is needed
            if ((st = swe_ctl_retarget(w.ctl, tout, stream)) != SWE_OK) return st;
            hc.s.done = 0;
        }
        fl.flags_final = pb->flags_at ? pb->flags_at + (size_t)j * plane : w.flags;
        int rounds = 0, stalled = 0;
        while (!hc.s.done) {
            const double t_before = hc.s.t;
            if (!(hc.s.dt >= 1e-6 * dt0))
                return fail(SWE_E_CFL, "time step collapsed at t = %g (dt = %g, initial %g)", hc.s.t, hc.s.dt,
                            dt0);
            double need = std::ceil((tout - hc.s.t) / hc.s.dt);
            int n = (int)std::min(std::max(need, 0.0) + 2.0, 100000.0);
            if (run1d) {
                ra.max_attempts = std::min(n, swe::RUN1D_RECORDS);
                ha.flags_final = fl.flags_final;
                HIP_TRY(swe::launch_fwd_run1d(ra, s));
                HIP_TRY(swe::launch_hist_flag(hf, ha, s));
            } else if ((st = swe_advance_flagged(G, P, pb->B, A, Bf, w.ctl, n, &fl, stream)) != SWE_OK) {
                return st;
            }
            HIP_TRY(hipMemcpyAsync(&hc, w.ctl, sizeof hc, hipMemcpyDeviceToHost, s));
            HIP_TRY(hipStreamSynchronize(s));
            if (hc.n_nonfinite) return fail(SWE_E_NONFINITE, "non-finite state near t = %g", hc.s.t);
            // A time step a million times below the initial one means the
            // wave speeds grew a million-fold: the state has blown up (a round
            // of such steps would not reach the output time in any useful
            // time, and once dt is below the resolution of t no step advances
            // it at all).
            stalled = hc.s.t > t_before ? 0 : stalled + 1;
            if (!hc.s.done && (!(hc.s.dt >= 1e-6 * dt0) || stalled >= 3))
                return fail(SWE_E_CFL, "time step collapsed at t = %g (dt = %g, initial %g)", hc.s.t, hc.s.dt,
                            dt0);
            if (++rounds > (run1d ? 400000 : 1000) || hc.s.n_rejected > 1000)
                return fail(SWE_E_CFL, "no progress at t = %g", hc.s.t);
        }
        if (pb->surface_flags_at) {
            swe_fields now = hc.s.cur ? Bf : A;
            if ((st = swe_surface_flag(G, P, pb->B, now, pb->surface_tol, pb->surface_flags_at + (size_t)j * plane,
                                       nullptr, stream)) != SWE_OK)
                return st;
        }
    }
    cur = hc.s.cur ? Bf : A;
    (void)nxt;
    res->n_fwd_steps = hc.s.n_accepted;
    res->n_rejected = hc.s.n_rejected;
    res->n_clamped = hc.n_clamped;
    res->n_flag_calls = 1 + hc.n_flag_calls;
    double t = hc.s.t;
    // final state into q_out
    size_t row_bytes = (size_t)G->nx * sizeof(double), pitch_bytes = (size_t)G->pitch * sizeof(double);
    double *dst[3] = {pb->q_out.f0, pb->q_out.f1, pb->q_out.f2};
    double *srcp[3] = {cur.f0, cur.f1, cur.f2};
    for (int c = 0; c < ncomp; ++c)
        HIP_TRY(hipMemcpy2DAsync(dst[c], pitch_bytes, srcp[c], pitch_bytes, row_bytes, G->ny,
                                 hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    res->t_end = t;
    return SWE_OK;
}

// ---------------------------------------------------------------------------
// allocation-free driver: the workspace is a fixed array in the library's
// device memory (every GPU the library runs on holds its own copy)
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[SWE_STATIC_WORKSPACE_BYTES];

// Device address of this GPU's copy of `scratch`, looked up once per device
// with that device current.  In host code `scratch` only names the symbol;
// its device address must come from the runtime.
static swe_status scratch_address(void **out)
{
    static std::mutex mu;
    static void *addr[64] = {};
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(SWE_E_HIP, "device %d out of range", dev);
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SWE_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        addr[dev] = p;
    }
    *out = addr[dev];
    return SWE_OK;
}

swe_status swe_run_static(const swe_problem *pb, swe_result *res, void *stream)
{
    swe_status st;
    if ((st = check_problem(pb)) != SWE_OK) return st;
    if (!res) return fail(SWE_E_INVAL, "result is NULL");
    const size_t need = ws_layout(pb, nullptr, nullptr);
    if (need > SWE_STATIC_WORKSPACE_BYTES)
        return fail(SWE_E_NOMEM, "problem needs %zu bytes of workspace, the static workspace holds %zu "
                    "(use swe_run with a workspace of the caller's)", need, (size_t)SWE_STATIC_WORKSPACE_BYTES);
    void *ws = nullptr;
    if ((st = scratch_address(&ws)) != SWE_OK) return st;
    return swe_run(pb, ws, SWE_STATIC_WORKSPACE_BYTES, res, stream);
}

} // extern "C"
