// Internal interface between the C ABI layer and the kernels (not installed).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "swe.h"
#include "swe_device.h"

namespace swe {

enum { MODEL_NL = 0, MODEL_LIN = 1, MODEL_ADJ = 2 };

struct FlagParams {
    int nx, ny, pitch, ncomp;
    int twod, nonlinear;
    int k_lo, k_hi;
    double sea_level, dry_tol, tol;
    const double *B, *q0, *q1, *q2, *frames;
    int8_t *flags;
    double *maxip;
    int8_t *flag_acc;
    double *maxip_acc;
    // snapshots on a grid of their own (interp != 0): the forward grid's
    // geometry, the adjoint grid and its bottom; frames then have its pitch
    int interp;
    double x_lo, y_lo, dx, dy;
    int anx, any, apitch;
    double ax_lo, ay_lo, adx, ady;
    const double *aB;
    // per snapshot the box (i_lo, i_hi, j_lo, j_hi) holding its non-zero
    // cells (on the snapshots' grid), or null: snapshots outside a cell's box
    // contribute |0| = 0 and are skipped
    const int *bounds;
};

// Device-side flag scheduling after a controlled step attempt.
struct FlagCtl {
    swe_ctl *ctl;
    int attempt, K, flag_every;
    double cfl_desired, cfl_max, t0, ts, tf;
    const double *a0, *a1, *a2, *b0, *b1, *b2;
    int8_t *flags_final;
};

// A one-dimensional phase marched in one workgroup (state in LDS).
constexpr int RUN1D_THREADS = 1024;           // 16 wavefronts
constexpr int RUN1D_WAVES = RUN1D_THREADS / 64;
constexpr int RUN1D_MAXS = 4;                 // strips of 60 cells per wavefront
constexpr int RUN1D_MAX_NX = RUN1D_WAVES * RUN1D_MAXS * 60;
constexpr int RUN1D_RECORDS = 256;            // flagged states kept per launch

struct Run1dArgs {
    KParams P;                 // grid, model, bottom; in* = plane set a, out* = plane set b
    // adjoint (fixed dt = P.dt): snapshot k = state after k*nsub steps from snapshot 0
    double *frames;            //   snapshot k, component c at frames + (2k + c)*fplane
    size_t fplane;
    int K, nsub;
    // forward under device-side control (P.ctl): up to max_attempts attempts;
    // the states that are to be flagged are recorded (two planes of nx each),
    // with their time and whether they end the segment
    int max_attempts, flag_every;
    double *hist, *hist_t;
    int *hist_done, *n_rec;
};

// Flagging of the recorded states of a 1D forward launch: m per record and
// cell (in order of the records), then the records folded into the outputs
// one after the other, as the per-attempt flag passes would.
struct HistArgs {
    const double *hist, *hist_t;
    const int *hist_done, *n_rec;
    double *m;
    double t0, ts, tf;
    int K;
    int8_t *flags_final;
};

struct CellParams {
    int nx, ny, pitch;
    double dx, dy, x_lo, y_lo;
    double g, sea_level, dry_tol;
    const double *B;
    double *o0, *o1, *o2;
};

// record a message for swe_last_error() and return st
swe_status fail(swe_status st, const char *fmt, ...);

// g and dry_tol lie in [1e-100, 1e100]: the step kernels' square roots and
// divisions of depths and wave speeds rely on operands far from the ends of
// the double range.
inline bool params_in_range(const swe_params *p)
{
    return p->g >= 1e-100 && p->g <= 1e100 && p->dry_tol >= 1e-100 && p->dry_tol <= 1e100;
}

hipError_t launch_step(int model, const KParams &P, hipStream_t s);
hipError_t launch_flag(const FlagParams &F, hipStream_t s);
hipError_t launch_frame_bounds(const double *frames, int nx, int ny, int pitch, int ncomp, int K, int *bounds,
                               hipStream_t s);
hipError_t launch_surface_flag(const CellParams &C, const double *q0, double tol, int nonlinear, int8_t *flags,
                               int8_t *flag_acc, hipStream_t s);
hipError_t launch_flag_ctl(const FlagParams &F, const FlagCtl &C, hipStream_t s);
hipError_t launch_level_step(const KParams &P, const LevelArgs &L, hipStream_t s);
hipError_t launch_level_persistent(const KParams &P, const LevelArgs &L, int n_steps, int nw, hipStream_t s);
int level_persistent_capacity();
// LDS bytes of a 1D run over nx cells, or 0 where it does not fit one workgroup
size_t run1d_lds_bytes(int nx);
hipError_t launch_adj_run1d(const Run1dArgs &A, hipStream_t s);
hipError_t launch_fwd_run1d(const Run1dArgs &A, hipStream_t s);
hipError_t launch_hist_flag(const FlagParams &F, const HistArgs &H, hipStream_t s);
hipError_t launch_count_diff(const double *a, const double *b, long long n, int *out, hipStream_t s);
hipError_t launch_ctl_set(swe_ctl *c, double t, double dt, double t_out, int cur, hipStream_t s);
hipError_t launch_ctl_retarget(swe_ctl *c, double t_out, hipStream_t s);
hipError_t launch_ctl_finish(swe_ctl *c, int n, double cfl_desired, double cfl_max, hipStream_t s);
hipError_t launch_target(const CellParams &C, double xc, double yc, double R, int shape, hipStream_t s);
hipError_t launch_init(const CellParams &C, const double *eta0, int nonlinear, hipStream_t s);
hipError_t launch_max_speed(const CellParams &C, const double *q0, const double *q1, const double *q2,
                            int mode, unsigned long long *out, hipStream_t s);

} // namespace swe
