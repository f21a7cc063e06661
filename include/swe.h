/*
 * swe.h - C ABI of the MI355X (gfx950) library for adjoint-guided refinement
 * flagging in shallow-water tsunami modelling.
 *
 * Method: Davis & LeVeque, "Adjoint methods for guiding adaptive mesh
 * refinement in tsunami modeling".  The library implements the data-parallel
 * hot path of that method:
 *   - the 2D shallow-water finite-volume step of eq. (swe) (Sec. 5), in
 *     wave-propagation form: f-wave Roe solver with the bathymetry source
 *     folded into the flux difference, MC-limited second-order corrections,
 *     transverse splitting of fluctuations, a dry-cell threshold and the CFL
 *     number of the step;
 *   - the 1D linearized equations of eqs. (swe_1d_linearized)/(hyp_linear);
 *   - the time-reversed adjoint q~_t - (A^T q~)_x = 0 (Sec. 4) in 1D and its
 *     2D form for A1, A2 of eq. (2d_hyperbolicsystem) (Sec. 5), with zero
 *     normal velocity at walls and wet/dry interfaces;
 *   - the snapshot window of eq. (ip_timerange) and the per-cell flag
 *     max_k |q^T q^_k| > tol of Secs. 4.1-4.2 with the wet/dry rule of Sec. 6;
 *   - the two-phase driver of Sec. 4 (adjoint snapshots, then the forward run
 *     with flagging).
 *
 * Conventions (all entry points):
 *   - Arithmetic is IEEE binary64 without fused multiply-add contraction.
 *   - Device buffers are plain device pointers allocated by the caller (the
 *     library never allocates or frees device memory).  A 2D field is one
 *     plane of ny rows of `pitch` doubles (pitch >= nx), x fastest, no ghost
 *     cells; cell (i, j) is at offset j*pitch + i and has centre
 *     (x_lo + (i+1/2) dx, y_lo + (j+1/2) dy).  Boundary ghost cells are
 *     synthesised by the kernels from the boundary conditions.
 *   - ny == 1 selects the one-dimensional scheme (linear model and adjoint);
 *     the linear model and the adjoint also run in 2D.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = default stream) and
 *     the call returns without waiting, except where stated.  Buffers must
 *     stay valid until the work has completed.
 *   - Return value: SWE_OK or a negative swe_status.  Argument errors are
 *     detected before anything is enqueued and leave all buffers untouched;
 *     swe_last_error() then returns a message (per calling thread).
 *   - Calls are reentrant and thread-safe for distinct buffers and streams.
 */
#ifndef SWE_H
#define SWE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SWE_API __attribute__((visibility("default")))

typedef enum {
    SWE_OK = 0,
    SWE_E_INVAL = -1,      /* bad argument (null pointer, size, dt, alias, ...) */
    SWE_E_CFL = -2,        /* the driver could not find an accepted step, or its time step
                              collapsed (a million times below the initial one: a blown-up state) */
    SWE_E_HIP = -3,        /* a HIP runtime call failed */
    SWE_E_NOMEM = -4,      /* the caller's workspace is too small */
    SWE_E_NONFINITE = -5,  /* a non-finite value appeared in the state */
    SWE_E_NEGDEPTH = -6    /* a negative depth had to be clamped */
} swe_status;

/* Largest nx of a grid (a row of one plane then spans < 2 GiB). */
#define SWE_MAX_NX (1 << 27)

typedef enum { SWE_BC_WALL = 0, SWE_BC_EXTRAP = 1 } swe_bc;
typedef enum { SWE_NONLINEAR = 0, SWE_LINEAR = 1 } swe_model;
typedef enum { SWE_TARGET_GAUSS = 0, SWE_TARGET_DISK = 1 } swe_target_shape;

/* Uniform grid.  ny == 1: one space dimension.  nx >= 2 and (ny == 1 or ny >= 2). */
typedef struct {
    int32_t nx, ny;
    int32_t pitch;          /* doubles between consecutive rows, >= nx */
    int32_t bc[4];          /* swe_bc for the x_lo, x_hi, y_lo, y_hi sides */
    double dx, dy;          /* cell sizes (m) */
    double x_lo, y_lo;      /* lower-left corner (m) */
} swe_grid;

typedef struct {
    int32_t model;          /* swe_model of the forward problem */
    int32_t order;          /* 1 (Godunov) or 2 (MC-limited corrections) */
    int32_t transverse;     /* 1: transverse splitting of fluctuations (2D) */
    int32_t reserved;
    double g;               /* gravity (m/s^2), in [1e-100, 1e100] */
    double sea_level;       /* eta_bar: the surface the equations are linearized about */
    double dry_tol;         /* a cell is wet iff its depth > dry_tol (m), in [1e-100, 1e100] */
    double cfl_desired;     /* target Courant number of the variable time step */
    double cfl_max;         /* steps with a larger Courant number are rejected */
} swe_params;

/* Three device planes.  Nonlinear: (h, hu, hv).  Linear and adjoint:
 * (eta, mu, gamma) - in 1D only f0, f1 are used. */
typedef struct { double *f0, *f1, *f2; } swe_fields;

/* Device-resident per-step outputs.  The step kernels max-reduce the Courant
 * number into cfl_bits (the bit pattern of a non-negative double, so integer
 * max is float max) and count clamped negative depths and non-finite results;
 * the caller zeroes the struct before the steps it wants to observe. */
typedef struct {
    uint64_t cfl_bits;
    int32_t n_clamped;
    int32_t n_nonfinite;
} swe_scalars;

/*
 * swe_step - one forward finite-volume step of length dt.
 * Nonlinear model (2D): eq. (swe) of Sec. 5 by the f-wave Roe solver; wet iff
 * h > dry_tol; a wet/dry interface is a wall (the dry side mirrors the wet
 * side); dry cells are not updated; after the update momenta are zeroed where
 * h <= dry_tol and negative depths are clamped to zero (counted).
 * Linear model: in 1D (ny == 1) eq. (hyp_linear) with A(x) of eq. (SWE_Aq) in
 * wave form; in 2D the equations of Sec. 5 linearized about the sea at rest,
 * q = (eta, mu, gamma), wave form with transverse terms (the discrete
 * transpose of adj_step at first order without transverse terms, and with
 * them over constant depth).  Wet iff hbar = max(0, sea_level - B) > dry_tol.
 * `in` and `out` must not alias.  B is the bottom elevation plane.
 * `scal` (device, may be NULL) receives the Courant number of the step.
 */
SWE_API swe_status swe_step(const swe_grid *grid, const swe_params *prm, const double *B,
                    swe_fields in, swe_fields out, double dt, swe_scalars *scal,
                    void *stream);

/*
 * adj_step - one step of length dt of the time-reversed adjoint (Sec. 4):
 * q~(x, s) = q^(x, tf - s) solves q~_s - (A^T q~)_x = 0 in 1D and
 * q~_s - (A1^T q~)_x - (A2^T q~)_y = 0 in 2D (Sec. 5), linearized about
 * the sea at rest at sea_level (hbar = max(0, sea_level - B)); walls at wet/dry
 * interfaces (zero normal velocity, Sec. 5); dry cells are not updated.
 */
SWE_API swe_status adj_step(const swe_grid *grid, const swe_params *prm, const double *B,
                    swe_fields in, swe_fields out, double dt, swe_scalars *scal,
                    void *stream);

/*
 * adj_target - the adjoint data phi = (I, 0, 0) of eqs. (phi_1d)/(phi_Alaska):
 * I = exp(-r^2/R^2) (SWE_TARGET_GAUSS) or [r <= R] (SWE_TARGET_DISK), r the
 * distance of the cell centre from (xc, yc) (1D: |x - xc|), and 0 in cells
 * that are dry for the adjoint.  Writes all planes of `phi`.
 */
SWE_API swe_status adj_target(const swe_grid *grid, const swe_params *prm, const double *B,
                      double xc, double yc, double R, int32_t shape, swe_fields phi,
                      void *stream);

/*
 * swe_init - forward initial state from the initial surface eta0 (the sea
 * floor displacement carried to the surface, Sec. 1): nonlinear
 * h = max(0, eta0 - B), hu = hv = 0; linear eta = eta0 where wet, else 0.
 */
SWE_API swe_status swe_init(const swe_grid *grid, const swe_params *prm, const double *B,
                    const double *eta0, swe_fields q, void *stream);

/*
 * swe_max_speed - device max over wet cells of the largest characteristic
 * speed over cell size (nonlinear: max((|u|+sqrt(gh))/dx, (|v|+sqrt(gh))/dy);
 * linear/adjoint: sqrt(g hbar)/dx and /dy), as the bit pattern of a
 * non-negative double max-reduced into *out_bits (caller zeroes it).
 * adjoint != 0 uses the adjoint's static coefficients.
 */
SWE_API swe_status swe_max_speed(const swe_grid *grid, const swe_params *prm, const double *B,
                         swe_fields q, int32_t adjoint, uint64_t *out_bits, void *stream);

/*
 * adj_window - snapshot window of eq. (ip_timerange) (Sec. 4.2) for forward
 * time t, with snapshots k = 0..K at reversed adjoint time s_k = k (tf-t0)/K
 * (q^(tau = tf - s_k)).  tau ranges over [t, T], T = min(t + (tf - ts), tf);
 * the outward-bracketing frames are
 *   k_lo = max(0, floor((tf - T)/ds)), k_hi = min(K, ceil((tf - t)/ds)),
 * a ratio within 1e-9 of an integer counting as that integer.  Host only, pure.
 * Returns SWE_OK with k_lo <= k_hi, or SWE_OK with k_lo = 1, k_hi = 0 (empty)
 * when t > tf; SWE_E_INVAL for K < 1 or tf <= t0.
 */
SWE_API swe_status adj_window(double t, double t0, double ts, double tf, int32_t K,
                      int32_t *k_lo, int32_t *k_hi);

/*
 * adj_flag - flagging pass (Secs. 4.1, 4.2, and Sec. 6 for wet/dry):
 *   m = max_{k_lo <= k <= k_hi} |(eta eta^_k + mu mu^_k) + gamma gamma^_k|
 * (1D: |eta eta^_k + mu mu^_k|), m = 0 where the forward or the adjoint cell is
 * dry, flag = (m > tol).  Forward eta = (h + B) - sea_level (nonlinear) or f0
 * (linear).  frames: (K+1) snapshots of ncomp (3 in 2D, 2 in 1D) planes with
 * the grid's pitch, snapshot k plane c at frames + (k*ncomp + c)*ny*pitch.
 * An empty window (k_lo > k_hi) gives m = 0.  flags (int8 plane) and the
 * optional maxip, flag_acc (|= flag), maxip_acc (= max(., m)) planes use the
 * grid's pitch.  bounds (device, nullable): the snapshots' non-zero boxes of
 * adj_frame_bounds; a snapshot whose box misses every cell of a group of 64
 * consecutive cells is not read for that group (its inner product there is
 * |0| = 0: the same m for a finite state, less traffic).
 */
SWE_API swe_status adj_flag(const swe_grid *grid, const swe_params *prm, const double *B,
                    swe_fields q, const double *frames, int32_t K, int32_t k_lo,
                    int32_t k_hi, double tol, int8_t *flags, double *maxip,
                    int8_t *flag_acc, double *maxip_acc, const int32_t *bounds, void *stream);

/*
 * adj_frame_bounds - for each snapshot k = 0..K of `frames` (laid out as for
 * adj_flag on `grid`), the smallest box holding every cell with a non-zero
 * value in any plane (a NaN counts as non-zero): bounds[4k..4k+3] =
 * (i_lo, i_hi, j_lo, j_hi), inclusive; (nx, -1, ny, -1) for a snapshot that is
 * zero everywhere.  The adjoint is exactly zero outside the domain of
 * dependence of the target (Sec. 4), so with a target of compact support
 * (the disk of Sec. 6) the snapshots near t_f have small boxes.  bounds:
 * device, 4*(K+1) int32, owned by the caller.  Enqueue only.  SWE_E_INVAL:
 * a bad grid, null frames or bounds, K < 0.
 */
SWE_API swe_status adj_frame_bounds(const swe_grid *grid, const double *frames, int32_t K, int32_t *bounds,
                                    void *stream);

/*
 * Device-side time-step control (the CFL rule of swe_run, phase B), so that a
 * sequence of forward steps needs no host round-trip and can be captured in
 * a HIP graph.  The control block lives in device memory (256-byte aligned
 * for speed: its Courant-number words then sit on lines of their own); the
 * state alternates between two plane sets a (cur = 0) and b (cur = 1).
 * After each attempt of length dt with Courant number cfl:
 *   cfl > cfl_max: rejected, dt = dt*cfl_desired/cfl;
 *   else accepted: cur ^= 1, t = (final ? t_out : t + dt),
 *        dt = dt*cfl_desired/cfl (unchanged if cfl = 0), done = final;
 * and the next dt is clamped to t_out - t (setting final) unless done.
 * Attempts while done do nothing.  Each step launch first applies the rule
 * to the previous attempt (whose Courant number is complete by then), so an
 * attempt costs exactly one kernel launch; swe_advance ends with one small
 * kernel that resolves the last attempt into ctl->s.
 */
#define SWE_CTL_SPREAD 8

typedef struct {
    double t;               /* time of the current state */
    double dt;              /* length of the next attempt */
    double t_out;           /* attempts never step past this time */
    int32_t cur;            /* 0: state in a, 1: state in b */
    int32_t final_step;     /* the next attempt ends exactly at t_out */
    int32_t done;           /* t == t_out */
    int32_t last_accepted;  /* the last attempt was accepted */
    int32_t n_accepted, n_rejected;
} swe_ctl_state;

typedef struct {
    swe_ctl_state s;        /* state after the last attempt (valid between swe_advance calls) */
    uint64_t cfl_bits;      /* Courant number of the last attempt */
    int32_t n_clamped, n_nonfinite;   /* cells clamped / non-finite in accepted attempts */
    int32_t n_flag_calls;   /* flag passes run by swe_advance_flagged */
    int32_t reserved;
    swe_ctl_state slot[2];  /* kernel-internal: state of the running attempts */
    uint8_t pad_[88];       /* kernel-internal: puts the ring 256 bytes in */
    /* kernel-internal: Courant numbers of the running attempts, attempt k's
     * being the largest of ring[k][j][0] over j < SWE_CTL_SPREAD: the
     * wavefronts of a launch spread their atomic maxima over these words, one
     * 128-byte line each (atomics on one word are serialised, and every
     * wavefront of the next attempt reads all of them: 8 words balance the
     * two); words 1 and 2 of each line
     * collect the attempt's clamped and non-finite cells, which are added to
     * n_clamped and n_nonfinite once the attempt is known to be accepted */
    uint64_t ring[3][SWE_CTL_SPREAD][16];
} swe_ctl;

/* swe_ctl_set - (device) ctl := {t, dt clamped to t_out - t, t_out, cur,
 * counters zero}.  Enqueued as a kernel (graph-safe). */
SWE_API swe_status swe_ctl_set(swe_ctl *ctl, double t, double dt, double t_out, int32_t cur,
                               void *stream);

/* swe_ctl_retarget - (device) start a new segment: t_out := t_out, done := 0,
 * dt re-clamped; t, dt, cur and the counters are kept. */
SWE_API swe_status swe_ctl_retarget(swe_ctl *ctl, double t_out, void *stream);

/*
 * swe_advance - n_attempts forward step attempts (model of prm: nonlinear
 * 2D or linear 1D) under the device-side control of `ctl`, each one a
 * swe_step from the current plane set into the other followed by the control
 * step above.  Enqueue only; read the control block back to see t, cur and
 * the counters.  a and b must not alias.
 */
SWE_API swe_status swe_advance(const swe_grid *grid, const swe_params *prm, const double *B,
                               swe_fields a, swe_fields b, swe_ctl *ctl, int32_t n_attempts,
                               void *stream);

/* ------------------------------------------------------------------------
 * Batched AMR level: many small patches (block-structured refinement, Sec. 1)
 * advanced together with one level-wide time step.
 * ------------------------------------------------------------------------ */

/* One patch: nx x ny cells stored at planes + offset with row pitch nx; its
 * own cell size and boundary conditions (walls for isolated patches). */
typedef struct {
    int64_t offset;
    int32_t nx, ny;         /* 2 <= nx, ny */
    int32_t bc[4];
    double dx, dy;
} swe_patch;

typedef enum {
    SWE_SCHED_STRIP = 0,    /* one patch strip (<= 60 columns) per wavefront */
    SWE_SCHED_PACKED = 1    /* strips of equal row count packed side by side into 64 lanes,
                               first-fit decreasing; jobs ordered longest first */
} swe_schedule_kind;

/*
 * swe_level_schedule - (host) build the wavefront schedule of a level.
 * A pass is one wavefront's work: up to 64 lanes, each lane a column of one
 * patch strip (the strip's columns plus 2 ghost columns each side); all its
 * patches are marched over rows pass_row0 .. pass_row0 + pass_rows - 1.  A job
 * is a run of passes (the strips of one patch), and jobs come longest first;
 * both launch modes take the passes in this order, each pass on its own.
 * With chunk_rows > 0 every pass taller than chunk_rows is cut into passes of
 * at most chunk_rows rows (each its own job: more wavefronts for small
 * levels, at the cost of the chunks' halo rows); with chunk_rows = 0 a pass
 * covers its patches' full height and every patch lies within one job.
 *   lanes:     n_passes*64 int64, lane = (patch << 32) | (role << 16) | (col + 32768),
 *              role bit 0: output column, bit 1: its west edge counts for the
 *              Courant number; -1 for an idle lane
 *   pass_rows, pass_row0: n_passes int32;  job_pass: n_jobs+1 int32 (passes of
 *              job j are job_pass[j] .. job_pass[j+1]-1)
 * Call with null outputs to get the sizes.  Returns n_passes (>= 0) and sets
 * *n_jobs, or a negative swe_status (SWE_E_INVAL for a patch with nx or ny
 * < 2, offset < 0, dx or dy <= 0, or a bc[k] that is not a swe_bc).
 * patches: host array.
 */
SWE_API int32_t swe_level_schedule(const swe_patch *patches, int32_t n_patches, int32_t kind, int32_t chunk_rows,
                                   int64_t *lanes, int32_t *pass_rows, int32_t *pass_row0, int32_t *job_pass,
                                   int32_t *n_jobs);

/* 32-bit words of a level's barrier (swe_level.sync). */
#define SWE_LEVEL_SYNC_WORDS 4096

/* A level on the device. */
typedef struct {
    int32_t n_patches, n_passes, n_jobs;
    int32_t chunk_rows;         /* the schedule's chunk_rows (0: whole patches) */
    const swe_patch *patches;   /* device table */
    const int64_t *lanes;       /* device, from swe_level_schedule */
    const int32_t *pass_rows;   /* device */
    const int32_t *job_pass;    /* device */
    uint32_t *sync;             /* device, SWE_LEVEL_SYNC_WORDS words zeroed once by the caller
                                   (persistent mode); word 2 is the barrier's error word */
    const int32_t *pass_row0;   /* device, first row of each pass (NULL: all 0) */
} swe_level;

/*
 * swe_level_advance - n_steps step attempts of the whole level (nonlinear
 * model) under device-side control `ctl` (the rule of swe_advance, with the
 * Courant number the max over all patches).  persistent = 0: one launch per
 * attempt, one wavefront per pass (graph-capturable).  persistent = 1: a
 * single cooperative launch of at most one wavefront per resident slot, in
 * workgroups of 8 (one per pass in eight, but at least one per CU while
 * there are passes for them), runs all attempts, the workgroups meeting at a grid
 * barrier after each attempt;
 * a barrier that does not open within a bounded spin sets sync[2] to nonzero
 * and the launch ends early (the caller checks sync[2]; the state is then
 * not a valid result).  The barrier orders each attempt's stores before the
 * next attempt's loads on every wavefront, so a level cut into row chunks
 * (chunk_rows > 0), whose chunks read halo rows that other wavefronts stored
 * in the previous attempt, runs in either mode.  State in a (cur = 0) /
 * b (cur = 1); B: bottom planes of the level.  Enqueue only.
 */
SWE_API swe_status swe_level_advance(const swe_level *level, const swe_params *prm, const double *B,
                                     swe_fields a, swe_fields b, swe_ctl *ctl, int32_t n_steps,
                                     int32_t persistent, void *stream);

/* One timed candidate of swe_level_tune. */
typedef struct {
    int32_t level;          /* index into the candidate levels */
    int32_t persistent;
    double us_per_attempt;
} swe_tune_entry;

/*
 * swe_level_tune - autotuner of the batched level: for every candidate level
 * schedule (levels[k], e.g. SWE_SCHED_STRIP and SWE_SCHED_PACKED of the same
 * patches) and both launch modes, run one untimed attempt from `init` (so
 * that one-time costs of the launch form are not timed), copy the state
 * `init` into `work_a`, run n_trial attempts from dt with the control rule,
 * time them with HIP events,
 * and compare the resulting state bit for bit with the first candidate's (kept
 * in `ref`).  Writes 2*n_levels entries to `out` (host) and the index of the
 * fastest into *best.  Returns SWE_E_HIP if two candidates disagree in any
 * bit (*mismatch, device int32, receives the count).  Synchronises `stream`.
 */
SWE_API swe_status swe_level_tune(const swe_level *const *levels, int32_t n_levels, const swe_params *prm,
                                  const double *B, swe_fields init, swe_fields work_a, swe_fields work_b,
                                  swe_fields ref, swe_ctl *ctl, int32_t *mismatch, double dt,
                                  int32_t n_trial, int64_t n_cells, swe_tune_entry *out, int32_t *best,
                                  void *stream);

/*
 * swe_surface_flag - the surface criterion the adjoint flagging is compared
 * with (Sec. 6: refine where the sea surface relative to sea level exceeds a
 * tolerance): flags[k] = 1 if cell k is wet and |eta| > tol, else 0, with
 * eta = (h + B) - sea_level and wet = h > dry_tol for the nonlinear model, and
 * eta = q.f0, wet = max(0, sea_level - B) > dry_tol for the linear model.
 * flags (nullable) and flag_acc (nullable, |= flag) are device int8 planes
 * with the grid's pitch.  Enqueue only.  SWE_E_INVAL: bad grid, null B or
 * q.f0, no output, non-finite tol.
 */
SWE_API swe_status swe_surface_flag(const swe_grid *grid, const swe_params *prm, const double *B, swe_fields q,
                                    double tol, int8_t *flags, int8_t *flag_acc, void *stream);

/*
 * adj_flag_interp - adj_flag with the snapshots on the adjoint's own grid
 * (Sec. 4: the adjoint is solved at a fixed, usually coarser resolution and
 * its values at the forward grid's locations come from linear, in 2D
 * bilinear, interpolation on the snapshot grid; Sec. 6: a cell that is wet in
 * the forward and dry in the adjoint problem gets inner product 0).
 * For forward cell (i, j) with centre x = x_lo + (i + 1/2) dx (y likewise),
 * on each axis of the adjoint grid u = (x - adj.x_lo)/adj.dx: the adjoint
 * cell is clamp(floor(u), 0, n-1) and the interpolation uses centres i0 and
 * i0 + 1 with i0 = clamp(floor(u - 1/2), 0, n-2) and weight
 * w = clamp(u - 1/2 - i0, 0, 1) (constant beyond the outermost centres);
 * q^ = (1-wy)((1-wx) q00 + wx q10) + wy((1-wx) q01 + wx q11).  The cell is
 * adjoint-wet iff max(0, sea_level - adj_B) > dry_tol in its adjoint cell.
 * frames: (K+1) * ncomp planes with adj_grid's pitch; bounds (nullable) are
 * boxes on adj_grid, and a snapshot is skipped for a cell when none of its
 * four interpolation corners lies in the box.  Other arguments and errors as
 * adj_flag.  Enqueue only.
 */
SWE_API swe_status adj_flag_interp(const swe_grid *grid, const swe_params *prm, const double *B, swe_fields q,
                                   const swe_grid *adj_grid, const double *adj_B, const double *frames,
                                   int32_t K, int32_t k_lo, int32_t k_hi, double tol, int8_t *flags,
                                   double *maxip, int8_t *flag_acc, double *maxip_acc, const int32_t *bounds,
                                   void *stream);

/* Flagging of a device-controlled forward run (see swe_advance_flagged). */
typedef struct {
    const double *frames;   /* (K+1) snapshots, as for adj_flag */
    int32_t K;
    int32_t flag_every;     /* >= 1 */
    double t0, ts, tf, tol;
    int8_t *flags_final;    /* flags of the attempt that reaches t_out (nullable) */
    int8_t *flag_acc;       /* OR of all flags (nullable) */
    double *maxip_acc;      /* max of all m (nullable) */
    const swe_grid *adj_grid;  /* snapshots on a grid of their own (as adj_flag_interp); NULL: the forward grid */
    const double *adj_B;       /* bottom on adj_grid (with adj_grid) */
    const int32_t *bounds;     /* non-zero boxes of the snapshots (adj_frame_bounds), nullable */
} swe_flagging;

/*
 * swe_advance_flagged - swe_advance with the flag pass of the driver after
 * every attempt, decided on the device: when the attempt is accepted and
 * either reaches t_out or brings the accepted-step count (since swe_ctl_set)
 * to a multiple of flag_every, the new state is flagged at the new time with
 * the window of adj_window; the flags of the attempt reaching t_out go to
 * flags_final.  Enqueue only.
 */
SWE_API swe_status swe_advance_flagged(const swe_grid *grid, const swe_params *prm, const double *B,
                                       swe_fields a, swe_fields b, swe_ctl *ctl, int32_t n_attempts,
                                       const swe_flagging *fl, void *stream);

/* ------------------------------------------------------------------------
 * Regridding: flagged cells -> rectangular boxes -> refined patches for the
 * batched level (the clustering step that follows flagging in block-
 * structured AMR, Sec. 1).
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t i_lo, j_lo;     /* lower-left cell of the box on the flagged grid */
    int32_t nx, ny;         /* box size in cells */
} swe_box;

/*
 * swe_cluster - (host) point clustering of the non-zero cells of flags
 * (ny rows of pitch bytes) into disjoint boxes by the signature method of
 * Berger and Rigoutsos.  Recursively, starting from the whole grid:
 *   1. shrink the box to the bounding box of its flagged cells (none: drop it);
 *   2. if n_flagged >= efficiency * area and both sides <= max_side, keep it;
 *   3. if it is efficient enough but too large, bisect the first side
 *      (x before y) longer than max_side at len/2;
 *   4. otherwise cut at a hole: a zero in the column (x) or row (y) signature,
 *      cutting before that column/row at c in [1, len-1]; among holes the
 *      one with the smallest |2c - len|, then x before y, then smaller c;
 *   5. else at the strongest inflection of a signature: with the Laplacian
 *      L[k] = S[k+1] - 2 S[k] + S[k-1] (1 <= k <= len-2), a cut at c = k+1
 *      where L[k] L[k+1] < 0, min_side <= c <= len - min_side, strength
 *      |L[k+1] - L[k]|; the strongest, then the smallest |2c - len|, then x
 *      before y, then smaller c;
 *   6. else bisect the longer side (x if equal) at len/2 if both halves have
 *      >= min_side cells, else the other side; if neither, keep the box.
 * The lower part is processed before the upper.  Returns the number of boxes
 * (writing at most max_boxes of them), or a negative swe_status
 * (SWE_E_INVAL: null pointers, sizes < 1, efficiency outside (0, 1],
 * min_side < 1, max_side < 2 min_side).
 */
SWE_API int32_t swe_cluster(const int8_t *flags, int32_t nx, int32_t ny, int32_t pitch, double efficiency,
                            int32_t min_side, int32_t max_side, swe_box *boxes, int32_t max_boxes);

/*
 * swe_prolong - fill refined patches from the coarse grid by piecewise-
 * constant injection: fine cell (i, j) of patch k (the box boxes[k] refined
 * by `ratio`, stored as described by patches[k], pitch = patches[k].nx) takes
 * the values of coarse cell (i_lo + i / ratio, j_lo + j / ratio), for the
 * three state planes and the bottom (a parent index outside the grid is
 * clamped to it).  Conserves mass and keeps a lake at rest at rest.  boxes and patches are device arrays of n entries; out_B / out_q
 * are the level's planes.  Enqueue only.  SWE_E_INVAL: null pointers,
 * n < 1, ratio < 1.
 */
SWE_API swe_status swe_prolong(const swe_grid *grid, const double *B, swe_fields q, const swe_box *boxes,
                               const swe_patch *patches, int32_t n, int32_t ratio, double *out_B,
                               swe_fields out_q, void *stream);

/* ------------------------------------------------------------------------
 * Serving: scenarios (a tsunami source on a grid, with its target region and
 * time window) arriving over time, run through the two-phase driver with
 * several in flight at once.
 * ------------------------------------------------------------------------ */
typedef struct {
    double arrival;             /* seconds after the start of swe_serve */
    swe_grid grid;              /* pitch must equal nx */
    swe_params params;
    const double *B_host;       /* host, ny*nx: bottom elevation */
    const double *eta0_host;    /* host, ny*nx: initial surface */
    double target_xc, target_yc, target_R;
    int32_t target_shape, K;
    double t0, ts, tf, tol;
    int32_t flag_every, reserved;
    int8_t *flag_acc_host;      /* host outputs, ny*nx each (nullable) */
    double *maxip_acc_host;
    double *q_host[3];          /* final state planes (nullable) */
} swe_request;

typedef struct {
    double admitted;            /* seconds after the start: memory and a slot granted */
    double finished;            /* results copied back */
    double latency;             /* finished - arrival (finished when not realtime) */
    int32_t status;             /* swe_status of the run */
    int32_t slot;               /* worker that ran it */
    int32_t n_adj_steps, n_fwd_steps;
    size_t bytes;               /* device footprint */
} swe_request_stats;

typedef struct {
    void *arena;                /* device memory scenarios are carved from (256-byte aligned) */
    size_t arena_bytes;
    int32_t max_active;         /* scenarios in flight, one stream and host thread each (>= 1) */
    int32_t realtime;           /* 1: a request is not admitted before its arrival time */
    /* optional (may be NULL): called on a worker thread after a request's
     * results are back, with its index in req, a copy of its complete stats
     * and user; calls come in completion order and may overlap; the callback
     * must not call swe_serve */
    void (*on_done)(int32_t index, const swe_request_stats *stats, void *user);
    void *user;
} swe_serve_config;

/* Device bytes one request occupies while it runs (0 on bad input). */
SWE_API size_t swe_serve_footprint(const swe_request *req);

/*
 * swe_serve - continuous serving of n requests (in order of arrival).
 * Requests are admitted first-come first-served as soon as (realtime) they
 * have arrived, a slot is free and their footprint fits in the arena (first
 * fit); each admitted request copies its inputs to the device, runs swe_run
 * on its slot's stream while other requests run on theirs, copies its outputs
 * back and frees its memory, which admits the next ones.  max_active = 1 gives
 * the plain sequential solver.  A request whose footprint exceeds the arena is
 * refused (status SWE_E_NOMEM) without blocking the others.  Blocks until all
 * requests are done; per-request timing in stats.  Returns the first failing
 * request's status, else SWE_OK.
 */
SWE_API swe_status swe_serve(const swe_request *req, int32_t n, const swe_serve_config *cfg,
                             swe_request_stats *stats);

/* Full problem of the two-phase driver. */
typedef struct {
    swe_grid grid;
    swe_params params;      /* params.model: NONLINEAR needs ny >= 2; LINEAR 1D or 2D */
    const double *B;        /* device bottom elevation */
    const double *eta0;     /* device initial surface */
    double target_xc, target_yc, target_R;
    int32_t target_shape;
    int32_t K;              /* snapshots k = 0..K */
    double t0, ts, tf;      /* run [t0, tf]; target time range [ts, tf] */
    double tol;             /* flagging tolerance */
    int32_t flag_every;     /* flag after every flag_every accepted steps (>= 1) */
    int32_t full_frames;    /* 0: the flag passes skip the snapshots that are exactly zero over a
                               group of cells (adj_frame_bounds); 1: they read every snapshot in full
                               (same results for finite states) */
    double *frames;         /* device, (K+1)*ncomp*ny*pitch doubles of the adjoint grid (output) */
    swe_fields q_out;       /* device, final forward state (output) */
    int8_t *flags_at;       /* device, (K+1)*ny*pitch: flags at t0 + j ds; nullable */
    int8_t *flag_acc;       /* device plane, OR of all flags (caller zeroes); nullable */
    double *maxip_acc;      /* device plane, max of all m (caller zeroes); nullable */
    double surface_tol;     /* tolerance of the surface criterion (with surface_flags_at) */
    int8_t *surface_flags_at; /* device, (K+1)*ny*pitch: swe_surface_flag at t0 + j ds, for
                                 comparison with flags_at; nullable */
    swe_grid adj_grid;      /* adj_grid.nx == 0: the adjoint runs on the forward grid; else on this
                               grid (same dimension, its own resolution), frames have its size and
                               the flags interpolate the snapshots (adj_flag_interp) */
    const double *adj_B;    /* device bottom on adj_grid (with adj_grid) */
    int32_t launch_per_step; /* 1D problems: 0 runs each phase of a grid of up to 3840 cells in one
                                workgroup (state in LDS, one launch per phase, the flagged states
                                recorded and flagged afterwards); 1 launches every step and flag
                                pass as for 2D grids (same results bit for bit for finite states;
                                the workgroup needs 32 B of LDS per cell, and a grid that does not
                                fit runs step by step either way).  2D: ignored. */
    int32_t reserved;
} swe_problem;

typedef struct {
    int32_t n_adj_steps, n_sub, n_fwd_steps, n_rejected, n_flag_calls, n_clamped;
    double dt_adj, t_end;
} swe_result;

/* Bytes of device workspace swe_run needs for this problem (0 on bad input). */
SWE_API size_t swe_run_workspace_bytes(const swe_problem *pb);

/*
 * swe_run - the two-phase driver of Sec. 4.
 * A. adjoint: q~(0) = phi; constant dt = ds/n_sub with ds = (tf - t0)/K,
 *    n_sub = ceil(ds/dt_cfl), dt_cfl = cfl_desired/max(cmax/dx, cmax/dy);
 *    snapshot k (k = 0..K) = q~ after k*n_sub steps, i.e. q^ at tf - k ds.
 * B. forward from t0 with the state of swe_init: flag at t0; then repeat
 *    { dt = dt0 at first, else dt*cfl_desired/cfl of the previous attempt
 *      (unchanged if cfl = 0), clamped to the next output time t0 + j ds
 *      (the last is tf); step; if cfl > cfl_max the step is discarded and
 *      retried; else accept, and flag when an output time was reached (flags
 *      at output j stored in flags_at[j]) or the number of accepted steps is
 *      a multiple of flag_every } until tf.
 * Synchronises `stream` (it reads the Courant number of each step) and
 * returns when the run has completed.  workspace: device, at least
 * swe_run_workspace_bytes(pb) bytes, 256-byte aligned.  Errors: SWE_E_NONFINITE
 * (a non-finite state), SWE_E_CFL (more than 1000 rejected attempts, or the
 * time step fell a million times below dt0 or stopped advancing t: the state
 * has blown up, e.g. a thin fast layer at a shoreline wall).
 */
SWE_API swe_status swe_run(const swe_problem *pb, void *workspace, size_t workspace_bytes,
                   swe_result *res, void *stream);

/*
 * swe_run_static - swe_run for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same driver, whose workspace is instead a fixed array of
 * SWE_STATIC_WORKSPACE_BYTES in the library's device memory (one per GPU,
 * held from the first call on that GPU until the process ends).  It calls no
 * allocating routine; the caller still provides every input and output of
 * the problem.  A problem whose swe_run_workspace_bytes exceed the array
 * (grids beyond about 1170^2 cells with pitch = nx) is refused with
 * SWE_E_NOMEM before anything is enqueued.  All calls on one GPU share its
 * array: calls that overlap in time on the same GPU (other host threads,
 * other streams) race and must be serialised by the caller.  Otherwise as
 * swe_run (synchronises `stream`, same results bit for bit).
 */
#define SWE_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
SWE_API swe_status swe_run_static(const swe_problem *pb, swe_result *res, void *stream);

/* Message for the last non-OK status returned on this thread ("" if none). */
SWE_API const char *swe_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SWE_H */
