/*
 * CPU oracle interface.  TEST INFRASTRUCTURE ONLY: used by the tests, the
 * smoke check and the CPU-baseline leg of the benchmark; never by the HIP
 * library, which has its own, separately written header.
 *
 * All arrays are host, float64 (flags int8), row-major (ny, nx), x fastest,
 * without ghost cells.  Returns 0 on success, negative on bad arguments.
 */
#ifndef SWE_ORACLE_H
#define SWE_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_BC_WALL = 0, OR_BC_EXTRAP = 1 };
enum { OR_NONLINEAR = 0, OR_LINEAR = 1 };

typedef struct {
    int nx, ny;           /* ny == 1: one space dimension (linear model / adjoint) */
    double dx, dy;
    double x_lo, y_lo;    /* lower-left corner; cell centres at x_lo + (i+1/2) dx */
    int bc[4];            /* x_lo, x_hi, y_lo, y_hi */
} or_grid;

typedef struct {
    double g, sea_level, dry_tol, cfl_desired, cfl_max;
    int order;            /* 1 or 2 */
    int transverse;       /* 0 or 1 */
} or_params;

typedef struct {
    or_grid grid;
    or_params params;
    int model;            /* OR_NONLINEAR (2D) or OR_LINEAR (1D or 2D) */
    const double *B, *eta0;
    double target_xc, target_yc, target_R;
    int target_shape;     /* 0 Gaussian, 1 disk */
    double t0, ts, tf, tol;
    int K, flag_every;
    double *frames;       /* (K+1) * ncomp planes of the adjoint grid */
    double *q_out[3];
    signed char *flags_at;  /* (K+1) * nx * ny, nullable */
    signed char *flag_acc;  /* nullable */
    double *maxip_acc;      /* nullable */
    double surface_tol;             /* tolerance of the surface criterion */
    signed char *surface_flags_at;  /* (K+1) * nx * ny surface flags at t0 and the output times, nullable */
    or_grid adj_grid;               /* nx == 0: the adjoint runs on the forward grid; else on this one */
    const double *adj_B;            /* bottom on adj_grid */
    double *maxip_at;               /* (K+1) * nx * ny: the max inner product m of the flag pass at t0 and
                                       at each output time (the values flags_at thresholds), nullable */
} or_problem;

typedef struct {
    int n_adj_steps, n_sub, n_fwd_steps, n_rejected, n_flag_calls, n_clamped, status;
    double dt_adj, t_end;
} or_result;

int or_swe_step(const or_grid *G, const or_params *P, const double *B,
                const double *h, const double *hu, const double *hv,
                double *ho, double *huo, double *hvo, double dt,
                double *cfl_out, int *n_clamped);
int or_lin_step(const or_grid *G, const or_params *P, const double *B,
                const double *q0, const double *q1, double *o0, double *o1,
                double dt, double *cfl_out);
int or_lin_step2d(const or_grid *G, const or_params *P, const double *B,
                  const double *q0, const double *q1, const double *q2,
                  double *o0, double *o1, double *o2, double dt, double *cfl_out);
int or_adj_step(const or_grid *G, const or_params *P, const double *B,
                const double *q0, const double *q1, const double *q2,
                double *o0, double *o1, double *o2, double dt, double *cfl_out);
void or_target(const or_grid *G, const or_params *P, const double *B,
               double xc, double yc, double R, int shape, double *phi);
void or_init_state(const or_grid *G, const or_params *P, int model, const double *B,
                   const double *eta0, double *q0, double *q1, double *q2);
double or_dt0(const or_grid *G, const or_params *P, int model, const double *B,
              const double *q0, const double *q1, const double *q2);
int or_adj_nsub(const or_grid *G, const or_params *P, const double *B,
                double t0, double tf, int K, double *dt_out);
int or_window(double t, double t0, double ts, double tf, int K, int *k_lo, int *k_hi);
void or_flag(const or_grid *G, const or_params *P, int model, const double *B,
             const double *q0, const double *q1, const double *q2,
             const double *frames, int K, int k_lo, int k_hi, double tol,
             signed char *flags, double *maxip, signed char *flag_acc, double *maxip_acc);
void or_surface_flag(const or_grid *G, const or_params *P, int model, const double *B,
                     const double *q0, double tol, signed char *flags, signed char *flag_acc);
void or_interp(const or_grid *G, const or_grid *Ga, const double *v, double *out);
void or_flag_interp(const or_grid *G, const or_params *P, int model, const double *B,
                    const double *q0, const double *q1, const double *q2,
                    const or_grid *Ga, const double *Ba, const double *frames, int K, int k_lo, int k_hi,
                    double tol, signed char *flags, double *maxip, signed char *flag_acc, double *maxip_acc);
int or_run(const or_problem *pb, or_result *res);
/* threads of the row loops (results do not depend on it) */
void or_set_threads(int n);
/* test hook: the two parts of the adjoint transverse split (pins only) */
void or_adj_split_parts(double cL, double cR, int ydir, const double *a, double *pos, double *neg);

#ifdef __cplusplus
}
#endif
#endif
