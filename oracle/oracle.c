/*
 * CPU oracle for adjoint-guided refinement flagging in shallow-water tsunami
 * modelling (Davis & LeVeque, "Adjoint methods for guiding adaptive mesh
 * refinement in tsunami modeling").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * HIP library is checked against.  Only the test-suite, the smoke check and
 * the CPU-baseline leg of the benchmark may load it; the library never does.
 * It shares no code, header, table or helper with the HIP path.
 *
 * Arithmetic: IEEE binary64, round-to-nearest, built with -ffp-contract=off
 * (no fused multiply-add), no fast-math.  Every expression is evaluated in the
 * order written.  OpenMP (if enabled) only splits independent rows; the
 * reductions are max (exact) and integer sums, so results do not depend on the
 * thread count.
 *
 * What is computed (paper sections and equations in brackets):
 *   - nonlinear 2D shallow water [eq. (swe), Sec. 5] by the wave-propagation
 *     finite-volume method: f-wave Roe solver with the bathymetry source
 *     folded into the flux difference, MC-limited second-order corrections,
 *     transverse fluctuation splitting, walls at wet/dry interfaces, dry-cell
 *     threshold and CFL number;
 *   - 1D linearized shallow water [eqs. (swe_1d_linearized), (hyp_linear),
 *     Sec. 3] in wave form;
 *   - the time-reversed adjoint q~_t - (A^T q~)_x = 0 in 1D and
 *     q~_t - (A1^T q~)_x - (A2^T q~)_y = 0 in 2D [eq. (adjoint1), Sec. 4 and
 *     the 2D adjoint of Sec. 5], with zero normal velocity at walls and
 *     wet/dry interfaces;
 *   - the target functional data phi = (I, 0, 0) [eqs. (phi_1d),
 *     (phi_Alaska)], Gaussian or disk shaped;
 *   - the snapshot window of eq. (ip_timerange) (Sec. 4.2) and the
 *     per-cell flag max_k |q^T q^_k| > tol with the wet/dry rule of Sec. 6;
 *   - the two-phase driver (adjoint snapshots, then forward run with
 *     flagging) of Sec. 4.
 * Readings where the paper is silent (numerical scheme details, window
 * bracketing, etc.) are listed in the design notes; each function below
 * states the rule it implements.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXD(a, b) ((a) > (b) ? (a) : (b))
#define MIND(a, b) ((a) < (b) ? (a) : (b))

/* ------------------------------------------------------------------------ */
/* padded arrays: two ghost cells on every side                             */
/* ------------------------------------------------------------------------ */
typedef struct {
    int nx, ny, ng;   /* ng = 2 in 2D; in 1D the y-direction has no ghosts */
    int px, py;       /* padded extents */
    double *v;
} pad_t;

static pad_t pad_new(int nx, int ny, int twod)
{
    pad_t p;
    p.nx = nx; p.ny = ny; p.ng = 2;
    p.px = nx + 4;
    p.py = twod ? ny + 4 : 1;
    p.v = (double *)calloc((size_t)p.px * (size_t)p.py, sizeof(double));
    return p;
}

/* element (i, j) with i in [-2, nx+2), j in [-2, ny+2) (2D) or j = 0 (1D) */
static inline double *PA(const pad_t *p, int i, int j)
{
    int jj = (p->py == 1) ? 0 : j + 2;
    return &p->v[(size_t)jj * p->px + (size_t)(i + 2)];
}

static void pad_free(pad_t *p) { free(p->v); p->v = NULL; }

/* Copy an interior (ny, nx) array into a padded one. */
static void pad_load(pad_t *p, const double *src)
{
    int ny = (p->py == 1) ? 1 : p->ny;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < p->nx; i++)
            *PA(p, i, j) = src[(size_t)j * p->nx + i];
}

/*
 * Ghost cells (walls are the boundary condition of the paper's examples,
 * Sec. 3 and the 2D adjoint boundary discussion of Sec. 5).
 *   WALL:   ghost k (k = 0, 1 counted outward) mirrors interior cell k; the
 *           component normal to that boundary is negated.
 *   EXTRAP: ghost copies the edge cell.
 * Fill order: first the x-ghosts of the interior rows, then the y-ghosts of
 * all padded columns (this defines the corner ghosts).
 * ncomp arrays are filled together; xneg / yneg give the index of the
 * component negated at x-walls / y-walls (-1: none).
 */
static void fill_ghosts(pad_t *a, int ncomp, const int bc[4], int xneg, int yneg)
{
    int nx = a[0].nx, ny = a[0].ny;
    int twod = a[0].py != 1;
    int nrows = twod ? ny : 1;
    for (int c = 0; c < ncomp; c++) {
        for (int j = 0; j < nrows; j++) {
            for (int k = 0; k < 2; k++) {
                /* low x side: ghost i = -1-k */
                if (bc[0] == OR_BC_WALL) {
                    double v = *PA(&a[c], k, j);
                    *PA(&a[c], -1 - k, j) = (c == xneg) ? -v : v;
                } else {
                    *PA(&a[c], -1 - k, j) = *PA(&a[c], 0, j);
                }
                /* high x side: ghost i = nx+k */
                if (bc[1] == OR_BC_WALL) {
                    double v = *PA(&a[c], nx - 1 - k, j);
                    *PA(&a[c], nx + k, j) = (c == xneg) ? -v : v;
                } else {
                    *PA(&a[c], nx + k, j) = *PA(&a[c], nx - 1, j);
                }
            }
        }
        if (!twod) continue;
        for (int i = -2; i < nx + 2; i++) {
            for (int k = 0; k < 2; k++) {
                if (bc[2] == OR_BC_WALL) {
                    double v = *PA(&a[c], i, k);
                    *PA(&a[c], i, -1 - k) = (c == yneg) ? -v : v;
                } else {
                    *PA(&a[c], i, -1 - k) = *PA(&a[c], i, 0);
                }
                if (bc[3] == OR_BC_WALL) {
                    double v = *PA(&a[c], i, ny - 1 - k);
                    *PA(&a[c], i, ny + k) = (c == yneg) ? -v : v;
                } else {
                    *PA(&a[c], i, ny + k) = *PA(&a[c], i, ny - 1);
                }
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* shared small pieces of the wave-propagation method                       */
/* ------------------------------------------------------------------------ */
enum { E_DRY = 0, E_WET = 1, E_WALL_LO = 2, E_WALL_HI = 3 };

/*
 * One edge, waves and speeds in the edge's normal frame (h-like, normal,
 * tangential) and fluctuations in the physical frame.
 */
typedef struct {
    int type;
    int nw;              /* number of wave families */
    double s[3];         /* speeds */
    double Z[3][3];      /* waves (f-waves, or plain waves for the 1D linear model) */
    double amdq[3], apdq[3];
    /* eigen-structure data used to split transverse fluctuations */
    double un, vt, r2c;  /* nonlinear: Roe normal/tangential velocity, 1/(2c) */
    double cl, cr, rc;   /* linear/adjoint: sound speeds of the two cells, 1/(cl+cr) */
} edge_t;

/* MC limiter: phi(theta) = max(0, min((1+theta)/2, 2, 2 theta)). */
static double mc_phi(double theta)
{
    double a = 0.5 * (1.0 + theta);
    double b = MIND(a, 2.0);
    double c = MIND(b, 2.0 * theta);
    return MAXD(0.0, c);
}

static double dot3(const double *a, const double *b)
{
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

/*
 * Limited wave p of edge e given the same family's wave at the upwind edge:
 *   theta = (Z_up . Z) / (Z . Z),  Ztilde = phi_MC(theta) Z,  0 if Z . Z = 0.
 */
static void limited_wave(const double *Z, const double *Zup, double *Zt)
{
    double dd = dot3(Z, Z);
    if (dd == 0.0) {
        Zt[0] = Zt[1] = Zt[2] = 0.0;
        return;
    }
    double theta = dot3(Zup, Z) / dd;
    double phi = mc_phi(theta);
    Zt[0] = phi * Z[0];
    Zt[1] = phi * Z[1];
    Zt[2] = phi * Z[2];
}

/*
 * Second-order correction flux of one edge (normal frame), from its waves and
 * the waves of its two neighbours along the sweep (lo = e-1, hi = e+1):
 *   F = 1/2 sum_p w_p(s_p) Ztilde_p, the upwind edge of family p being lo if
 *   s_p > 0 and hi otherwise.
 * fwave = 1: w = sgn(s) (1 - nu|s|)   (f-waves)
 * fwave = 0: w = |s| (1 - nu|s|)      (plain waves)
 */
static void correction(const edge_t *e, const edge_t *lo, const edge_t *hi,
                       double nu, int fwave, double *F)
{
    double cx[3] = {0.0, 0.0, 0.0};
    for (int p = 0; p < e->nw; p++) {
        const edge_t *up = (e->s[p] > 0.0) ? lo : hi;
        double Zt[3];
        limited_wave(e->Z[p], up->Z[p], Zt);
        double as = fabs(e->s[p]);
        double a = 1.0 - nu * as;
        double w;
        if (fwave)
            w = (e->s[p] > 0.0) ? a : ((e->s[p] < 0.0) ? -a : 0.0);
        else
            w = as * a;
        cx[0] = cx[0] + w * Zt[0];
        cx[1] = cx[1] + w * Zt[1];
        cx[2] = cx[2] + w * Zt[2];
    }
    F[0] = 0.5 * cx[0];
    F[1] = 0.5 * cx[1];
    F[2] = 0.5 * cx[2];
}

/* Split waves into fluctuations: negative speeds left, positive right, zero
 * speed half to each side; p in increasing order. */
static void fluctuations_normal(const edge_t *e, double *am, double *ap)
{
    am[0] = am[1] = am[2] = 0.0;
    ap[0] = ap[1] = ap[2] = 0.0;
    for (int p = 0; p < e->nw; p++) {
        for (int c = 0; c < 3; c++) {
            double z = e->Z[p][c];
            if (e->s[p] < 0.0) {
                am[c] = am[c] + z;
            } else if (e->s[p] > 0.0) {
                ap[c] = ap[c] + z;
            } else {
                am[c] = am[c] + 0.5 * z;
                ap[c] = ap[c] + 0.5 * z;
            }
        }
    }
}

/* normal frame <-> physical frame.  x-edges: (h, hu, hv) = (h, n, t);
 * y-edges: (h, hu, hv) = (h, t, n). */
static void to_phys(int ydir, const double *nf, double *ph)
{
    if (!ydir) { ph[0] = nf[0]; ph[1] = nf[1]; ph[2] = nf[2]; }
    else       { ph[0] = nf[0]; ph[1] = nf[2]; ph[2] = nf[1]; }
}
static void to_normal(int ydir, const double *ph, double *nf)
{
    if (!ydir) { nf[0] = ph[0]; nf[1] = ph[1]; nf[2] = ph[2]; }
    else       { nf[0] = ph[0]; nf[1] = ph[2]; nf[2] = ph[1]; }
}

/* ------------------------------------------------------------------------ */
/* nonlinear shallow water: f-wave Roe solver                               */
/* ------------------------------------------------------------------------ */
/*
 * Cell data in an edge's normal frame: depth h, normal momentum hn,
 * tangential momentum ht, bottom B, and the velocities un = hn/h, vt = ht/h,
 * sq = sqrt(h) (only meaningful in wet cells).
 */
typedef struct { double h, hn, ht, B, un, vt, sq; int wet; } nlcell_t;

/*
 * f-wave Riemann solver for eq. (swe) across one edge, bathymetry source
 * folded into the flux difference (f-wave method for spatially varying
 * fluxes and sources, Bale-LeVeque-Mitran-Rossmanith 2002):
 *   Roe averages  hbar = (hL+hR)/2,
 *                 uhat = (sqL uL + sqR uR)/(sqL+sqR), vhat likewise,
 *                 chat = sqrt(g hbar);   speeds uhat - chat, uhat, uhat + chat
 *   flux jump minus source:
 *     d1 = hnR - hnL
 *     d2 = (hnR uR - hnL uL) + g hbar ((hR - hL) + (BR - BL))
 *     d3 = hnR vR - hnL vL
 *   (g hbar (dh + dB) equals 1/2 g d(h^2) + g hbar dB; this grouping makes a
 *   lake at rest produce exactly zero waves.)
 *   beta1 = (s3 d1 - d2)/(2 chat), beta3 = (d2 - s1 d1)/(2 chat),
 *   beta2 = d3 - vhat d1;  Z1 = beta1 (1, s1, vhat), Z2 = (0, 0, beta2),
 *   Z3 = beta3 (1, s3, vhat).
 * Wet/dry: a cell is wet iff h > dry_tol.  If exactly one side is dry it is
 * replaced by the mirror image of the wet side (h, -hn, ht, B) - a wall - and
 * only the fluctuation into the wet cell is kept.  Dry-dry edges carry nothing.
 */
static void nl_solve(const nlcell_t *Lc, const nlcell_t *Rc, double g, edge_t *e)
{
    memset(e, 0, sizeof(*e));
    e->nw = 3;
    nlcell_t L = *Lc, R = *Rc;
    if (!L.wet && !R.wet) {
        e->type = E_DRY;
        return;
    }
    if (L.wet && !R.wet) {
        e->type = E_WALL_LO;
        R = L; R.hn = -L.hn; R.un = -L.un;
    } else if (!L.wet && R.wet) {
        e->type = E_WALL_HI;
        L = R; L.hn = -R.hn; L.un = -R.un;
    } else {
        e->type = E_WET;
    }
    double hbar = 0.5 * (L.h + R.h);
    double rsw = 1.0 / (L.sq + R.sq);
    double uhat = (L.sq * L.un + R.sq * R.un) * rsw;
    double vhat = (L.sq * L.vt + R.sq * R.vt) * rsw;
    double ghbar = g * hbar;
    double chat = sqrt(ghbar);
    double s1 = uhat - chat, s2 = uhat, s3 = uhat + chat;
    double d1 = R.hn - L.hn;
    double d2 = (R.hn * R.un - L.hn * L.un) + ghbar * ((R.h - L.h) + (R.B - L.B));
    double d3 = R.hn * R.vt - L.hn * L.vt;
    double r2c = 1.0 / (2.0 * chat);
    double beta1 = (s3 * d1 - d2) * r2c;
    double beta3 = (d2 - s1 * d1) * r2c;
    double beta2 = d3 - vhat * d1;
    e->s[0] = s1; e->s[1] = s2; e->s[2] = s3;
    e->Z[0][0] = beta1; e->Z[0][1] = beta1 * s1; e->Z[0][2] = beta1 * vhat;
    e->Z[1][0] = 0.0;   e->Z[1][1] = 0.0;        e->Z[1][2] = beta2;
    e->Z[2][0] = beta3; e->Z[2][1] = beta3 * s3; e->Z[2][2] = beta3 * vhat;
    e->un = uhat; e->vt = vhat; e->r2c = r2c;
}

/*
 * Split a physical fluctuation a on the eigenvectors of a wet-wet edge
 * (nonlinear Roe eigen-structure, normal frame):
 *   r1 = (1, s1, vt), r2 = (0, 0, 1), r3 = (1, s3, vt)
 *   g1 = (s3 a_h - a_n)/(2c), g3 = (a_n - s1 a_h)/(2c), g2 = a_t - vt a_h
 * and return sum_p k_p r_p (physical frame) with k_p = max(s_p, 0) g_p
 * (positive = 1) or min(s_p, 0) g_p (positive = 0).
 */
static void nl_split(const edge_t *e, int ydir, const double *a_ph, int positive, double *out_ph)
{
    double a[3];
    to_normal(ydir, a_ph, a);
    double gm[3];
    gm[0] = (e->s[2] * a[0] - a[1]) * e->r2c;
    gm[1] = a[2] - e->vt * a[0];
    gm[2] = (a[1] - e->s[0] * a[0]) * e->r2c;
    double r[3][3] = {{1.0, e->s[0], e->vt}, {0.0, 0.0, 1.0}, {1.0, e->s[2], e->vt}};
    double k[3];
    for (int p = 0; p < 3; p++)
        k[p] = (positive ? MAXD(e->s[p], 0.0) : MIND(e->s[p], 0.0)) * gm[p];
    double nf[3];
    for (int c = 0; c < 3; c++)
        nf[c] = (k[0] * r[0][c] + k[1] * r[1][c]) + k[2] * r[2][c];
    to_phys(ydir, nf, out_ph);
}

/* index helpers for the edge arrays */
typedef struct { int nx, ny; edge_t *x, *y; } edges2d_t;
/* x-edge at i-1/2 (between cells i-1 and i), i in [-1, nx+1], row j in [-1, ny] */
static inline edge_t *XE(const edges2d_t *E, int i, int j)
{
    return &E->x[(size_t)(j + 1) * (E->nx + 3) + (i + 1)];
}
/* y-edge at j-1/2 (between rows j-1 and j), column i in [-1, nx], j in [-1, ny+1] */
static inline edge_t *YE(const edges2d_t *E, int i, int j)
{
    return &E->y[(size_t)(j + 1) * (E->nx + 2) + (i + 1)];
}

static edges2d_t edges_new(int nx, int ny)
{
    edges2d_t E;
    E.nx = nx; E.ny = ny;
    E.x = (edge_t *)calloc((size_t)(nx + 3) * (ny + 2), sizeof(edge_t));
    E.y = (edge_t *)calloc((size_t)(nx + 2) * (ny + 3), sizeof(edge_t));
    return E;
}
static void edges_free(edges2d_t *E) { free(E->x); free(E->y); }

/* Split function type: split a physical fluctuation on edge e (ydir) */
typedef void (*split_fn)(const edge_t *e, int ydir, const double *a, int positive, double *out);

/*
 * Generic unsplit 2D wave-propagation update (LeVeque 2002, Ch. 21) given
 * solved edges:
 *   Ft(i-1/2,j) = Fcorr - (nu_y/2) [A+ B+dQ(i-1,j-1/2) + A+ B-dQ(i-1,j+1/2)
 *                                   + A- B+dQ(i,j-1/2) + A- B-dQ(i,j+1/2)]
 *   Gt(i,j-1/2) = Gcorr - (nu_x/2) [B+ A+dQ(i-1/2,j-1) + B+ A-dQ(i+1/2,j-1)
 *                                   + B- A+dQ(i-1/2,j) + B- A-dQ(i+1/2,j)]
 * each transverse fluctuation being split with the eigen-structure of the
 * edge that receives it (the pair of cells sharing the receiving cell), and
 * contributing only if both that edge and the source edge are wet-wet.
 *   Q^{n+1} = Q - nu_x (A+dQ_W + A-dQ_E) - nu_y (B+dQ_S + B-dQ_N)
 *               - nu_x (Ft_E - Ft_W) - nu_y (Gt_N - Gt_S)
 * evaluated left to right.  Cells with wet[] == 0 are not updated.
 * Corrections are only formed on wet-wet edges.
 */
static void update2d(const edges2d_t *E, const pad_t *Q, int ncomp, const unsigned char *wet,
                     double nux, double nuy, int order, int transverse, int fwave,
                     split_fn split, double **out)
{
    int nx = E->nx, ny = E->ny;
    double hnux = 0.5 * nux, hnuy = 0.5 * nuy;
    /* correction fluxes, physical frame */
    double *Ft = (double *)calloc((size_t)3 * (nx + 1) * ny, sizeof(double));
    double *Gt = (double *)calloc((size_t)3 * nx * (ny + 1), sizeof(double));
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++) {
        for (int i = 0; i <= nx; i++) {
            const edge_t *e = XE(E, i, j);
            double *F = &Ft[3 * ((size_t)j * (nx + 1) + i)];
            F[0] = F[1] = F[2] = 0.0;
            if (e->type != E_WET) continue;
            double Fn[3] = {0.0, 0.0, 0.0}, Fp[3];
            if (order == 2) correction(e, XE(E, i - 1, j), XE(E, i + 1, j), nux, fwave, Fn);
            to_phys(0, Fn, Fp);
            if (transverse) {
                double ts[3] = {0.0, 0.0, 0.0}, part[3];
                const edge_t *src[4] = {YE(E, i - 1, j), YE(E, i - 1, j + 1), YE(E, i, j), YE(E, i, j + 1)};
                const double *fl[4] = {src[0]->apdq, src[1]->amdq, src[2]->apdq, src[3]->amdq};
                const int pos[4] = {1, 1, 0, 0};
                for (int m = 0; m < 4; m++) {
                    if (src[m]->type != E_WET) continue;
                    split(e, 0, fl[m], pos[m], part);
                    ts[0] = ts[0] + part[0];
                    ts[1] = ts[1] + part[1];
                    ts[2] = ts[2] + part[2];
                }
                for (int c = 0; c < 3; c++) Fp[c] = Fp[c] - hnuy * ts[c];
            }
            F[0] = Fp[0]; F[1] = Fp[1]; F[2] = Fp[2];
        }
    }
#pragma omp parallel for schedule(static)
    for (int j = 0; j <= ny; j++) {
        for (int i = 0; i < nx; i++) {
            const edge_t *e = YE(E, i, j);
            double *G = &Gt[3 * ((size_t)j * nx + i)];
            G[0] = G[1] = G[2] = 0.0;
            if (e->type != E_WET) continue;
            double Gn[3] = {0.0, 0.0, 0.0}, Gp[3];
            if (order == 2) correction(e, YE(E, i, j - 1), YE(E, i, j + 1), nuy, fwave, Gn);
            to_phys(1, Gn, Gp);
            if (transverse) {
                double ts[3] = {0.0, 0.0, 0.0}, part[3];
                const edge_t *src[4] = {XE(E, i, j - 1), XE(E, i + 1, j - 1), XE(E, i, j), XE(E, i + 1, j)};
                const double *fl[4] = {src[0]->apdq, src[1]->amdq, src[2]->apdq, src[3]->amdq};
                const int pos[4] = {1, 1, 0, 0};
                for (int m = 0; m < 4; m++) {
                    if (src[m]->type != E_WET) continue;
                    split(e, 1, fl[m], pos[m], part);
                    ts[0] = ts[0] + part[0];
                    ts[1] = ts[1] + part[1];
                    ts[2] = ts[2] + part[2];
                }
                for (int c = 0; c < 3; c++) Gp[c] = Gp[c] - hnux * ts[c];
            }
            G[0] = Gp[0]; G[1] = Gp[1]; G[2] = Gp[2];
        }
    }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; j++) {
        for (int i = 0; i < nx; i++) {
            size_t k = (size_t)j * nx + i;
            for (int c = 0; c < ncomp; c++) {
                double q = *PA(&Q[c], i, j);
                if (wet[k]) {
                    const double *FW = &Ft[3 * ((size_t)j * (nx + 1) + i)];
                    const double *FE = &Ft[3 * ((size_t)j * (nx + 1) + i + 1)];
                    const double *GS = &Gt[3 * ((size_t)j * nx + i)];
                    const double *GN = &Gt[3 * ((size_t)(j + 1) * nx + i)];
                    q = q - nux * (XE(E, i, j)->apdq[c] + XE(E, i + 1, j)->amdq[c]);
                    q = q - nuy * (YE(E, i, j)->apdq[c] + YE(E, i, j + 1)->amdq[c]);
                    q = q - nux * (FE[c] - FW[c]);
                    q = q - nuy * (GN[c] - GS[c]);
                }
                out[c][k] = q;
            }
        }
    }
    free(Ft);
    free(Gt);
}

/* CFL number: max over edges touching an interior cell of nu |s_p|. */
static double cfl2d(const edges2d_t *E, double nux, double nuy)
{
    int nx = E->nx, ny = E->ny;
    double cfl = 0.0;
#pragma omp parallel for reduction(max : cfl) schedule(static)
    for (int j = 0; j < ny; j++)
        for (int i = 0; i <= nx; i++) {
            const edge_t *e = XE(E, i, j);
            for (int p = 0; p < e->nw; p++) cfl = MAXD(cfl, nux * fabs(e->s[p]));
        }
#pragma omp parallel for reduction(max : cfl) schedule(static)
    for (int j = 0; j <= ny; j++)
        for (int i = 0; i < nx; i++) {
            const edge_t *e = YE(E, i, j);
            for (int p = 0; p < e->nw; p++) cfl = MAXD(cfl, nuy * fabs(e->s[p]));
        }
    return cfl;
}

static void nl_split_cb(const edge_t *e, int ydir, const double *a, int positive, double *out)
{
    nl_split(e, ydir, a, positive, out);
}

int or_swe_step(const or_grid *G, const or_params *P, const double *B,
                const double *h, const double *hu, const double *hv,
                double *ho, double *huo, double *hvo, double dt,
                double *cfl_out, int *n_clamped)
{
    int nx = G->nx, ny = G->ny;
    if (nx < 1 || ny < 1 || !(dt > 0.0)) return -1;
    pad_t Q[4] = {pad_new(nx, ny, 1), pad_new(nx, ny, 1), pad_new(nx, ny, 1), pad_new(nx, ny, 1)};
    pad_load(&Q[0], h);
    pad_load(&Q[1], hu);
    pad_load(&Q[2], hv);
    pad_load(&Q[3], B);
    fill_ghosts(Q, 4, G->bc, 1, 2);

    /* per-cell data on the padded grid */
    size_t npad = (size_t)Q[0].px * Q[0].py;
    double *uu = (double *)calloc(npad, sizeof(double));
    double *vv = (double *)calloc(npad, sizeof(double));
    double *sq = (double *)calloc(npad, sizeof(double));
    unsigned char *wp = (unsigned char *)calloc(npad, 1);
    for (int j = -2; j < ny + 2; j++)
        for (int i = -2; i < nx + 2; i++) {
            size_t k = (size_t)(j + 2) * Q[0].px + (i + 2);
            double hh = *PA(&Q[0], i, j);
            wp[k] = hh > P->dry_tol;
            if (wp[k]) {
                sq[k] = sqrt(hh);
                uu[k] = *PA(&Q[1], i, j) / hh;
                vv[k] = *PA(&Q[2], i, j) / hh;
            }
        }
#define CELL_X(i, j, C) do { size_t kk = (size_t)((j) + 2) * Q[0].px + ((i) + 2); \
        (C).h = *PA(&Q[0], i, j); (C).hn = *PA(&Q[1], i, j); (C).ht = *PA(&Q[2], i, j); \
        (C).B = *PA(&Q[3], i, j); (C).un = uu[kk]; (C).vt = vv[kk]; (C).sq = sq[kk]; (C).wet = wp[kk]; } while (0)
#define CELL_Y(i, j, C) do { size_t kk = (size_t)((j) + 2) * Q[0].px + ((i) + 2); \
        (C).h = *PA(&Q[0], i, j); (C).hn = *PA(&Q[2], i, j); (C).ht = *PA(&Q[1], i, j); \
        (C).B = *PA(&Q[3], i, j); (C).un = vv[kk]; (C).vt = uu[kk]; (C).sq = sq[kk]; (C).wet = wp[kk]; } while (0)

    edges2d_t E = edges_new(nx, ny);
#pragma omp parallel for schedule(static)
    for (int j = -1; j <= ny; j++)
        for (int i = -1; i <= nx + 1; i++) {
            nlcell_t L, R;
            CELL_X(i - 1, j, L);
            CELL_X(i, j, R);
            edge_t *e = XE(&E, i, j);
            nl_solve(&L, &R, P->g, e);
            double am[3], ap[3];
            fluctuations_normal(e, am, ap);
            if (e->type == E_WALL_LO) ap[0] = ap[1] = ap[2] = 0.0;
            if (e->type == E_WALL_HI) am[0] = am[1] = am[2] = 0.0;
            to_phys(0, am, e->amdq);
            to_phys(0, ap, e->apdq);
        }
#pragma omp parallel for schedule(static)
    for (int j = -1; j <= ny + 1; j++)
        for (int i = -1; i <= nx; i++) {
            nlcell_t L, R;
            CELL_Y(i, j - 1, L);
            CELL_Y(i, j, R);
            edge_t *e = YE(&E, i, j);
            nl_solve(&L, &R, P->g, e);
            double am[3], ap[3];
            fluctuations_normal(e, am, ap);
            if (e->type == E_WALL_LO) ap[0] = ap[1] = ap[2] = 0.0;
            if (e->type == E_WALL_HI) am[0] = am[1] = am[2] = 0.0;
            to_phys(1, am, e->amdq);
            to_phys(1, ap, e->apdq);
        }
#undef CELL_X
#undef CELL_Y

    double nux = dt / G->dx, nuy = dt / G->dy;
    unsigned char *wet = (unsigned char *)calloc((size_t)nx * ny, 1);
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) wet[(size_t)j * nx + i] = h[(size_t)j * nx + i] > P->dry_tol;
    double *out[3] = {ho, huo, hvo};
    update2d(&E, Q, 3, wet, nux, nuy, P->order, P->transverse, 1, nl_split_cb, out);

    /* dry-cell fix: momenta vanish where the depth is not above the dry
     * tolerance; a negative depth is clamped to zero and counted */
    int ncl = 0;
    for (size_t k = 0; k < (size_t)nx * ny; k++) {
        if (!(ho[k] > P->dry_tol)) {
            huo[k] = 0.0;
            hvo[k] = 0.0;
        }
        if (ho[k] < 0.0) {
            ho[k] = 0.0;
            ncl++;
        }
    }
    /* Courant number: the edges' wave speeds, and each wet interior cell's
     * own speeds |u| + sqrt(g) sqrt(h), |v| + sqrt(g) sqrt(h).  The cell
     * speeds matter where a thin layer moves fast next to a wall or a much
     * deeper neighbour: the Roe averages of its edges hide its velocity. */
    if (cfl_out) {
        double cfl = cfl2d(&E, nux, nuy);
        const double sg = sqrt(P->g);
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                size_t k = (size_t)(j + 2) * Q[0].px + (i + 2);
                if (!wp[k]) continue;
                const double c = sg * sq[k];
                cfl = MAXD(cfl, nux * (fabs(uu[k]) + c));
                cfl = MAXD(cfl, nuy * (fabs(vv[k]) + c));
            }
        *cfl_out = cfl;
    }
    if (n_clamped) *n_clamped = ncl;

    edges_free(&E);
    free(wet); free(uu); free(vv); free(sq); free(wp);
    for (int c = 0; c < 4; c++) pad_free(&Q[c]);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* linearized equations about the sea at rest: static coefficients          */
/* ------------------------------------------------------------------------ */
/* hbar = max(0, sea_level - B); a cell is wet iff hbar > dry_tol;
 * c = sqrt(g hbar), gh = g hbar. */
typedef struct { double c, gh; int wet; } lincoef_t;

static void lin_coefs(const pad_t *Bp, const or_params *P, lincoef_t *out)
{
    int nrows = Bp->py;
    for (int jj = 0; jj < nrows; jj++)
        for (int ii = 0; ii < Bp->px; ii++) {
            double b = Bp->v[(size_t)jj * Bp->px + ii];
            double hb = MAXD(0.0, P->sea_level - b);
            lincoef_t *o = &out[(size_t)jj * Bp->px + ii];
            o->wet = hb > P->dry_tol;
            o->gh = P->g * hb;
            o->c = sqrt(o->gh);
        }
}

/*
 * Linear forward, 1D, wave form (LeVeque 2002, acoustics with variable
 * coefficients): q = (eta, mu), A = [[0, 1], [g hbar, 0]].
 *   alpha1 = (cR deta - dmu)/(cL + cR), alpha2 = (cL deta + dmu)/(cL + cR)
 *   W1 = alpha1 (1, -cL) with s1 = -cL,  W2 = alpha2 (1, cR) with s2 = cR
 *   A-dQ = s1 W1,  A+dQ = s2 W2
 * Wet/dry and walls as in the nonlinear solver (mirror (eta, -mu)).
 */
static void lin_solve(double eL, double mL, const lincoef_t *cl,
                      double eR, double mR, const lincoef_t *cr, edge_t *e)
{
    memset(e, 0, sizeof(*e));
    e->nw = 2;
    double cL = cl->c, cR = cr->c;
    if (!cl->wet && !cr->wet) { e->type = E_DRY; return; }
    if (cl->wet && !cr->wet) { e->type = E_WALL_LO; eR = eL; mR = -mL; cR = cL; }
    else if (!cl->wet && cr->wet) { e->type = E_WALL_HI; eL = eR; mL = -mR; cL = cR; }
    else e->type = E_WET;
    double deta = eR - eL, dmu = mR - mL;
    double rc = 1.0 / (cL + cR);
    double a1 = (cR * deta - dmu) * rc;
    double a2 = (cL * deta + dmu) * rc;
    e->s[0] = -cL; e->s[1] = cR;
    e->Z[0][0] = a1; e->Z[0][1] = a1 * (-cL); e->Z[0][2] = 0.0;
    e->Z[1][0] = a2; e->Z[1][1] = a2 * cR;    e->Z[1][2] = 0.0;
    e->cl = cL; e->cr = cR; e->rc = rc;
    for (int c = 0; c < 3; c++) {
        e->amdq[c] = e->s[0] * e->Z[0][c];
        e->apdq[c] = e->s[1] * e->Z[1][c];
    }
    if (e->type == E_WALL_LO) e->apdq[0] = e->apdq[1] = e->apdq[2] = 0.0;
    if (e->type == E_WALL_HI) e->amdq[0] = e->amdq[1] = e->amdq[2] = 0.0;
}

/*
 * Adjoint, time-reversed: q~_t + F(q~)_x = 0 with F = -A^T q~
 * = -(g hbar mu~, eta~, 0) along x (and -(g hbar gamma~, 0, eta~) along y),
 * solved in f-wave form with the eigenvectors of -A^T:
 *   d1 = ghL muL - ghR muR,  d2 = etaL - etaR          (flux jump)
 *   beta1 = (d1 + cR d2)/(cL + cR), beta2 = (cL d2 - d1)/(cL + cR)
 *   Z1 = beta1 (cL, 1, 0) at speed -cL (A-dQ), Z2 = beta2 (-cR, 1, 0) at +cR (A+dQ)
 * Normal frame (eta, normal component, tangential component).  Walls at
 * wet/dry interfaces and domain edges mirror (eta, -mu_n, mu_t): zero normal
 * adjoint velocity (Sec. 5).
 */
static void adj_solve(double eL, double nL, double tL, const lincoef_t *cl,
                      double eR, double nR, double tR, const lincoef_t *cr, edge_t *e)
{
    (void)tL; (void)tR;
    memset(e, 0, sizeof(*e));
    e->nw = 2;
    double cL = cl->c, cR = cr->c, ghL = cl->gh, ghR = cr->gh;
    if (!cl->wet && !cr->wet) { e->type = E_DRY; return; }
    if (cl->wet && !cr->wet) { e->type = E_WALL_LO; eR = eL; nR = -nL; cR = cL; ghR = ghL; }
    else if (!cl->wet && cr->wet) { e->type = E_WALL_HI; eL = eR; nL = -nR; cL = cR; ghL = ghR; }
    else e->type = E_WET;
    double d1 = ghL * nL - ghR * nR;
    double d2 = eL - eR;
    double rc = 1.0 / (cL + cR);
    double b1 = (d1 + cR * d2) * rc;
    double b2 = (cL * d2 - d1) * rc;
    e->s[0] = -cL; e->s[1] = cR;
    e->Z[0][0] = b1 * cL;    e->Z[0][1] = b1; e->Z[0][2] = 0.0;
    e->Z[1][0] = b2 * (-cR); e->Z[1][1] = b2; e->Z[1][2] = 0.0;
    e->cl = cL; e->cr = cR; e->rc = rc;
}

/*
 * Split a physical adjoint fluctuation a on a wet-wet edge (normal frame),
 * variable-coefficient eigenvectors of the two cells: (cL, 1, 0) at -cL from
 * the low cell and (-cR, 1, 0) at +cR from the high cell:
 *   gl = (a_e + cR a_n)/(cL + cR), gr = (cL a_n - a_e)/(cL + cR)
 *   positive part = (cR gr) (-cR, 1, 0),  negative part = (-cL gl) (cL, 1, 0)
 */
static void adj_split(const edge_t *e, int ydir, const double *a_ph, int positive, double *out_ph)
{
    double a[3];
    to_normal(ydir, a_ph, a);
    double nf[3];
    if (positive) {
        double gr = (e->cl * a[1] - a[0]) * e->rc;
        double k = e->cr * gr;
        nf[0] = k * (-e->cr); nf[1] = k; nf[2] = 0.0;
    } else {
        double gl = (a[0] + e->cr * a[1]) * e->rc;
        double k = (-e->cl) * gl;
        nf[0] = k * e->cl; nf[1] = k; nf[2] = 0.0;
    }
    to_phys(ydir, nf, out_ph);
}

/*
 * Test hook (the pins only): the positive and negative parts of the adjoint
 * transverse split of the physical fluctuation a on a wet-wet edge whose
 * cells have sound speeds cL (low) and cR (high).
 */
void or_adj_split_parts(double cL, double cR, int ydir, const double *a, double *pos, double *neg)
{
    edge_t e;
    memset(&e, 0, sizeof e);
    e.type = E_WET;
    e.nw = 2;
    e.cl = cL;
    e.cr = cR;
    e.rc = 1.0 / (cL + cR);
    adj_split(&e, ydir, a, 1, pos);
    adj_split(&e, ydir, a, 0, neg);
}

/* ------------------------------------------------------------------------ */
/* 1D sweep (linear forward and adjoint)                                    */
/* ------------------------------------------------------------------------ */
static int step1d(const or_grid *G, const or_params *P, const double *B,
                  const double *q0, const double *q1, double *o0, double *o1,
                  double dt, double *cfl_out, int adjoint)
{
    int nx = G->nx;
    pad_t Q[3] = {pad_new(nx, 1, 0), pad_new(nx, 1, 0), pad_new(nx, 1, 0)};
    pad_load(&Q[0], q0);
    pad_load(&Q[1], q1);
    pad_load(&Q[2], B);
    fill_ghosts(Q, 3, G->bc, 1, -1);
    lincoef_t *cf = (lincoef_t *)calloc((size_t)Q[0].px, sizeof(lincoef_t));
    lin_coefs(&Q[2], P, cf);
    /* edges i-1/2 for i in [-1, nx+1] */
    edge_t *E = (edge_t *)calloc((size_t)nx + 3, sizeof(edge_t));
    for (int i = -1; i <= nx + 1; i++) {
        edge_t *e = &E[i + 1];
        const lincoef_t *cl = &cf[i - 1 + 2], *cr = &cf[i + 2];
        double eL = *PA(&Q[0], i - 1, 0), mL = *PA(&Q[1], i - 1, 0);
        double eR = *PA(&Q[0], i, 0), mR = *PA(&Q[1], i, 0);
        if (adjoint) {
            adj_solve(eL, mL, 0.0, cl, eR, mR, 0.0, cr, e);
            double am[3], ap[3];
            fluctuations_normal(e, am, ap);
            if (e->type == E_WALL_LO) ap[0] = ap[1] = ap[2] = 0.0;
            if (e->type == E_WALL_HI) am[0] = am[1] = am[2] = 0.0;
            memcpy(e->amdq, am, sizeof am);
            memcpy(e->apdq, ap, sizeof ap);
        } else {
            lin_solve(eL, mL, cl, eR, mR, cr, e);
        }
    }
    double nu = dt / G->dx;
    double cfl = 0.0;
    for (int i = 0; i <= nx; i++) {
        const edge_t *e = &E[i + 1];
        for (int p = 0; p < e->nw; p++) cfl = MAXD(cfl, nu * fabs(e->s[p]));
    }
    double *F = (double *)calloc((size_t)3 * (nx + 1), sizeof(double));
    for (int i = 0; i <= nx; i++) {
        const edge_t *e = &E[i + 1];
        if (e->type != E_WET || P->order != 2) continue;
        correction(e, &E[i], &E[i + 2], nu, adjoint ? 1 : 0, &F[3 * i]);
    }
    double *out[2] = {o0, o1};
    for (int i = 0; i < nx; i++) {
        for (int c = 0; c < 2; c++) {
            double q = *PA(&Q[c], i, 0);
            if (cf[i + 2].wet) {
                q = q - nu * (E[i + 1].apdq[c] + E[i + 2].amdq[c]);
                q = q - nu * (F[3 * (i + 1) + c] - F[3 * i + c]);
            }
            out[c][i] = q;
        }
    }
    if (cfl_out) *cfl_out = cfl;
    free(F); free(E); free(cf);
    for (int c = 0; c < 3; c++) pad_free(&Q[c]);
    return 0;
}

int or_lin_step(const or_grid *G, const or_params *P, const double *B,
                const double *q0, const double *q1, double *o0, double *o1,
                double dt, double *cfl_out)
{
    if (G->ny != 1 || G->nx < 1 || !(dt > 0.0)) return -1;
    return step1d(G, P, B, q0, q1, o0, o1, dt, cfl_out, 0);
}

/*
 * Linear forward, 2D (the 2D equations of Sec. 5 linearized about the sea at
 * rest): q = (eta, mu, gamma), A1 = [[0,1,0],[g hbar,0,0],[0,0,0]] and A2 the
 * same with the roles of mu and gamma exchanged.  Each edge is solved in its
 * normal frame (eta, normal, tangential) with the two acoustic waves of
 * lin_solve; the jump in the tangential momentum is a wave of speed 0, which
 * carries no fluctuation and no correction.
 * Transverse split of a physical fluctuation a on the edge that receives it,
 * with the variable-coefficient eigenvectors of the edge's two cells,
 * (1, -cL) at -cL from the low cell and (1, cR) at +cR from the high cell:
 *   a = b1 (1, -cL) + b2 (1, cR):  b1 = (cR a_e - a_n)/(cL + cR),
 *                                  b2 = (cL a_e + a_n)/(cL + cR)
 *   positive part = cR b2 (1, cR, 0),  negative part = -cL b1 (1, -cL, 0)
 * (each part is speed times wave, the wave form of the normal solve).
 */
static void lin2_split(const edge_t *e, int ydir, const double *a_ph, int positive, double *out_ph)
{
    double a[3];
    to_normal(ydir, a_ph, a);
    double nf[3];
    if (positive) {
        double b2 = (e->cl * a[0] + a[1]) * e->rc;
        double k = e->cr * b2;
        nf[0] = k; nf[1] = k * e->cr; nf[2] = 0.0;
    } else {
        double b1 = (e->cr * a[0] - a[1]) * e->rc;
        double k = (-e->cl) * b1;
        nf[0] = k; nf[1] = k * (-e->cl); nf[2] = 0.0;
    }
    to_phys(ydir, nf, out_ph);
}

static void lin2_split_cb(const edge_t *e, int ydir, const double *a, int positive, double *out)
{
    lin2_split(e, ydir, a, positive, out);
}

int or_lin_step2d(const or_grid *G, const or_params *P, const double *B,
                  const double *q0, const double *q1, const double *q2,
                  double *o0, double *o1, double *o2, double dt, double *cfl_out)
{
    int nx = G->nx, ny = G->ny;
    if (nx < 1 || ny < 2 || !(dt > 0.0)) return -1;
    pad_t Q[4] = {pad_new(nx, ny, 1), pad_new(nx, ny, 1), pad_new(nx, ny, 1), pad_new(nx, ny, 1)};
    pad_load(&Q[0], q0);
    pad_load(&Q[1], q1);
    pad_load(&Q[2], q2);
    pad_load(&Q[3], B);
    fill_ghosts(Q, 4, G->bc, 1, 2);
    size_t npad = (size_t)Q[0].px * Q[0].py;
    lincoef_t *cf = (lincoef_t *)calloc(npad, sizeof(lincoef_t));
    lin_coefs(&Q[3], P, cf);
#define CF(i, j) (&cf[(size_t)((j) + 2) * Q[0].px + ((i) + 2)])
    edges2d_t E = edges_new(nx, ny);
#pragma omp parallel for schedule(static)
    for (int j = -1; j <= ny; j++)
        for (int i = -1; i <= nx + 1; i++) {
            edge_t *e = XE(&E, i, j);
            lin_solve(*PA(&Q[0], i - 1, j), *PA(&Q[1], i - 1, j), CF(i - 1, j),
                      *PA(&Q[0], i, j), *PA(&Q[1], i, j), CF(i, j), e);
            double am[3], ap[3];
            memcpy(am, e->amdq, sizeof am);
            memcpy(ap, e->apdq, sizeof ap);
            to_phys(0, am, e->amdq);
            to_phys(0, ap, e->apdq);
        }
#pragma omp parallel for schedule(static)
    for (int j = -1; j <= ny + 1; j++)
        for (int i = -1; i <= nx; i++) {
            edge_t *e = YE(&E, i, j);
            lin_solve(*PA(&Q[0], i, j - 1), *PA(&Q[2], i, j - 1), CF(i, j - 1),
                      *PA(&Q[0], i, j), *PA(&Q[2], i, j), CF(i, j), e);
            double am[3], ap[3];
            memcpy(am, e->amdq, sizeof am);
            memcpy(ap, e->apdq, sizeof ap);
            to_phys(1, am, e->amdq);
            to_phys(1, ap, e->apdq);
        }
    double nux = dt / G->dx, nuy = dt / G->dy;
    unsigned char *wet = (unsigned char *)calloc((size_t)nx * ny, 1);
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) wet[(size_t)j * nx + i] = CF(i, j)->wet;
#undef CF
    double *out[3] = {o0, o1, o2};
    update2d(&E, Q, 3, wet, nux, nuy, P->order, P->transverse, 0, lin2_split_cb, out);
    if (cfl_out) *cfl_out = cfl2d(&E, nux, nuy);
    edges_free(&E);
    free(wet);
    free(cf);
    for (int c = 0; c < 4; c++) pad_free(&Q[c]);
    return 0;
}

static void adj_split_cb(const edge_t *e, int ydir, const double *a, int positive, double *out)
{
    adj_split(e, ydir, a, positive, out);
}

int or_adj_step(const or_grid *G, const or_params *P, const double *B,
                const double *q0, const double *q1, const double *q2,
                double *o0, double *o1, double *o2, double dt, double *cfl_out)
{
    int nx = G->nx, ny = G->ny;
    if (nx < 1 || ny < 1 || !(dt > 0.0)) return -1;
    if (ny == 1) return step1d(G, P, B, q0, q1, o0, o1, dt, cfl_out, 1);

    pad_t Q[4] = {pad_new(nx, ny, 1), pad_new(nx, ny, 1), pad_new(nx, ny, 1), pad_new(nx, ny, 1)};
    pad_load(&Q[0], q0);
    pad_load(&Q[1], q1);
    pad_load(&Q[2], q2);
    pad_load(&Q[3], B);
    fill_ghosts(Q, 4, G->bc, 1, 2);
    size_t npad = (size_t)Q[0].px * Q[0].py;
    lincoef_t *cf = (lincoef_t *)calloc(npad, sizeof(lincoef_t));
    lin_coefs(&Q[3], P, cf);
#define CF(i, j) (&cf[(size_t)((j) + 2) * Q[0].px + ((i) + 2)])

    edges2d_t E = edges_new(nx, ny);
#pragma omp parallel for schedule(static)
    for (int j = -1; j <= ny; j++)
        for (int i = -1; i <= nx + 1; i++) {
            edge_t *e = XE(&E, i, j);
            adj_solve(*PA(&Q[0], i - 1, j), *PA(&Q[1], i - 1, j), *PA(&Q[2], i - 1, j), CF(i - 1, j),
                      *PA(&Q[0], i, j), *PA(&Q[1], i, j), *PA(&Q[2], i, j), CF(i, j), e);
            double am[3], ap[3];
            fluctuations_normal(e, am, ap);
            if (e->type == E_WALL_LO) ap[0] = ap[1] = ap[2] = 0.0;
            if (e->type == E_WALL_HI) am[0] = am[1] = am[2] = 0.0;
            to_phys(0, am, e->amdq);
            to_phys(0, ap, e->apdq);
        }
#pragma omp parallel for schedule(static)
    for (int j = -1; j <= ny + 1; j++)
        for (int i = -1; i <= nx; i++) {
            edge_t *e = YE(&E, i, j);
            adj_solve(*PA(&Q[0], i, j - 1), *PA(&Q[2], i, j - 1), *PA(&Q[1], i, j - 1), CF(i, j - 1),
                      *PA(&Q[0], i, j), *PA(&Q[2], i, j), *PA(&Q[1], i, j), CF(i, j), e);
            double am[3], ap[3];
            fluctuations_normal(e, am, ap);
            if (e->type == E_WALL_LO) ap[0] = ap[1] = ap[2] = 0.0;
            if (e->type == E_WALL_HI) am[0] = am[1] = am[2] = 0.0;
            to_phys(1, am, e->amdq);
            to_phys(1, ap, e->apdq);
        }
    double nux = dt / G->dx, nuy = dt / G->dy;
    unsigned char *wet = (unsigned char *)calloc((size_t)nx * ny, 1);
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) wet[(size_t)j * nx + i] = CF(i, j)->wet;
#undef CF
    double *out[3] = {o0, o1, o2};
    update2d(&E, Q, 3, wet, nux, nuy, P->order, P->transverse, 1, adj_split_cb, out);
    if (cfl_out) *cfl_out = cfl2d(&E, nux, nuy);
    edges_free(&E);
    free(wet); free(cf);
    for (int c = 0; c < 4; c++) pad_free(&Q[c]);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* target functional, initial states, time steps                            */
/* ------------------------------------------------------------------------ */
/*
 * phi = (I, 0, 0) (eqs. (phi_1d), (phi_Alaska)); I is a Gaussian
 * exp(-r^2/R^2) (shape 0) or the disk indicator r <= R (shape 1), with r the
 * distance of the cell centre from (xc, yc) (1D: |x - xc|).  I = 0 in cells
 * that are dry for the adjoint (hbar <= dry_tol).
 */
void or_target(const or_grid *G, const or_params *P, const double *B,
               double xc, double yc, double R, int shape, double *phi)
{
    int ny = G->ny;
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < G->nx; i++) {
            size_t k = (size_t)j * G->nx + i;
            double x = G->x_lo + (i + 0.5) * G->dx;
            double ddx = x - xc;
            double r2 = ddx * ddx;
            if (ny > 1) {
                double y = G->y_lo + (j + 0.5) * G->dy;
                double ddy = y - yc;
                r2 = r2 + ddy * ddy;
            }
            double v = (shape == 0) ? exp(-r2 / (R * R)) : ((r2 <= R * R) ? 1.0 : 0.0);
            double hb = MAXD(0.0, P->sea_level - B[k]);
            phi[k] = (hb > P->dry_tol) ? v : 0.0;
        }
}

/* Nonlinear initial state h = max(0, eta0 - B), zero momenta.  Linear:
 * eta = eta0 where wet (hbar > dry_tol), 0 elsewhere, zero momenta. */
void or_init_state(const or_grid *G, const or_params *P, int model, const double *B,
                   const double *eta0, double *q0, double *q1, double *q2)
{
    size_t n = (size_t)G->nx * G->ny;
    for (size_t k = 0; k < n; k++) {
        if (model == OR_NONLINEAR) {
            q0[k] = MAXD(0.0, eta0[k] - B[k]);
        } else {
            double hb = MAXD(0.0, P->sea_level - B[k]);
            q0[k] = (hb > P->dry_tol) ? eta0[k] : 0.0;
        }
        q1[k] = 0.0;
        if (q2) q2[k] = 0.0;
    }
}

/*
 * Initial forward time step: cfl_desired / max over wet cells of the largest
 * characteristic speed over the cell size,
 *   nonlinear: max((|u| + sqrt(g h))/dx, (|v| + sqrt(g h))/dy)
 *   linear:    sqrt(g hbar)/dx (and /dy in 2D)
 * Returns 0 if no cell is wet.
 */
double or_dt0(const or_grid *G, const or_params *P, int model, const double *B,
              const double *q0, const double *q1, const double *q2)
{
    size_t n = (size_t)G->nx * G->ny;
    double m = 0.0;
    for (size_t k = 0; k < n; k++) {
        double a, b;
        if (model == OR_NONLINEAR) {
            double h = q0[k];
            if (!(h > P->dry_tol)) continue;
            double c = sqrt(P->g * h);
            a = (fabs(q1[k] / h) + c) / G->dx;
            b = (G->ny > 1) ? (fabs(q2[k] / h) + c) / G->dy : 0.0;
        } else {
            double hb = MAXD(0.0, P->sea_level - B[k]);
            if (!(hb > P->dry_tol)) continue;
            double c = sqrt(P->g * hb);
            a = c / G->dx;
            b = (G->ny > 1) ? c / G->dy : 0.0;
        }
        m = MAXD(m, MAXD(a, b));
    }
    return (m > 0.0) ? P->cfl_desired / m : 0.0;
}

/*
 * Adjoint sub-stepping between snapshots: ds = (tf - t0)/K, the largest
 * stable step dt_cfl = cfl_desired / max(cmax/dx, cmax/dy) (cmax over wet
 * cells), n_sub = ceil(ds/dt_cfl), dt = ds/n_sub (constant).
 */
int or_adj_nsub(const or_grid *G, const or_params *P, const double *B,
                double t0, double tf, int K, double *dt_out)
{
    size_t n = (size_t)G->nx * G->ny;
    double cmax = 0.0;
    for (size_t k = 0; k < n; k++) {
        double hb = MAXD(0.0, P->sea_level - B[k]);
        if (hb > P->dry_tol) cmax = MAXD(cmax, sqrt(P->g * hb));
    }
    double ds = (tf - t0) / K;
    if (!(cmax > 0.0) || !(ds > 0.0)) return -1;
    double sx = cmax / G->dx;
    double sy = (G->ny > 1) ? cmax / G->dy : 0.0;
    double dt_cfl = P->cfl_desired / MAXD(sx, sy);
    int nsub = (int)ceil(ds / dt_cfl);
    if (nsub < 1) nsub = 1;
    if (dt_out) *dt_out = ds / nsub;
    return nsub;
}

/* ------------------------------------------------------------------------ */
/* window and flags                                                         */
/* ------------------------------------------------------------------------ */
static double snap(double r)
{
    double rr = nearbyint(r);
    return (fabs(r - rr) <= 1e-9) ? rr : r;
}

/*
 * Snapshot window for forward time t (eq. (ip_timerange), Sec. 4.2): the
 * adjoint of data at time that(in [ts, tf]) is the tf-data adjoint shifted by
 * tf - that, so tau ranges over [t, T] with T = min(t + tf - ts, tf).  In
 * reversed adjoint time s = tf - tau this is [tf - T, tf - t]; frame k sits at
 * s = k ds with ds = (tf - t0)/K.  The frames bracketing that range outward
 * (as the two-snapshot rule of eq. (ip_timepoint) does for a single time) are
 *   k_lo = max(0, floor((tf - T)/ds)), k_hi = min(K, ceil((tf - t)/ds)),
 * a ratio within 1e-9 of an integer being taken as that integer.
 * Returns 0 and no window if t > tf.
 */
int or_window(double t, double t0, double ts, double tf, int K, int *k_lo, int *k_hi)
{
    double ds = (tf - t0) / K;
    double T = MIND(t + (tf - ts), tf);
    double sa = tf - T;
    double sb = tf - t;
    if (sb < 0.0) {
        *k_lo = 1;
        *k_hi = 0;
        return 0;
    }
    double ra = snap(sa / ds), rb = snap(sb / ds);
    int lo = (int)floor(ra), hi = (int)ceil(rb);
    if (lo < 0) lo = 0;
    if (hi > K) hi = K;
    *k_lo = lo;
    *k_hi = hi;
    return 1;
}

/*
 * Flags (Sec. 4.1, 4.2 and the wet/dry rule of Sec. 6): for each cell,
 *   m = max_{k in [k_lo, k_hi]} |(eta eta^_k + mu mu^_k) + gamma gamma^_k|
 * (1D: |eta eta^_k + mu mu^_k|), m = 0 if the cell is dry in the forward or in
 * the adjoint problem, and flag = (m > tol).  Forward eta = (h + B) - sea_level
 * for the nonlinear model, the first component for the linear model.
 * frames: (K+1) frames of ncomp (ny, nx) planes.
 * Accumulators (if non-null): flag_acc |= flag, maxip_acc = max(maxip_acc, m).
 */
void or_flag(const or_grid *G, const or_params *P, int model, const double *B,
             const double *q0, const double *q1, const double *q2,
             const double *frames, int K, int k_lo, int k_hi, double tol,
             signed char *flags, double *maxip, signed char *flag_acc, double *maxip_acc)
{
    (void)K;
    int twod = G->ny > 1;
    int ncomp = twod ? 3 : 2;
    size_t n = (size_t)G->nx * G->ny;
#pragma omp parallel for schedule(static)
    for (size_t k = 0; k < n; k++) {
        double hb = MAXD(0.0, P->sea_level - B[k]);
        int adj_wet = hb > P->dry_tol;
        int fwd_wet = (model == OR_NONLINEAR) ? (q0[k] > P->dry_tol) : adj_wet;
        double m = 0.0;
        if (adj_wet && fwd_wet) {
            double eta = (model == OR_NONLINEAR) ? (q0[k] + B[k]) - P->sea_level : q0[k];
            for (int f = k_lo; f <= k_hi; f++) {
                const double *fr = frames + (size_t)f * ncomp * n;
                double ip = eta * fr[k] + q1[k] * fr[n + k];
                if (twod) ip = ip + q2[k] * fr[2 * n + k];
                m = MAXD(m, fabs(ip));
            }
        }
        signed char fl = (m > tol) ? 1 : 0;
        if (flags) flags[k] = fl;
        if (maxip) maxip[k] = m;
        if (flag_acc) flag_acc[k] = (signed char)(flag_acc[k] | fl);
        if (maxip_acc) maxip_acc[k] = MAXD(maxip_acc[k], m);
    }
}

/*
 * Adjoint values at the forward grid's cell centres when the adjoint was
 * solved on a grid of its own (Sec. 4: linear, in 2D bilinear, interpolation
 * from the data on the snapshot grid).  On each axis, for a point x and an
 * adjoint axis of n centres x_lo + (c + 1/2) d:
 *   u = (x - x_lo)/d;  containing cell ic = clamp(floor(u), 0, n-1);
 *   i0 = clamp(floor(u - 1/2), 0, n-2) (0 if n = 1);
 *   w = clamp(u - 1/2 - i0, 0, 1) (0 if n = 1): constant beyond the outer centres.
 */
static void interp_axis(double x, double x_lo, double d, int n, int *i0, double *w, int *ic)
{
    double u = (x - x_lo) / d;
    double c = floor(u);
    if (c < 0.0) c = 0.0;
    if (c > n - 1) c = n - 1;
    *ic = (int)c;
    double xi = u - 0.5;
    double f = floor(xi);
    double top = (n >= 2) ? (double)(n - 2) : 0.0;
    if (f < 0.0) f = 0.0;
    if (f > top) f = top;
    *i0 = (int)f;
    double ww = (n >= 2) ? xi - f : 0.0;
    if (ww < 0.0) ww = 0.0;
    if (ww > 1.0) ww = 1.0;
    *w = ww;
}

/* value of the adjoint-grid plane v at the centre of forward cell (i, j):
 * (1-wy)((1-wx) v00 + wx v10) + wy((1-wx) v01 + wx v11), 1D: (1-wx) v0 + wx v1 */
static double interp_at(const or_grid *G, const or_grid *Ga, const double *v, int i, int j)
{
    int i0, ic, j0 = 0, jc = 0;
    double wx, wy = 0.0;
    double x = G->x_lo + (i + 0.5) * G->dx;
    interp_axis(x, Ga->x_lo, Ga->dx, Ga->nx, &i0, &wx, &ic);
    int i1 = (Ga->nx >= 2) ? i0 + 1 : i0;
    if (G->ny > 1) {
        double y = G->y_lo + (j + 0.5) * G->dy;
        interp_axis(y, Ga->y_lo, Ga->dy, Ga->ny, &j0, &wy, &jc);
        int j1 = (Ga->ny >= 2) ? j0 + 1 : j0;
        double v00 = v[(size_t)j0 * Ga->nx + i0], v10 = v[(size_t)j0 * Ga->nx + i1];
        double v01 = v[(size_t)j1 * Ga->nx + i0], v11 = v[(size_t)j1 * Ga->nx + i1];
        return (1.0 - wy) * ((1.0 - wx) * v00 + wx * v10) + wy * ((1.0 - wx) * v01 + wx * v11);
    }
    return (1.0 - wx) * v[i0] + wx * v[i1];
}

void or_interp(const or_grid *G, const or_grid *Ga, const double *v, double *out)
{
    for (int j = 0; j < G->ny; j++)
        for (int i = 0; i < G->nx; i++) out[(size_t)j * G->nx + i] = interp_at(G, Ga, v, i, j);
}

/*
 * or_flag with the snapshots on the adjoint grid Ga (bottom Ba): the inner
 * product uses the interpolated snapshot values; the cell is adjoint-wet iff
 * the adjoint cell containing its centre is wet (Sec. 6: wet in the forward
 * and dry in the adjoint problem gives 0).
 */
void or_flag_interp(const or_grid *G, const or_params *P, int model, const double *B,
                    const double *q0, const double *q1, const double *q2,
                    const or_grid *Ga, const double *Ba, const double *frames, int K, int k_lo, int k_hi,
                    double tol, signed char *flags, double *maxip, signed char *flag_acc, double *maxip_acc)
{
    (void)K;
    int twod = G->ny > 1;
    int ncomp = twod ? 3 : 2;
    size_t na = (size_t)Ga->nx * Ga->ny;
#pragma omp parallel for schedule(static)
    for (int j = 0; j < G->ny; j++) {
        for (int i = 0; i < G->nx; i++) {
            size_t k = (size_t)j * G->nx + i;
            int fwd_wet = (model == OR_NONLINEAR) ? (q0[k] > P->dry_tol)
                                                  : (MAXD(0.0, P->sea_level - B[k]) > P->dry_tol);
            int i0, ic, jc = 0, j0 = 0;
            double w;
            interp_axis(G->x_lo + (i + 0.5) * G->dx, Ga->x_lo, Ga->dx, Ga->nx, &i0, &w, &ic);
            if (twod) interp_axis(G->y_lo + (j + 0.5) * G->dy, Ga->y_lo, Ga->dy, Ga->ny, &j0, &w, &jc);
            int adj_wet = MAXD(0.0, P->sea_level - Ba[(size_t)jc * Ga->nx + ic]) > P->dry_tol;
            double m = 0.0;
            if (adj_wet && fwd_wet) {
                double eta = (model == OR_NONLINEAR) ? (q0[k] + B[k]) - P->sea_level : q0[k];
                for (int f = k_lo; f <= k_hi; f++) {
                    const double *fr = frames + (size_t)f * ncomp * na;
                    double ip = eta * interp_at(G, Ga, fr, i, j) + q1[k] * interp_at(G, Ga, fr + na, i, j);
                    if (twod) ip = ip + q2[k] * interp_at(G, Ga, fr + 2 * na, i, j);
                    m = MAXD(m, fabs(ip));
                }
            }
            signed char fl = (m > tol) ? 1 : 0;
            if (flags) flags[k] = fl;
            if (maxip) maxip[k] = m;
            if (flag_acc) flag_acc[k] = (signed char)(flag_acc[k] | fl);
            if (maxip_acc) maxip_acc[k] = MAXD(maxip_acc[k], m);
        }
    }
}

/*
 * Surface flagging, the default refinement criterion the adjoint method is
 * compared with (Sec. 6): a cell is flagged when the sea surface relative to
 * sea level exceeds the tolerance, read here as |eta| > tol (a trough counts
 * as a wave as much as a crest), in cells that are wet.  eta = (h + B) -
 * sea_level, wet = h > dry_tol (nonlinear); eta = first component, wet =
 * adjoint-wet (linear).  flag_acc (if non-null) |= flag.
 */
void or_surface_flag(const or_grid *G, const or_params *P, int model, const double *B,
                     const double *q0, double tol, signed char *flags, signed char *flag_acc)
{
    size_t n = (size_t)G->nx * G->ny;
    for (size_t k = 0; k < n; k++) {
        int wet;
        double eta;
        if (model == OR_NONLINEAR) {
            wet = q0[k] > P->dry_tol;
            eta = (q0[k] + B[k]) - P->sea_level;
        } else {
            wet = MAXD(0.0, P->sea_level - B[k]) > P->dry_tol;
            eta = q0[k];
        }
        signed char fl = (wet && fabs(eta) > tol) ? 1 : 0;
        if (flags) flags[k] = fl;
        if (flag_acc) flag_acc[k] = (signed char)(flag_acc[k] | fl);
    }
}

/* ------------------------------------------------------------------------ */
/* driver                                                                   */
/* ------------------------------------------------------------------------ */
/*
 * Two-phase run (Sec. 4):
 * A. adjoint: q~(0) = phi, advanced with constant dt = ds/n_sub; frame k
 *    (k = 0..K) is q~ at reversed time k ds, i.e. q^(tau = tf - k ds).
 * B. forward from t0 with the initial state of eta0: flag at t0 (and, if
 *    asked, surface-flag at t0 and at every output time), then repeat
 *      choose dt (initially dt0, then dt cfl_desired/cfl of the last accepted
 *      or rejected attempt, unchanged if cfl = 0), clamped to the next output
 *      time t0 + j ds (the last one is tf);
 *      step; if cfl > cfl_max discard and retry with dt cfl_desired/cfl;
 *      otherwise accept, and flag if an output time was reached (flags at
 *      output j are stored) or the number of accepted steps is a multiple of
 *      flag_every (every step for flag_every = 1, as in Sec. 4.1);
 *    until tf.
 */
int or_run(const or_problem *pb, or_result *res)
{
    const or_grid *G = &pb->grid;
    const or_params *P = &pb->params;
    int twod = G->ny > 1;
    int ncomp = twod ? 3 : 2;
    size_t n = (size_t)G->nx * G->ny;
    int K = pb->K;
    memset(res, 0, sizeof(*res));
    if (K < 1 || !(pb->tf > pb->t0) || pb->flag_every < 1) return -1;
    if (!twod && pb->model != OR_LINEAR) return -1;

    /* phase A, on the adjoint's own grid if one is given */
    int interp = pb->adj_grid.nx != 0;
    const or_grid *GA = interp ? &pb->adj_grid : G;
    const double *BA = interp ? pb->adj_B : pb->B;
    if (interp && ((GA->ny > 1) != twod || !BA)) return -1;
    size_t na = (size_t)GA->nx * GA->ny;
    size_t nmax = na > n ? na : n;
    double dt_adj = 0.0;
    int nsub = or_adj_nsub(GA, P, BA, pb->t0, pb->tf, K, &dt_adj);
    if (nsub < 1) return -1;
    double *a[3], *b[3];
    for (int c = 0; c < 3; c++) {
        a[c] = (double *)calloc(nmax, sizeof(double));
        b[c] = (double *)calloc(nmax, sizeof(double));
    }
    or_target(GA, P, BA, pb->target_xc, pb->target_yc, pb->target_R, pb->target_shape, a[0]);
    for (int c = 0; c < ncomp; c++) memcpy(pb->frames + (size_t)c * na, a[c], na * sizeof(double));
    for (int k = 1; k <= K; k++) {
        for (int s = 0; s < nsub; s++) {
            double cfl;
            or_adj_step(GA, P, BA, a[0], a[1], a[2], b[0], b[1], b[2], dt_adj, &cfl);
            for (int c = 0; c < 3; c++) { double *t = a[c]; a[c] = b[c]; b[c] = t; }
            res->n_adj_steps++;
        }
        for (int c = 0; c < ncomp; c++)
            memcpy(pb->frames + ((size_t)k * ncomp + c) * na, a[c], na * sizeof(double));
    }
    for (int c = 0; c < 3; c++) {
        memset(a[c], 0, nmax * sizeof(double));
        memset(b[c], 0, nmax * sizeof(double));
    }
    res->n_sub = nsub;
    res->dt_adj = dt_adj;

    /* phase B */
    or_init_state(G, P, pb->model, pb->B, pb->eta0, a[0], a[1], a[2]);
    double ds = (pb->tf - pb->t0) / K;
    double t = pb->t0;
    signed char *fl = (signed char *)calloc(n, 1);
    int klo, khi;
#define DO_FLAG(store_idx) do { \
        int ok = or_window(t, pb->t0, pb->ts, pb->tf, K, &klo, &khi); \
        if (!ok) { klo = 1; khi = 0; } \
        double *m_out = ((store_idx) >= 0 && pb->maxip_at) ? pb->maxip_at + (size_t)(store_idx) * n : NULL; \
        if (interp) \
            or_flag_interp(G, P, pb->model, pb->B, a[0], a[1], a[2], GA, BA, pb->frames, K, klo, khi, \
                           pb->tol, fl, m_out, pb->flag_acc, pb->maxip_acc); \
        else \
            or_flag(G, P, pb->model, pb->B, a[0], a[1], a[2], pb->frames, K, klo, khi, pb->tol, \
                    fl, m_out, pb->flag_acc, pb->maxip_acc); \
        if ((store_idx) >= 0 && pb->flags_at) memcpy(pb->flags_at + (size_t)(store_idx) * n, fl, n); \
        if ((store_idx) >= 0 && pb->surface_flags_at) \
            or_surface_flag(G, P, pb->model, pb->B, a[0], pb->surface_tol, \
                            pb->surface_flags_at + (size_t)(store_idx) * n, NULL); \
        res->n_flag_calls++; } while (0)

    DO_FLAG(0);
    double dt = or_dt0(G, P, pb->model, pb->B, a[0], a[1], a[2]);
    if (!(dt > 0.0)) { res->status = -1; goto done; }
    int j = 1;
    while (j <= K) {
        double tout = (j == K) ? pb->tf : pb->t0 + j * ds;
        int final = 0;
        if (dt >= tout - t) { dt = tout - t; final = 1; }
        double cfl = 0.0;
        int ncl = 0;
        if (pb->model == OR_NONLINEAR)
            or_swe_step(G, P, pb->B, a[0], a[1], a[2], b[0], b[1], b[2], dt, &cfl, &ncl);
        else if (twod)
            or_lin_step2d(G, P, pb->B, a[0], a[1], a[2], b[0], b[1], b[2], dt, &cfl);
        else
            or_lin_step(G, P, pb->B, a[0], a[1], b[0], b[1], dt, &cfl);
        if (cfl > P->cfl_max) {
            res->n_rejected++;
            dt = dt * P->cfl_desired / cfl;
            if (res->n_rejected > 1000) { res->status = -2; goto done; }
            continue;
        }
        for (int c = 0; c < 3; c++) { double *tp = a[c]; a[c] = b[c]; b[c] = tp; }
        res->n_clamped += ncl;
        res->n_fwd_steps++;
        t = final ? tout : t + dt;
        if (final) {
            DO_FLAG(j);
            j++;
        } else if (res->n_fwd_steps % pb->flag_every == 0) {
            DO_FLAG(-1);
        }
        if (cfl > 0.0) dt = dt * P->cfl_desired / cfl;
    }
#undef DO_FLAG
done:
    res->t_end = t;
    for (int c = 0; c < ncomp; c++) memcpy(pb->q_out[c], a[c], n * sizeof(double));
    free(fl);
    for (int c = 0; c < 3; c++) { free(a[c]); free(b[c]); }
    return res->status;
}

/* Threads of the row loops from now on (tiny grids run fastest on one);
 * a no-op without OpenMP.  Results never depend on it. */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
