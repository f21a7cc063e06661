/* Exercises the oracle's entry points on small grids under ASan/UBSan. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"
#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); return 1; } } while (0)
static unsigned s = 777u;
static double rnd(void) { s = s * 1664525u + 1013904223u; return (s >> 8) / 16777216.0; }
int main(void)
{
    or_params P = {9.81, 0.0, 1e-3, 0.9, 1.0, 2, 1};
    for (int rep = 0; rep < 6; rep++) {
        int nx = 2 + (int)(rnd() * 40), ny = 2 + (int)(rnd() * 30);
        or_grid G = {nx, ny, 1000.0, 1200.0, 0.0, 0.0, {rep & 1, 0, (rep >> 1) & 1, 0}};
        size_t n = (size_t)nx * ny;
        double *B = malloc(n * 8), *q[3], *o[3], *f = calloc((size_t)4 * 3 * n, 8);
        for (int c = 0; c < 3; c++) { q[c] = calloc(n, 8); o[c] = calloc(n, 8); }
        for (size_t k = 0; k < n; k++) {
            B[k] = -3000.0 * rnd() + (rnd() < 0.1 ? 3100.0 : 0.0);   /* some dry land */
            q[0][k] = B[k] < 0 ? -B[k] + 0.5 * rnd() : 0.0;
            q[1][k] = q[0][k] * (rnd() - 0.5);
            q[2][k] = q[0][k] * (rnd() - 0.5);
        }
        double cfl; int ncl;
        CHECK(or_swe_step(&G, &P, B, q[0], q[1], q[2], o[0], o[1], o[2], 5.0, &cfl, &ncl) == 0);
        CHECK(or_adj_step(&G, &P, B, q[0], q[1], q[2], o[0], o[1], o[2], 1.0, &cfl) == 0);
        CHECK(or_lin_step2d(&G, &P, B, q[0], q[1], q[2], o[0], o[1], o[2], 1.0, &cfl) == 0);
        or_grid G1 = {nx, 1, 1000.0, 1.0, 0.0, 0.0, {0, 0, 0, 0}};
        CHECK(or_lin_step(&G1, &P, B, q[0], q[1], o[0], o[1], 1.0, &cfl) == 0);
        CHECK(or_adj_step(&G1, &P, B, q[0], q[1], q[2], o[0], o[1], o[2], 1.0, &cfl) == 0);
        or_target(&G, &P, B, 5000.0, 5000.0, 3000.0, 0, o[0]);
        or_init_state(&G, &P, 0, B, q[0], o[0], o[1], o[2]);
        (void)or_dt0(&G, &P, 0, B, q[0], q[1], q[2]);
        double dt;
        (void)or_adj_nsub(&G, &P, B, 0.0, 100.0, 3, &dt);
        signed char *fl = calloc(n, 1), *acc = calloc(n, 1);
        double *mx = calloc(n, 8), *macc = calloc(n, 8);
        for (int k = 0; k < (int)(4 * 3 * n); k++) f[k] = rnd() - 0.5;
        or_flag(&G, &P, 0, B, q[0], q[1], q[2], f, 3, 1, 3, 0.1, fl, mx, acc, macc);
        or_surface_flag(&G, &P, 0, B, q[0], 0.1, fl, acc);
        or_grid Ga = {nx / 2 + 1, ny / 2 + 1, 2000.0, 2400.0, 0.0, 0.0, {0, 0, 0, 0}};
        size_t na = (size_t)Ga.nx * Ga.ny;
        double *fa = calloc((size_t)4 * 3 * na, 8), *Ba = malloc(na * 8);
        for (size_t k = 0; k < na; k++) Ba[k] = -1000.0;
        or_interp(&G, &Ga, Ba, mx);
        or_flag_interp(&G, &P, 0, B, q[0], q[1], q[2], &Ga, Ba, fa, 3, 0, 3, 0.1, fl, mx, acc, macc);
        int lo, hi;
        (void)or_window(50.0, 0.0, 20.0, 100.0, 3, &lo, &hi);
        /* the two-phase driver, with and without an adjoint grid of its own */
        double *eta0 = calloc(n, 8), *frames = calloc((size_t)5 * 3 * n, 8), *maxat = calloc((size_t)5 * n, 8);
        signed char *fat = calloc((size_t)5 * n, 1), *sfat = calloc((size_t)5 * n, 1);
        for (size_t k = 0; k < n; k++) eta0[k] = 0.5 * exp(-(double)(k % nx) / 3.0);
        or_problem pb;
        memset(&pb, 0, sizeof pb);
        pb.grid = G; pb.params = P; pb.model = 0; pb.B = B; pb.eta0 = eta0;
        pb.target_xc = 3000.0; pb.target_yc = 3000.0; pb.target_R = 4000.0;
        pb.t0 = 0.0; pb.ts = 20.0; pb.tf = 60.0; pb.tol = 1e-3; pb.K = 4; pb.flag_every = 2;
        pb.frames = frames; pb.q_out[0] = o[0]; pb.q_out[1] = o[1]; pb.q_out[2] = o[2];
        pb.flags_at = fat; pb.flag_acc = acc; pb.maxip_acc = macc; pb.surface_tol = 0.1; pb.surface_flags_at = sfat;
        pb.maxip_at = maxat;
        or_result res;
        (void)or_run(&pb, &res);
        double *fa2 = calloc((size_t)5 * 3 * na, 8);
        pb.adj_grid = Ga; pb.adj_B = Ba; pb.frames = fa2;
        (void)or_run(&pb, &res);
        free(fa2); free(eta0); free(frames); free(maxat); free(fat); free(sfat);
        free(fa); free(Ba); free(fl); free(acc); free(mx); free(macc);
        for (int c = 0; c < 3; c++) { free(q[c]); free(o[c]); }
        free(B); free(f);
    }
    double pos[3], neg[3], a[3] = {1.0, 2.0, 3.0};
    or_adj_split_parts(100.0, 150.0, 1, a, pos, neg);
    or_set_threads(1);
    printf("oracle paths ok\n");
    return 0;
}
