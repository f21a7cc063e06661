// Exercises the library's host-only code paths under ASan/UBSan.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>
#include "swe.h"
#define CHECK(c) do { if (!(c)) { std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); return 1; } } while (0)
int main() {
    // snapshot window over random arguments
    unsigned s = 12345u;
    auto rnd = [&]() { s = s * 1664525u + 1013904223u; return (s >> 8) / 16777216.0; };
    for (int k = 0; k < 20000; ++k) {
        int K = 1 + (int)(rnd() * 80);
        double t0 = 0.0, tf = 7200.0, ts = rnd() * tf, t = rnd() * 1.1 * tf;
        int lo, hi;
        CHECK(adj_window(t, t0, ts, tf, K, &lo, &hi) == SWE_OK);
        CHECK((lo <= hi && lo >= 0 && hi <= K) || (lo == 1 && hi == 0));
    }
    // level schedules of random patch sets, every kind and chunking
    for (int rep = 0; rep < 20; ++rep) {
        int n = 1 + (int)(rnd() * 300);
        std::vector<swe_patch> p(n);
        long long off = 0;
        for (int k = 0; k < n; ++k) {
            std::memset(&p[k], 0, sizeof p[k]);
            p[k].nx = 2 + (int)(rnd() * 70); p[k].ny = 2 + (int)(rnd() * 70);
            p[k].dx = p[k].dy = 100.0; p[k].offset = off; off += (long long)p[k].nx * p[k].ny;
        }
        for (int kind = 0; kind < 2; ++kind)
            for (int chunk : {0, 1, 7, 16}) {
                int nj = 0;
                int np = swe_level_schedule(p.data(), n, kind, chunk, nullptr, nullptr, nullptr, nullptr, &nj);
                CHECK(np > 0 && nj > 0);
                std::vector<long long> lanes((size_t)np * 64);
                std::vector<int> rows(np), row0(np), jp(nj + 1);
                int nj2 = 0;
                CHECK(swe_level_schedule(p.data(), n, kind, chunk, (int64_t *)lanes.data(), rows.data(), row0.data(),
                                         jp.data(), &nj2) == np && nj2 == nj);
            }
    }
    // clustering of random flag fields
    for (int rep = 0; rep < 30; ++rep) {
        int nx = 1 + (int)(rnd() * 200), ny = 1 + (int)(rnd() * 200), pitch = nx + (int)(rnd() * 5);
        std::vector<signed char> f((size_t)ny * pitch, 0);
        double dens = rnd() * 0.3;
        for (int j = 0; j < ny; ++j) for (int i = 0; i < nx; ++i) f[(size_t)j * pitch + i] = rnd() < dens;
        std::vector<swe_box> b(4096);
        int nb = swe_cluster((const int8_t *)f.data(), nx, ny, pitch, 0.7, 4, 32, b.data(), (int)b.size());
        CHECK(nb >= 0);
        int nb2 = swe_cluster((const int8_t *)f.data(), nx, ny, pitch, 0.7, 4, 32, b.data(), 1);   // truncated output
        CHECK(nb2 == nb);
    }
    // footprints, workspaces and argument checks that must fail before any device work
    swe_request rq; std::memset(&rq, 0, sizeof rq);
    rq.grid.nx = rq.grid.ny = rq.grid.pitch = 256; rq.grid.dx = rq.grid.dy = 4000.0;
    rq.params.order = 2; rq.params.transverse = 1; rq.params.g = 9.81; rq.params.dry_tol = 1e-3;
    rq.params.cfl_desired = 0.9; rq.params.cfl_max = 1.0;
    std::vector<double> host(256 * 256, -100.0);
    rq.B_host = host.data(); rq.eta0_host = host.data(); rq.K = 32; rq.tf = 7200; rq.ts = 3600; rq.tol = 1e-4;
    rq.flag_every = 4; rq.target_R = 2e4;
    CHECK(swe_serve_footprint(&rq) > 0);
    swe_problem pb; std::memset(&pb, 0, sizeof pb);
    pb.grid = rq.grid; pb.params = rq.params; pb.K = 8; pb.tf = 100; pb.flag_every = 1; pb.target_R = 1e4;
    double fake;
    pb.B = pb.eta0 = &fake; pb.frames = &fake; pb.q_out.f0 = pb.q_out.f1 = pb.q_out.f2 = &fake;
    CHECK(swe_run_workspace_bytes(&pb) > 0);
    swe_result res;
    pb.grid.nx = pb.grid.ny = pb.grid.pitch = 1300;
    CHECK(swe_run_static(&pb, &res, nullptr) == SWE_E_NOMEM);
    CHECK(std::strlen(swe_last_error()) > 0);
    swe_grid g = rq.grid; swe_params pr = rq.params; swe_fields a = {&fake, &fake, &fake};
    CHECK(swe_step(&g, &pr, &fake, a, a, 1.0, nullptr, nullptr) == SWE_E_INVAL);   // in aliases out
    g.nx = 1;
    CHECK(swe_step(&g, &pr, &fake, a, a, 1.0, nullptr, nullptr) == SWE_E_INVAL);
    std::printf("host paths ok\n");
    return 0;
}
