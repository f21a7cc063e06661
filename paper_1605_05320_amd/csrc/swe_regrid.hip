// Regridding: signature clustering of flagged cells into boxes (host) and
// piecewise-constant injection of the coarse state into refined patches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "swe.h"
#include "swe_internal.h"

namespace {

struct Box {
    int i, j, nx, ny;
};

// The flagged cells are listed once; a box's recursion then works on the
// part of the list inside it (the list is partitioned at every cut), so each
// level of the recursion costs the number of flagged cells, not the area of
// the boxes.  Shrinking, counting and the signatures see exactly the flagged
// cells of the box, as a scan of its area would.
class Clusterer {
public:
    Clusterer(const int8_t *f, int nx, int ny, int pitch, double eff, int min_side, int max_side)
        : eff_(eff), min_(min_side), max_(max_side)
    {
        // eight cells at a time: flags are sparse, and a word of zeros is skipped whole
        for (int j = 0; j < ny; ++j) {
            const int8_t *row = f + (size_t)j * pitch;
            int i = 0;
            for (; i + 8 <= nx; i += 8) {
                uint64_t w;
                std::memcpy(&w, row + i, sizeof w);
                if (w == 0) continue;
                for (int k = 0; k < 8; ++k)
                    if (row[i + k] != 0) pts_.push_back(Pt{i + k, j});
            }
            for (; i < nx; ++i)
                if (row[i] != 0) pts_.push_back(Pt{i, j});
        }
    }

    void run(std::vector<Box> &out) { run(0, pts_.size(), out); }

private:
    struct Pt {
        int i, j;
    };

    // the flagged cells pts_[p0..p1) (all of them inside the box being split)
    void run(size_t p0, size_t p1, std::vector<Box> &out)
    {
        if (p0 == p1) return;
        const Box b = bounding_box(p0, p1);
        const long long nflag = (long long)(p1 - p0);
        const long long area = (long long)b.nx * b.ny;
        const bool efficient = (double)nflag >= eff_ * (double)area;
        if (efficient && b.nx <= max_ && b.ny <= max_) {
            out.push_back(b);
            return;
        }
        int dim = -1, c = -1;
        if (efficient) {
            dim = b.nx > max_ ? 0 : 1;
            c = (dim == 0 ? b.nx : b.ny) / 2;
        } else if (!choose_cut(b, p0, p1, dim, c)) {
            out.push_back(b);
            return;
        }
        const int edge = (dim == 0 ? b.i : b.j) + c;
        const auto mid = std::stable_partition(pts_.begin() + p0, pts_.begin() + p1, [&](const Pt &p) {
            return (dim == 0 ? p.i : p.j) < edge;
        });
        const size_t pm = (size_t)(mid - pts_.begin());
        run(p0, pm, out);
        run(pm, p1, out);
    }

    Box bounding_box(size_t p0, size_t p1) const
    {
        int i0 = pts_[p0].i, i1 = i0, j0 = pts_[p0].j, j1 = j0;
        for (size_t k = p0 + 1; k < p1; ++k) {
            const Pt &p = pts_[k];
            i0 = std::min(i0, p.i); i1 = std::max(i1, p.i);
            j0 = std::min(j0, p.j); j1 = std::max(j1, p.j);
        }
        return Box{i0, j0, i1 - i0 + 1, j1 - j0 + 1};
    }

    void signatures(const Box &b, size_t p0, size_t p1, std::vector<long long> &sx, std::vector<long long> &sy) const
    {
        sx.assign(b.nx, 0);
        sy.assign(b.ny, 0);
        for (size_t k = p0; k < p1; ++k) {
            ++sx[pts_[k].i - b.i];
            ++sy[pts_[k].j - b.j];
        }
    }

    bool choose_cut(const Box &b, size_t p0, size_t p1, int &dim, int &cut) const
    {
        std::vector<long long> s[2];
        signatures(b, p0, p1, s[0], s[1]);
        const int len[2] = {b.nx, b.ny};
        // holes
        int best_d = -1, best_c = -1;
        long long best_dist = 0;
        for (int d = 0; d < 2; ++d)
            for (int c = 1; c < len[d]; ++c) {
                if (s[d][c] != 0) continue;
                long long dist = std::llabs(2LL * c - len[d]);
                if (best_d < 0 || dist < best_dist) {
                    best_d = d; best_c = c; best_dist = dist;
                }
            }
        if (best_d >= 0) {
            dim = best_d; cut = best_c;
            return true;
        }
        // inflection points of the signatures
        long long best_strength = -1;
        for (int d = 0; d < 2; ++d) {
            const int n = len[d];
            for (int k = 1; k + 2 <= n - 1; ++k) {
                long long lk = s[d][k + 1] - 2 * s[d][k] + s[d][k - 1];
                long long lk1 = s[d][k + 2] - 2 * s[d][k + 1] + s[d][k];
                if (!(lk * lk1 < 0)) continue;
                int c = k + 1;
                if (c < min_ || n - c < min_) continue;
                long long strength = std::llabs(lk1 - lk);
                long long dist = std::llabs(2LL * c - n);
                if (strength > best_strength || (strength == best_strength && dist < best_dist)) {
                    best_strength = strength; best_dist = dist; best_d = d; best_c = c;
                }
            }
        }
        if (best_d >= 0) {
            dim = best_d; cut = best_c;
            return true;
        }
        // bisection
        const int first = b.nx >= b.ny ? 0 : 1;
        for (int t = 0; t < 2; ++t) {
            int d = t == 0 ? first : 1 - first;
            int c = len[d] / 2;
            if (c >= min_ && len[d] - c >= min_) {
                dim = d; cut = c;
                return true;
            }
        }
        return false;
    }

    std::vector<Pt> pts_;
    double eff_;
    int min_, max_;
};

__global__ void __launch_bounds__(256) k_prolong(swe::CellParams C, const double *q0, const double *q1,
                                                 const double *q2, const swe_box *boxes, const swe_patch *patches,
                                                 int ratio, double *oB, double *o0, double *o1, double *o2)
{
    const int p = blockIdx.y;
    const swe_box bx = boxes[p];
    const swe_patch pt = patches[p];
    const long long n = (long long)pt.nx * pt.ny;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(idx / pt.nx), i = (int)(idx - (long long)j * pt.nx);
        int ci = bx.i_lo + i / ratio, cj = bx.j_lo + j / ratio;
        ci = ci < 0 ? 0 : (ci >= C.nx ? C.nx - 1 : ci);      // a box outside the grid reads its edge
        cj = cj < 0 ? 0 : (cj >= C.ny ? C.ny - 1 : cj);
        const size_t kc = (size_t)cj * C.pitch + ci;
        const size_t kf = (size_t)pt.offset + idx;
        oB[kf] = C.B[kc];
        o0[kf] = q0[kc];
        o1[kf] = q1[kc];
        if (o2) o2[kf] = q2[kc];
    }
}

} // namespace

extern "C" {

int32_t swe_cluster(const int8_t *flags, int32_t nx, int32_t ny, int32_t pitch, double efficiency, int32_t min_side,
                    int32_t max_side, swe_box *boxes, int32_t max_boxes)
{
    using swe::fail;
    if (!flags || (!boxes && max_boxes > 0)) return fail(SWE_E_INVAL, "null flags or boxes");
    if (nx < 1 || ny < 1 || pitch < nx || max_boxes < 0) return fail(SWE_E_INVAL, "bad sizes");
    if (!(efficiency > 0.0 && efficiency <= 1.0)) return fail(SWE_E_INVAL, "efficiency must be in (0, 1]");
    if (min_side < 1 || max_side < 2 * min_side) return fail(SWE_E_INVAL, "need min_side >= 1, max_side >= 2 min_side");
    std::vector<Box> out;
    Clusterer(flags, nx, ny, pitch, efficiency, min_side, max_side).run(out);
    for (size_t k = 0; k < out.size() && (int32_t)k < max_boxes; ++k)
        boxes[k] = swe_box{out[k].i, out[k].j, out[k].nx, out[k].ny};
    return (int32_t)out.size();
}

swe_status swe_prolong(const swe_grid *grid, const double *B, swe_fields q, const swe_box *boxes,
                       const swe_patch *patches, int32_t n, int32_t ratio, double *out_B, swe_fields out_q,
                       void *stream)
{
    using swe::fail;
    if (!grid || !B || !q.f0 || !q.f1 || !boxes || !patches || !out_B || !out_q.f0 || !out_q.f1)
        return fail(SWE_E_INVAL, "null argument");
    if (grid->ny > 1 && (!q.f2 || !out_q.f2)) return fail(SWE_E_INVAL, "null third plane in 2D");
    if (n < 1 || ratio < 1) return fail(SWE_E_INVAL, "need n >= 1 and ratio >= 1");
    if (grid->nx < 1 || grid->ny < 1 || grid->pitch < grid->nx) return fail(SWE_E_INVAL, "bad grid");
    swe::CellParams C;
    std::memset(&C, 0, sizeof C);
    C.nx = grid->nx; C.ny = grid->ny; C.pitch = grid->pitch;
    C.B = B;
    // one row of blocks per patch; a patch has at most 64 x 64 cells in the
    // level layouts, more are covered by the grid-stride loop
    dim3 g(16, (unsigned)n), blk(256);
    hipLaunchKernelGGL(k_prolong, g, blk, 0, (hipStream_t)stream, C, q.f0, q.f1, grid->ny > 1 ? q.f2 : nullptr,
                       boxes, patches, ratio, out_B, out_q.f0, out_q.f1, grid->ny > 1 ? out_q.f2 : nullptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SWE_E_HIP, "prolongation launch: %s", hipGetErrorString(e));
    return SWE_OK;
}

} // extern "C"
