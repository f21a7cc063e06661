// HIP kernels for gfx950: the marching finite-volume step (2D and 1D),
// the flagging pass and the small per-cell helpers (target data, initial
// state, max characteristic speed).
//
// Marching step.  One wavefront owns a strip of 64 columns (60 output
// columns plus a 2-column halo on each side; lane l holds column
// i = 60*strip + l - 2) and marches down `ly` rows.  Everything a row needs
// from the rows above and below is carried in registers (cells of rows
// r..r+2, y-edges r-1/2, r+1/2, r+3/2, x-edges of rows r and r+1, the
// correction flux G of edge r-1/2), and everything it needs from the
// columns left and right comes from neighbouring lanes by cross-lane
// shuffles.  So each edge of a strip is solved exactly once, the state is
// read once per strip (plus 5 halo rows per march and 4 halo columns per
// strip) and written once, there is no LDS footprint and no barrier.
#include "swe_device.h"
#include "swe_internal.h"

namespace swe {

// A-dQ and edge type of the x-edge east of this lane's cell (lane + 1).
struct XFl {
    double am[3];
    int t;
};

// What the row below still needs of a y-edge once it becomes the southern
// edge of the current row: its waves (limiter of the next y-edge) and its
// upward fluctuation (update and transverse terms).
struct YPrev {
    double z[3][3];
    double ap[3];
    int type;
};

template <class M>
__device__ __forceinline__ void keep_yprev(const Edge &e, YPrev &y)
{
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int c = 0; c < 3; ++c) y.z[p][c] = (p < M::NW && M::zc(p, c)) ? e.z[p][c] : 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) y.ap[c] = e.ap[c];
    y.type = e.type;
}

// The state of the row being updated (the rest of its cell data is no longer needed).
struct QRow {
    double q[3];
    bool upd;
};

template <class M>
__device__ __forceinline__ void keep_qrow(const typename M::Cell &c, QRow &r)
{
#pragma unroll
    for (int k = 0; k < 3; ++k) r.q[k] = M::q(c, k);
    r.upd = M::updates(c);
}

// y-edge correction flux from a YPrev-style lower neighbour (SUB: sub_edge
// holds for e on every lane).
template <class M, bool SUB>
__device__ __forceinline__ void g_tilde_r(const Edge &e, const YPrev &lo, const Edge &hi, const KParams &P,
                                          double nuy, double hnux,
                                          const double *t0, int ty0, const double *t1, int ty1,
                                          const double *t2, int ty2, const double *t3, int ty3,
                                          double G[3])
{
    G[0] = 0.0; G[1] = 0.0; G[2] = 0.0;
    if (e.type != E_WET) return;
    double Gn[3] = {0.0, 0.0, 0.0};
    if (P.order == 2) {
        double cx[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int p = 0; p < M::NW; ++p) {
            double uz[3];
            if (SUB && p == 0) {
#pragma unroll
                for (int c = 0; c < 3; ++c) uz[c] = hi.z[p][c];
                limited_wave<M, -1>(e, p, uz, nuy, cx);
            } else if (SUB && p == M::NW - 1) {
#pragma unroll
                for (int c = 0; c < 3; ++c) uz[c] = lo.z[p][c];
                limited_wave<M, 1>(e, p, uz, nuy, cx);
            } else {
                const bool upwind_lo = e.s[p] > 0.0;
#pragma unroll
                for (int c = 0; c < 3; ++c) uz[c] = upwind_lo ? lo.z[p][c] : hi.z[p][c];
                limited_wave<M, 0>(e, p, uz, nuy, cx);
            }
        }
        Gn[0] = 0.5 * cx[0]; Gn[1] = 0.5 * cx[1]; Gn[2] = 0.5 * cx[2];
    }
    to_phys(true, Gn, G);
    if (P.transverse)
        transverse_gather<M, SUB>(e, true, hnux, t0, ty0 == E_WET, t1, ty1 == E_WET, t2, ty2 == E_WET,
                                  t3, ty3 == E_WET, G);
}

// Correction fluxes of row r: G(i, r + 1/2) of y-edge yN (whose lower
// neighbour is yS) and F(i - 1/2, r) of x-edge xCur (limiter from lanes -1/+1,
// transverse terms from the y-edges of columns i-1 (lane - 1) and i (own)).
// SUB: sub_edge holds for yN and xCur on every lane.  Every lane of the
// wavefront must call this (shuffles).
template <class M, bool SUB>
__device__ __forceinline__ void row_fluxes(const KParams &P, const Edge &yN, const YPrev &yS, const Edge &yNN,
                                           const Edge &xCur, const XFl &xCurE, const Edge &xNext,
                                           const XFl &xNextE, double nux, double nuy, double hnux, double hnuy,
                                           double G_N[3], double F_W[3])
{
    g_tilde_r<M, SUB>(yN, yS, yNN, P, nuy, hnux, xCur.ap, xCur.type, xCurE.am, xCurE.t,
                      xNext.ap, xNext.type, xNextE.am, xNextE.t, G_N);
    F_W[0] = 0.0; F_W[1] = 0.0; F_W[2] = 0.0;
    double Fn[3] = {0.0, 0.0, 0.0};
    if (P.order == 2) correction_lanes<M, SUB>(xCur, nux, Fn);
    double yS_ap_W[3], yN_am_W[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        yS_ap_W[c] = from_lo(yS.ap[c]);
        yN_am_W[c] = from_lo(yN.am[c]);
    }
    int yS_t_W = from_lo(yS.type), yN_t_W = from_lo(yN.type);
    if (xCur.type == E_WET) {
        to_phys(false, Fn, F_W);
        if (P.transverse)
            transverse_gather<M, SUB>(xCur, false, hnuy, yS_ap_W, yS_t_W == E_WET, yN_am_W,
                                      yN_t_W == E_WET, yS.ap, yS.type == E_WET, yN.am,
                                      yN.type == E_WET, F_W);
    }
}

// What a marching wavefront carries from row to row.
template <class M>
struct Window {
    QRow qC;                 // row r (being updated)
    typename M::Cell cD, cE; // rows r + 1, r + 2
    YPrev yS;                // y-edge r - 1/2
    Edge yN, xCur;           // y-edge r + 1/2, x-edge of row r
    XFl xCurE;               // its east neighbour's A-dQ
    Edge yNN, xNext;         // y-edge r + 3/2, x-edge of row r + 1
    double G_S[3];           // G of edge r - 1/2
    RawCell rE;              // stored values of row r + 3, loaded one row ahead
    double smx, smy;         // largest |s| of the counted x- and y-edges
    double scell;            // largest cell term of the Courant number (rows j0 .. j1-1)
    double o[3];             // updated row, stored at the start of the next row
    bool ost;                //   by this lane
    // the edge carries no waves on any lane of the wavefront (sea at rest)
    bool zyS, zyN, zxCur, zyNN, zxNext;
};

// Stores of row r through buffer resources that cover exactly that row's
// cells (rows are wave-uniform on the uniform grid): lanes with st false get
// an offset beyond the resource and their stores are dropped, so the stores
// need no branch around them (loads and stores share one memory counter; a
// branch would merge counter states with and without the stores, and waits
// for later loads would then wait for the stores as well).  With st false on
// every lane, r is not used.
__device__ __forceinline__ void store_row_buffer(const KParams &P, int r, int i, bool st, const double (&o)[3])
{
    const size_t row = (size_t)(r > 0 ? r : 0) * P.pitch;
    const int nbytes = P.nx * (int)sizeof(double);
    const int off = st ? i * (int)sizeof(double) : 0x7ffffff8;
    double *planes[3] = {P.out0, P.out1, P.out2};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(planes[c] + row, 0, nbytes, BUF_WORD3);
        const unsigned long long b = (unsigned long long)__double_as_longlong(o[c]);
        const unsigned int v __attribute__((ext_vector_type(2))) = {(unsigned int)b, (unsigned int)(b >> 32)};
        __builtin_amdgcn_raw_buffer_store_b64(v, rs, off, 0, 0);
    }
}

// Wavefront priority by progress down the march: 3 for its first third, 2
// for the second, 1 for the rest and 0 for the last row.  A SIMD issues from
// its highest-priority ready wavefront, the oldest among equals, so with
// equal priorities the first of two wavefronts runs ahead, ends early, and
// leaves the other to finish alone with its latency uncovered; stepping the
// priority down lets the one further behind catch up, and the pair runs
// together to the end (measured 45.6 -> 42.9 us per 1024^2 step).  k: rows
// done, L: rows to do.
__device__ __forceinline__ void march_priority(int k, int L)
{
    if (k == L / 3) __builtin_amdgcn_s_setprio(2);
    else if (k == 2 * L / 3) __builtin_amdgcn_s_setprio(1);
    else if (k == L - 1) __builtin_amdgcn_s_setprio(0);
}

// Row r, first part: row r + 2's cell data and the waves of the row's two
// new edges (y-edge r + 3/2, x-edge (i - 1/2, r + 1)), without the wall and
// dry-edge cases when all their cells are wet on every lane (lane 0's x-edge,
// whose west cell is a zero fill, reaches no result and is not asked).
template <class M, bool WETPATH, bool BUFST>
__device__ __forceinline__ void new_edges(const KParams &P, const Geo &G, int lane, int i, int r, int j1, double sg,
                                          double nux, double nuy, Window<M> &W)
{
    W.cE = M::cell(P, W.rE);
    // row r - 1 goes out just before row r + 3's loads: both then have this
    // row's work to complete in before anything waits for them
    if (BUFST) store_row_buffer(P, r - 1, i, W.ost, W.o);
    W.rE = M::raw(P, G, i, r + 3);                 // in flight during this row
    if (r + 2 < j1) W.scell = fmax_(W.scell, M::cell_cfl(W.cE, sg, nux, nuy));
    typename M::Cell lD = M::lo_cell(W.cD);
    if (WETPATH && __all(W.cD.wet && W.cE.wet && (lD.wet || lane == 0))) {
        M::template waves<true>(W.cD, W.cE, true, P, W.yNN);
        M::template waves<true>(lD, W.cD, false, P, W.xNext);
    } else {
        M::template waves<false>(W.cD, W.cE, true, P, W.yNN);
        M::template waves<false>(lD, W.cD, false, P, W.xNext);
    }
    W.zyNN = __all(M::zero_waves(W.yNN));
    W.zxNext = __all(M::zero_waves(W.xNext));
}

// Row r, second part: fluctuations of the new edges, correction fluxes,
// update and store of row r, then the window moves down one row.  SUB_NEW:
// sub_edge holds for the new edges on every lane; SUB: for yN and xCur.
template <class M, bool SUB_NEW, bool SUB, bool BUFST>
__device__ __forceinline__ void finish_row(const KParams &P, const Geo &G, int i, int r, bool row_ok, bool core,
                                           double nux, double nuy, double hnux, double hnuy, Window<M> &W,
                                           int &nclamp, int &nbad)
{
    M::template fluct<SUB_NEW>(W.yNN, true);
    M::template fluct<SUB_NEW>(W.xNext, false);
    XFl xNextE;
#pragma unroll
    for (int c = 0; c < 3; ++c) xNextE.am[c] = from_hi(W.xNext.am[c]);
    xNextE.t = from_hi(W.xNext.type);

    // Where the edges around row r carry no waves on any lane, both
    // correction fluxes are zero (no limited waves, nothing to split).
    double G_N[3], F_W[3];
    if (W.zyS && W.zyN && W.zxCur && W.zxNext) {
        G_N[0] = 0.0; G_N[1] = 0.0; G_N[2] = 0.0;
        F_W[0] = 0.0; F_W[1] = 0.0; F_W[2] = 0.0;
    } else {
        row_fluxes<M, SUB>(P, W.yN, W.yS, W.yNN, W.xCur, W.xCurE, W.xNext, xNextE, nux, nuy, hnux, hnuy, G_N,
                           F_W);
    }
    double F_E[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) F_E[c] = from_hi(F_W[c]);

    double o[3] = {0.0, 0.0, 0.0};
    if (core && row_ok) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double qv = W.qC.q[c];
            if (W.qC.upd) {
                qv = qv - nux * (W.xCur.ap[c] + W.xCurE.am[c]);
                qv = qv - nuy * (W.yS.ap[c] + W.yN.am[c]);
                qv = qv - nux * (F_E[c] - F_W[c]);
                qv = qv - nuy * (G_N[c] - W.G_S[c]);
            }
            o[c] = qv;
        }
        if (M::DRYFIX) {
            // nonlinear dry-cell fix
            if (!(o[0] > P.dry_tol)) { o[1] = 0.0; o[2] = 0.0; }
            if (o[0] < 0.0) { o[0] = 0.0; ++nclamp; }
        }
        if (!isfinite(o[0]) || !isfinite(o[1]) || !isfinite(o[2])) ++nbad;
        if (!BUFST) {
            size_t k = (size_t)(G.base + (long long)r * G.pitch + i);
            P.out0[k] = o[0];
            P.out1[k] = o[1];
            P.out2[k] = o[2];
        }
    }
    if (BUFST) {
#pragma unroll
        for (int c = 0; c < 3; ++c) W.o[c] = o[c];
        W.ost = core && row_ok;
    }
    if (row_ok) {
#pragma unroll
        for (int p = 0; p < M::NW; ++p) {
            W.smx = fmax_(W.smx, fabs(W.xCur.s[p]));
            W.smy = fmax_(W.smy, fabs(W.yN.s[p]));
        }
    }

    // move the window down one row, keeping only what is still needed
    keep_yprev<M>(W.yN, W.yS);
    W.yN = W.yNN;
    W.xCur = W.xNext;
    W.xCurE = xNextE;
    keep_qrow<M>(W.cD, W.qC);
    W.cD = W.cE;
    W.zyS = W.zyN;
    W.zyN = W.zyNN;
    W.zxCur = W.zxNext;
#pragma unroll
    for (int c = 0; c < 3; ++c) W.G_S[c] = G_N[c];
}

// The marching step of one wavefront: lane `lane` holds column i of the grid
// G (its own patch in a batched level), rows j0 .. j1-1 are updated; the loop
// runs to jend (uniform over the wavefront), rows from j1 on are computed but
// neither stored nor counted.  core: the lane's cell is an output cell;
// xedge_in: its west edge counts for the Courant number.
//
// While every lane's edges have s_1 < 0 < s_NW (or are dry) - the case
// everywhere in subcritical flow - rows run the forms that know those signs
// (same values); from the first row where that fails the rest of the march
// runs the general forms.  The Courant number is nu max|s| over the edges,
// which equals the largest nu|s| exactly (rounding is monotonic), and the
// cells' own terms (nonlinear model) over the march's rows.
template <class M, bool WETPATH = true, bool SUBPATH = true, bool BUFST = false, bool PRIO = false>
__device__ __forceinline__ void march(const KParams &P, const Geo &G, int lane, int i, int j0, int j1,
                                      int jend, bool core, bool xedge_in, double dx, double dy,
                                      double &cfl, int &nclamp, int &nbad)
{
    const double nux = P.dt / dx, nuy = P.dt / dy;
    const double hnux = 0.5 * nux, hnuy = 0.5 * nuy;
    using Cell = typename M::Cell;
    const double sg = sqrt(P.g);
    if (PRIO) __builtin_amdgcn_s_setprio(3);
    Window<M> W;
    W.smx = 0.0;
    W.smy = 0.0;
    W.scell = 0.0;
    {
        // all five rows' loads in flight before the first is used
        const RawCell rA = M::raw(P, G, i, j0 - 2), rB = M::raw(P, G, i, j0 - 1), rC = M::raw(P, G, i, j0),
                      rD = M::raw(P, G, i, j0 + 1);
        W.rE = M::raw(P, G, i, j0 + 2);
        Cell cA = M::cell(P, rA);
        Cell cB = M::cell(P, rB);
        Cell cC = M::cell(P, rC);
        W.cD = M::cell(P, rD);
        if (j0 < j1) W.scell = fmax_(W.scell, M::cell_cfl(cC, sg, nux, nuy));
        if (j0 + 1 < j1) W.scell = fmax_(W.scell, M::cell_cfl(W.cD, sg, nux, nuy));
        Edge yS2, yS0, xPrev;
        Cell lB = M::lo_cell(cB);
        Cell lC = M::lo_cell(cC);
        // y-edges j0 - 3/2, j0 - 1/2, j0 + 1/2; x-edges (i - 1/2, j0 - 1), (i - 1/2, j0)
        if (WETPATH && __all(cA.wet && cB.wet && cC.wet && W.cD.wet && ((lB.wet && lC.wet) || lane == 0))) {
            M::template waves<true>(cA, cB, true, P, yS2);
            M::template waves<true>(cB, cC, true, P, yS0);
            M::template waves<true>(cC, W.cD, true, P, W.yN);
            M::template waves<true>(lB, cB, false, P, xPrev);
            M::template waves<true>(lC, cC, false, P, W.xCur);
        } else {
            M::template waves<false>(cA, cB, true, P, yS2);
            M::template waves<false>(cB, cC, true, P, yS0);
            M::template waves<false>(cC, W.cD, true, P, W.yN);
            M::template waves<false>(lB, cB, false, P, xPrev);
            M::template waves<false>(lC, cC, false, P, W.xCur);
        }
        const bool sub5 = SUBPATH && __all(sub_edge<M>(yS2) && sub_edge<M>(yS0) && sub_edge<M>(W.yN) &&
                                           sub_edge<M>(xPrev) && sub_edge<M>(W.xCur));
        if (sub5) {
            M::template fluct<true>(yS2, true);
            M::template fluct<true>(yS0, true);
            M::template fluct<true>(W.yN, true);
            M::template fluct<true>(xPrev, false);
            M::template fluct<true>(W.xCur, false);
        } else {
            M::template fluct<false>(yS2, true);
            M::template fluct<false>(yS0, true);
            M::template fluct<false>(W.yN, true);
            M::template fluct<false>(xPrev, false);
            M::template fluct<false>(W.xCur, false);
        }
        XFl ePrev;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            ePrev.am[c] = from_hi(xPrev.am[c]);
            W.xCurE.am[c] = from_hi(W.xCur.am[c]);
        }
        ePrev.t = from_hi(xPrev.type);
        W.xCurE.t = from_hi(W.xCur.type);
        W.zyS = __all(M::zero_waves(yS0));
        W.zyN = __all(M::zero_waves(W.yN));
        W.zxCur = __all(M::zero_waves(W.xCur));
        YPrev lo2;
        keep_yprev<M>(yS2, lo2);
        if (W.zyS && W.zxCur && __all(M::zero_waves(xPrev))) {
            W.G_S[0] = 0.0; W.G_S[1] = 0.0; W.G_S[2] = 0.0;
        } else if (sub5) {
            g_tilde_r<M, true>(yS0, lo2, W.yN, P, nuy, hnux, xPrev.ap, xPrev.type, ePrev.am, ePrev.t,
                               W.xCur.ap, W.xCur.type, W.xCurE.am, W.xCurE.t, W.G_S);
        } else {
            g_tilde_r<M, false>(yS0, lo2, W.yN, P, nuy, hnux, xPrev.ap, xPrev.type, ePrev.am, ePrev.t,
                                W.xCur.ap, W.xCur.type, W.xCurE.am, W.xCurE.t, W.G_S);
        }
        if (j0 < j1)
#pragma unroll
            for (int p = 0; p < M::NW; ++p) W.smy = fmax_(W.smy, fabs(yS0.s[p]));
        keep_yprev<M>(yS0, W.yS);
        keep_qrow<M>(cC, W.qC);
    }
    W.ost = false;
    W.o[0] = 0.0; W.o[1] = 0.0; W.o[2] = 0.0;

    // One exit, at the latch (an exit between a row's loads and its stores
    // makes the compiler join the two ways before the back-edge, and the
    // waits it places there then cover the stores just issued).
    int r = j0;
    if (SUBPATH && r < jend && __all(sub_edge<M>(W.yN) && sub_edge<M>(W.xCur))) {
        bool sub_new;
        do {
            if (PRIO) march_priority(r - j0, jend - j0);
            new_edges<M, WETPATH, BUFST>(P, G, lane, i, r, j1, sg, nux, nuy, W);
            sub_new = __all(sub_edge<M>(W.yNN) && sub_edge<M>(W.xNext));
            if (sub_new) {
                finish_row<M, true, true, BUFST>(P, G, i, r, r < j1, core, nux, nuy, hnux, hnuy, W, nclamp, nbad);
                ++r;
            }
        } while (sub_new && r < jend);
        if (r < jend) {            // the row whose new edges ended the loop
            finish_row<M, false, false, BUFST>(P, G, i, r, r < j1, core, nux, nuy, hnux, hnuy, W, nclamp, nbad);
            ++r;
        }
    }
    for (; r < jend; ++r) {
        if (PRIO) march_priority(r - j0, jend - j0);
        new_edges<M, WETPATH, BUFST>(P, G, lane, i, r, j1, sg, nux, nuy, W);
        finish_row<M, false, false, BUFST>(P, G, i, r, r < j1, core, nux, nuy, hnux, hnuy, W, nclamp, nbad);
    }
    if (BUFST) store_row_buffer(P, r - 1, i, W.ost, W.o);   // the last row
    const double cx = xedge_in ? nux * W.smx : 0.0, cy = core ? nuy * W.smy : 0.0;
    const double cc = core ? W.scell : 0.0;
    cfl = fmax_(cfl, fmax_(fmax_(cx, cy), cc));
}

// Wavefront epilogue: Courant number and counters of the launch (clamped
// and non-finite cells, summed over the wavefront's lanes).
__device__ __forceinline__ void march_epilogue(const KParams &P, int lane, double cfl, int nclamp, int nbad)
{
    cfl = wave_max(cfl);
    int sc = 0, sb = 0;
    if (__any(nclamp > 0 || nbad > 0)) {
        sc = wave_sum(nclamp);
        sb = wave_sum(nbad);
    }
    if (lane == 0) {
        unsigned long long *line =
            P.cfl_bits ? P.cfl_bits + (P.cfl_spread > 1 ? (size_t)(blockIdx.x % P.cfl_spread) * P.cfl_stride : 0)
                       : nullptr;
        if (P.counts_in_ring) {
            // controlled attempt: counted once its acceptance is known
            if (sc) atomicAdd(line + 1, (unsigned long long)sc);
            if (sb) atomicAdd(line + 2, (unsigned long long)sb);
        } else {
            if (sc && P.n_clamped) atomicAdd(P.n_clamped, sc);
            if (sb && P.n_nonfinite) atomicAdd(P.n_nonfinite, sb);
        }
        if (line) atomicMax(line, (unsigned long long)__double_as_longlong(cfl));
    }
}

template <class M>
__global__ void __launch_bounds__(WAVE, 2) k_march2d(KParams P)
{
    if (!resolve_ctl(P)) return;
    const int lane = threadIdx.x;
    const int G = P.nstrips * P.nchunks;
    const int t = P.xcd_remap ? xcd_logical_block(blockIdx.x, G) : blockIdx.x;
    const int strip = t / P.nchunks, chunk = t - strip * P.nchunks;
    const int i = strip * STRIP + lane - HALO;
    const int j0 = chunk * P.ly + min(chunk, P.lyr);
    const int j1 = min(j0 + P.ly + (chunk < P.lyr ? 1 : 0), P.ny);
    const bool core = lane >= HALO && lane < WAVE - HALO && i < P.nx;
    const bool xedge_in = lane >= HALO && lane <= WAVE - HALO && i <= P.nx;
    double cfl = 0.0;
    int nclamp = 0, nbad = 0;
    march<M, true, true, true, true>(P, uniform_geo(P), lane, i, j0, j1, j1, core, xedge_in, P.dx, P.dy, cfl,
                                     nclamp, nbad);
    march_epilogue(P, lane, cfl, nclamp, nbad);
}

// ---------------------------------------------------------------------------
// Batched level: wavefront passes over packed patch strips.
// ---------------------------------------------------------------------------
// One pass: each lane decodes its patch and column from the schedule, then the
// whole wavefront marches `rows` rows (lanes of shorter patches compute the
// extra rows without storing them; idle lanes load from patch 0 and store
// nothing).
template <class M>
__device__ __forceinline__ void level_pass(const KParams &P, const LevelArgs &L, int pass, double &cfl,
                                           int &nclamp, int &nbad)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const long long v = L.lanes[(size_t)pass * WAVE + lane];
    const bool idle = v < 0;
    const int patch = idle ? 0 : (int)(v >> 32);
    const int role = idle ? 0 : (int)((v >> 16) & 0xffff);
    const int col = idle ? 0 : (int)(v & 0xffff) - 32768;
    const swe_patch pt = L.patches[patch];
    Geo G;
    G.nx = pt.nx; G.ny = pt.ny; G.pitch = pt.nx;
    G.bcm = pack_bc(pt.bc);
    G.base = pt.offset;
    const int rows = L.pass_rows[pass];
    const int row0 = L.pass_row0 ? L.pass_row0[pass] : 0;
    march<M, true, true>(P, G, lane, col, row0, min(row0 + rows, pt.ny), row0 + rows, (role & 1) != 0, (role & 2) != 0,
             pt.dx, pt.dy, cfl, nclamp, nbad);
}

// One level step attempt: one wavefront per pass.
__global__ void __launch_bounds__(WAVE, 2) k_level_step(KParams P, LevelArgs L)
{
    if (!resolve_ctl(P)) return;
    double cfl = 0.0;
    int nclamp = 0, nbad = 0;
    level_pass<NL>(P, L, blockIdx.x, cfl, nclamp, nbad);
    march_epilogue(P, threadIdx.x, cfl, nclamp, nbad);
}

// Workgroup state of the persistent level kernel in LDS: the pass counter,
// the barrier's verdict, and each wavefront's Courant number (bit pattern)
// and counts of the attempt.
struct LvlShared {
    int next_pass;
    int ok;
    unsigned long long cfl_bits[LVL_WAVES];
    int ncl[LVL_WAVES], nbad[LVL_WAVES];
};

// Grid barrier of the persistent level kernel, one arrival per workgroup.
// Each wavefront leaves its Courant number and counts of the attempt in LDS
// and has its stores complete (in its XCD's L2) before the workgroup meets at
// s_barrier.  Thread 0 then adds the workgroup's Courant number and counts to
// the attempt's ring line (one atomic each for the workgroup: the largest bit
// pattern and the sums, the same words as one atomic per wavefront would
// leave), releases everything to device scope (written back past the L2),
// arrives, waits for the generation word to move on, and acquires (caches
// invalidated), so rows that workgroups on other XCDs stored in this attempt
// (the halo rows of a patch cut into row chunks) are read as stored.
// Arrivals go up a two-level tree (LVL_GROUP workgroups per counter, then one
// arrival per counter at the top) when there is more than one counter; the
// 256 workgroups of one wave of a 256-CU part arrive at a single counter
// (measured: one counter for all costs less than counters of 8 or 16
// workgroups, whose last arrivals wait for a second atomic).  A barrier that does not open within a bounded spin raises
// the error word and lets the workgroup go on, so every wavefront always
// reaches the end of the kernel.  Thread 0 also resets the workgroup's pass
// counter for the next attempt.  sync words: [1] generation, [2] error,
// [3] top-level count; counter of group k at word LVL_SYNC_LINE * (k + 1)
// (one 128-byte line each).
__device__ __forceinline__ bool level_barrier(uint32_t *sync, unsigned nb, unsigned long long *line,
                                              LvlShared &sh)
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (threadIdx.x == 0) {
        sh.next_pass = 0;
        unsigned long long m = 0;
        int sc = 0, sb = 0;
#pragma unroll
        for (int k = 0; k < LVL_WAVES; ++k) {
            m = sh.cfl_bits[k] > m ? sh.cfl_bits[k] : m;
            sc += sh.ncl[k];
            sb += sh.nbad[k];
        }
        if (sc) atomicAdd(line + 1, (unsigned long long)sc);
        if (sb) atomicAdd(line + 2, (unsigned long long)sb);
        atomicMax(line, m);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        int ok = 1;
        const unsigned g = __hip_atomic_load(&sync[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned grp = blockIdx.x / LVL_GROUP, ngrp = (nb + LVL_GROUP - 1) / LVL_GROUP;
        const unsigned in_grp = min(nb - grp * LVL_GROUP, (unsigned)LVL_GROUP);
        uint32_t *cnt = &sync[LVL_SYNC_LINE * (grp + 1)];
        bool last = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == in_grp - 1;
        if (last && ngrp > 1) {
            // the group's releases precede its arrivals: pass them on
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            cnt = &sync[3];
            last = __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == ngrp - 1;
        }
        if (last) {
            // every release precedes its arrival: pass them on to the waiters
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            __hip_atomic_store(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_s_waitcnt(0);
            __hip_atomic_fetch_add(&sync[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            long long spins = 0;
            while (__hip_atomic_load(&sync[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(1);
                if (++spins > (1ll << 23)) {
                    __hip_atomic_fetch_or(&sync[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        sh.ok = ok;
    }
    __syncthreads();
    return sh.ok != 0;
}

// All attempts of a level in one launch of workgroups of LVL_WAVES
// wavefronts.  The unit of work is the pass, as in the launch per attempt: a
// pass reads only the previous attempt's state (the planes alternate), so the
// passes of one attempt never depend on each other, and the strips and row
// chunks of one patch may run on different wavefronts.  Workgroup b owns
// passes k nb + b for even k and k nb + nb-1-b for odd k (nb workgroups; the
// passes come in the schedule's job order, longest first, so the snake order
// gives every workgroup a like share), and its wavefronts take them in that
// order from a counter in LDS as they become free.  After each attempt the
// workgroups meet at the barrier and every wavefront applies the control rule
// to the level's Courant number itself.
__global__ void __launch_bounds__(WAVE * LVL_WAVES, 2) k_level_persistent(KParams P, LevelArgs L, int n_steps)
{
    __shared__ LvlShared sh;
    swe_ctl *c = P.ctl;
    const int lane = threadIdx.x & (WAVE - 1), wave = threadIdx.x / WAVE;
    const int nb = gridDim.x, b = blockIdx.x;
    if (threadIdx.x == 0) sh.next_pass = 0;
    __syncthreads();
    swe_ctl_state S = c->s;
    unsigned long long last_bits = 0;
    bool ran = false;
    for (int a = 0; a < n_steps && !S.done; ++a) {
        if (blockIdx.x == 0 && threadIdx.x < SWE_CTL_SPREAD)
            for (int k = 0; k < 3; ++k)
                __hip_atomic_store(&c->ring[(a + 1) % 3][threadIdx.x][k], 0ull, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        KParams Q = P;
        Q.dt = S.dt;
        if (S.cur) {
            Q.in0 = P.out0; Q.in1 = P.out1; Q.in2 = P.out2;
            Q.out0 = const_cast<double *>(P.in0); Q.out1 = const_cast<double *>(P.in1);
            Q.out2 = const_cast<double *>(P.in2);
        }
        aim_ring(Q, c, a % 3);
        double cfl = 0.0;
        int nclamp = 0, nbad = 0;
        for (;;) {
            int k = 0;
            if (lane == 0) k = atomicAdd(&sh.next_pass, 1);
            k = __shfl(k, 0, WAVE);
            const long long ps = (long long)k * nb + ((k & 1) ? nb - 1 - b : b);
            if (ps >= L.n_passes) break;
            level_pass<NL>(Q, L, (int)ps, cfl, nclamp, nbad);
        }
        cfl = wave_max(cfl);
        int sc = 0, sb = 0;
        if (__any(nclamp > 0 || nbad > 0)) {
            sc = wave_sum(nclamp);
            sb = wave_sum(nbad);
        }
        if (lane == 0) {
            sh.cfl_bits[wave] = (unsigned long long)__double_as_longlong(cfl);
            sh.ncl[wave] = sc;
            sh.nbad[wave] = sb;
        }
        // the pass counter is read again only after the barrier's closing s_barrier
        if (!level_barrier(L.sync, nb, Q.cfl_bits + (size_t)(b % Q.cfl_spread) * Q.cfl_stride, sh)) break;
        last_bits = 0;
        for (int j = 0; j < SWE_CTL_SPREAD; ++j) {
            const unsigned long long v =
                __hip_atomic_load(&c->ring[a % 3][j][0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            last_bits = v > last_bits ? v : last_bits;
        }
        S = ctl_apply(S, __longlong_as_double((long long)last_bits), P.cfl_desired, P.cfl_max);
        if (blockIdx.x == 0 && threadIdx.x == 0 && S.last_accepted) {
            unsigned long long ncl = 0, nbad = 0;
            for (int j = 0; j < SWE_CTL_SPREAD; ++j) {
                ncl += __hip_atomic_load(&c->ring[a % 3][j][1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                nbad += __hip_atomic_load(&c->ring[a % 3][j][2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            c->n_clamped = c->n_clamped + (int)ncl;
            c->n_nonfinite = c->n_nonfinite + (int)nbad;
        }
        ran = true;
    }
    // Workgroup 0 leaves the loop after the last attempt or after an accepted
    // final step.  Another workgroup may read the last attempt's ring words
    // only after the clear below; it then takes a Courant number of 0, which
    // gives the same decision (accepted) in the second case and no decision
    // that matters in the first, and only workgroup 0's state is stored.
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        c->s = S;
        if (ran) c->cfl_bits = last_bits;
        clear_ring(c);
    }
}

// One row (ny == 1): the x-sweep of the marching step without y-terms, on
// the lanes of one strip (lane l holds cell i = strip*STRIP + l - HALO, whose
// data is c).  Writes the strip's cells to o0, o1 and returns the lane's
// contribution to the Courant number; counts non-finite results in nbad.
template <class M>
__device__ __forceinline__ double step1d_lanes(const KParams &P, const typename M::Cell &c, int lane, int i,
                                               double nu, double *o0, double *o1, int &nbad)
{
    const bool core = lane >= HALO && lane < WAVE - HALO && i < P.nx;
    const bool xedge_in = lane >= HALO && lane <= WAVE - HALO && i <= P.nx;
    using Cell = typename M::Cell;
    Cell l = M::lo_cell(c);
    Edge x;
    M::solve(l, c, false, P, x);
    double F[3] = {0.0, 0.0, 0.0};
    if (P.order == 2) {
        double Fn[3] = {0.0, 0.0, 0.0};
        correction_lanes<M>(x, nu, Fn);
        if (x.type == E_WET) to_phys(false, Fn, F);
    }
    double FE[3], amE[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) { FE[k] = from_hi(F[k]); amE[k] = from_hi(x.am[k]); }
    if (core) {
        double o[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            double qv = M::q(c, k);
            if (M::updates(c)) {
                qv = qv - nu * (x.ap[k] + amE[k]);
                qv = qv - nu * (FE[k] - F[k]);
            }
            o[k] = qv;
        }
        if (!isfinite(o[0]) || !isfinite(o[1])) ++nbad;
        o0[i] = o[0];
        o1[i] = o[1];
    }
    double cfl = 0.0;
    if (xedge_in)
#pragma unroll
        for (int p = 0; p < M::NW; ++p) cfl = dmax(cfl, nu * fabs(x.s[p]));
    return cfl;
}

template <class M>
__global__ void __launch_bounds__(WAVE) k_step1d(KParams P)
{
    if (!resolve_ctl(P)) return;
    const int lane = threadIdx.x;
    const int i = blockIdx.x * STRIP + lane - HALO;
    const double nu = P.dt / P.dx;
    int nbad = 0;
    const double cfl = step1d_lanes<M>(P, M::load(P, uniform_geo(P), i, 0), lane, i, nu, P.out0, P.out1, nbad);
    march_epilogue(P, lane, cfl, 0, nbad);
}

// ---------------------------------------------------------------------------
// A one-dimensional phase in one workgroup.  A 1D grid of a few thousand
// cells cannot fill the chip, and with one launch per step (and one per flag
// pass) its run is bound by launch latency.  Here one workgroup keeps the
// state in LDS (two buffers) and marches every step of the phase: its
// wavefronts take the strips of k_step1d round-robin (same lanes and halos,
// the same arithmetic through step1d_lanes) and meet at one barrier per step.
// The linear models' cell coefficients depend on the bottom only and are
// computed once per lane.
// ---------------------------------------------------------------------------
struct Strip1d {
    int mi, neg;        // mapped cell index of the lane; wall ghost (normal momentum negated)
    double c, gh;       // static part of the linear cell
    int wet;
};

template <class M>
__device__ __forceinline__ void strip1d_init(const KParams &P, int strip, int lane, Strip1d &st)
{
    const Geo G = uniform_geo(P);
    const int i = strip * STRIP + lane - HALO;
    RawCell r;
    st.mi = map_index(i, G.nx, (G.bcm & 1) ? BC_EXTRAP : BC_WALL, (G.bcm & 2) ? BC_EXTRAP : BC_WALL, r.nxg);
    r.nyg = false;
    r.q0 = 0.0;
    r.q1 = 0.0;
    r.q2 = 0.0;
    r.B = P.B[st.mi];
    const LinCell c = M::cell(P, r);
    st.neg = r.nxg;
    st.c = c.c;
    st.gh = c.gh;
    st.wet = c.wet;
}

// the cell of lane `lane` from the state planes q0, q1 (the values lin_cell
// gives for the raw cell)
__device__ __forceinline__ LinCell strip1d_cell(const Strip1d &st, const double *q0, const double *q1)
{
    LinCell c;
    c.q0 = q0[st.mi];
    const double m = q1[st.mi];
    c.q1 = st.neg ? -m : m;
    c.q2 = 0.0;
    c.c = st.c;
    c.gh = st.gh;
    c.wet = st.wet;
    return c;
}

// Adjoint phase: snapshot 0 is given; snapshot k is the state after nsub
// steps of dt = P.dt from snapshot k - 1.
template <class M>
__global__ void __launch_bounds__(RUN1D_THREADS) k_adj_run1d(Run1dArgs A)
{
    extern __shared__ double lds[];
    const int nx = A.P.nx;
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1), nwaves = blockDim.x / WAVE;
    const int nstrips = (nx + STRIP - 1) / STRIP;
    // plane comp of state buffer b (offsets from lds, so that the accesses
    // stay LDS accesses: through a table of pointers they became flat ones,
    // each of which waited for the global stores in flight)
    auto q = [&](int b, int comp) __attribute__((always_inline)) { return lds + (2 * b + comp) * nx; };
    for (int k = threadIdx.x; k < nx; k += blockDim.x) {
        q(0, 0)[k] = A.frames[k];
        q(0, 1)[k] = A.frames[A.fplane + k];
    }
    Strip1d st[RUN1D_MAXS];
#pragma unroll
    for (int s = 0; s < RUN1D_MAXS; ++s) {
        const int strip = wave + s * nwaves;
        if (strip < nstrips) strip1d_init<M>(A.P, strip, lane, st[s]);
    }
    __syncthreads();
    const double nu = A.P.dt / A.P.dx;
    int cur = 0;
    for (int k = 1; k <= A.K; ++k) {
        for (int sub = 0; sub < A.nsub; ++sub) {
#pragma unroll
            for (int s = 0; s < RUN1D_MAXS; ++s) {
                const int strip = wave + s * nwaves;
                if (strip >= nstrips) break;
                int nbad = 0;
                (void)step1d_lanes<M>(A.P, strip1d_cell(st[s], q(cur, 0), q(cur, 1)), lane,
                                      strip * STRIP + lane - HALO, nu, q(cur ^ 1, 0), q(cur ^ 1, 1), nbad);
            }
            __syncthreads();
            cur ^= 1;
        }
        // the next step writes the other buffer; the one after waits at a
        // barrier that every thread reaches only after its copy
        double *f = A.frames + (size_t)2 * k * A.fplane;
        for (int i = threadIdx.x; i < nx; i += blockDim.x) {
            f[i] = q(cur, 0)[i];
            f[A.fplane + i] = q(cur, 1)[i];
        }
    }
}

// Forward phase under device-side control: the attempts of swe_advance with
// flagging, the control rule applied by every thread to the attempt's
// Courant number (the maximum of the lanes' values as bit patterns; equal to
// the per-step launches' for every finite state, whose run fails either way
// when a value is NaN).  The states that are to be flagged are recorded for
// k_hist_flag.  At the end the control block holds what the per-step launches
// and k_ctl_finish leave there.
template <class M>
__global__ void __launch_bounds__(RUN1D_THREADS) k_fwd_run1d(Run1dArgs A)
{
    extern __shared__ double lds[];
    const int nx = A.P.nx;
    const int wave = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1), nwaves = blockDim.x / WAVE;
    const int nstrips = (nx + STRIP - 1) / STRIP;
    // plane comp of state buffer b (offsets from lds, so that the accesses
    // stay LDS accesses: through a table of pointers they became flat ones,
    // each of which waited for the global stores in flight)
    auto q = [&](int b, int comp) __attribute__((always_inline)) { return lds + (2 * b + comp) * nx; };
    unsigned long long *red = (unsigned long long *)(lds + 4 * nx);   // [2][RUN1D_WAVES]
    int *redn = (int *)(red + 2 * RUN1D_WAVES);                        // [2][RUN1D_WAVES]
    swe_ctl *c = A.P.ctl;
    swe_ctl_state S = c->s;
    const double *g0 = S.cur ? A.P.out0 : A.P.in0, *g1 = S.cur ? A.P.out1 : A.P.in1;
    for (int k = threadIdx.x; k < nx; k += blockDim.x) {
        q(0, 0)[k] = g0[k];
        q(0, 1)[k] = g1[k];
    }
    Strip1d st[RUN1D_MAXS];
#pragma unroll
    for (int s = 0; s < RUN1D_MAXS; ++s) {
        const int strip = wave + s * nwaves;
        if (strip < nstrips) strip1d_init<M>(A.P, strip, lane, st[s]);
    }
    __syncthreads();
    int cur = 0, nrec = 0, nbad_acc = 0, a = 0;
    unsigned long long last_bits = 0;
    for (; a < A.max_attempts && !S.done; ++a) {
        const double nu = S.dt / A.P.dx;
        unsigned long long bits = 0;
        int nbad = 0;
#pragma unroll
        for (int s = 0; s < RUN1D_MAXS; ++s) {
            const int strip = wave + s * nwaves;
            if (strip >= nstrips) break;
            const double cf = step1d_lanes<M>(A.P, strip1d_cell(st[s], q(cur, 0), q(cur, 1)), lane,
                                              strip * STRIP + lane - HALO, nu, q(cur ^ 1, 0), q(cur ^ 1, 1), nbad);
            const unsigned long long b = (unsigned long long)__double_as_longlong(cf);
            bits = b > bits ? b : bits;
        }
        bits = wave_max_u64(bits);
        if (__any(nbad > 0)) nbad = wave_sum(nbad);
        if (lane == 0) {
            // (the launch has RUN1D_WAVES wavefronts: every slot is written)
            red[(a & 1) * RUN1D_WAVES + wave] = bits;
            redn[(a & 1) * RUN1D_WAVES + wave] = nbad;
        }
        __syncthreads();
        // the slots of this attempt are read before the next barrier; the
        // next attempt writes the other half
        unsigned long long all = 0;
        int nball = 0;
#pragma unroll
        for (int w = 0; w < RUN1D_WAVES; ++w) {
            const unsigned long long v = red[(a & 1) * RUN1D_WAVES + w];
            all = v > all ? v : all;
            nball += redn[(a & 1) * RUN1D_WAVES + w];
        }
        S = ctl_apply(S, __longlong_as_double((long long)all), A.P.cfl_desired, A.P.cfl_max);
        last_bits = all;
        if (S.last_accepted) {
            cur ^= 1;
            nbad_acc += nball;
            if (A.hist && (S.done || S.n_accepted % A.flag_every == 0)) {
                double *h = A.hist + (size_t)nrec * 2 * nx;
                for (int k = threadIdx.x; k < nx; k += blockDim.x) {
                    h[k] = q(cur, 0)[k];
                    h[nx + k] = q(cur, 1)[k];
                }
                if (threadIdx.x == 0) {
                    A.hist_t[nrec] = S.t;
                    A.hist_done[nrec] = S.done;
                }
                ++nrec;
            }
        }
    }
    const bool any = A.max_attempts > 0;
    if (any && a < A.max_attempts) {
        // attempts left after the segment ended run as skipped launches: the
        // last of them resolves with Courant number 0 (accepted flag cleared)
        S = ctl_apply(S, 0.0, A.P.cfl_desired, A.P.cfl_max);
        last_bits = 0;
    }
    double *o0 = S.cur ? A.P.out0 : const_cast<double *>(A.P.in0);
    double *o1 = S.cur ? A.P.out1 : const_cast<double *>(A.P.in1);
    for (int k = threadIdx.x; k < nx; k += blockDim.x) {
        o0[k] = q(cur, 0)[k];
        o1[k] = q(cur, 1)[k];
    }
    if (threadIdx.x == 0) {
        if (any) {
            c->s = S;
            c->cfl_bits = last_bits;
            if (nbad_acc) c->n_nonfinite = c->n_nonfinite + nbad_acc;
            if (nrec) c->n_flag_calls = c->n_flag_calls + nrec;
            clear_ring(c);
        }
        *A.n_rec = nrec;
    }
}

// ---------------------------------------------------------------------------
// Device-side step control (single thread).
// ---------------------------------------------------------------------------

__global__ void k_ctl_set(swe_ctl *c, double t, double dt, double t_out, int cur)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    swe_ctl_state S;
    S.t = t;
    S.dt = dt;
    S.t_out = t_out;
    S.cur = cur;
    S.final_step = 0;
    S.done = 0;
    S.last_accepted = 0;
    S.n_accepted = 0;
    S.n_rejected = 0;
    ctl_clamp(S);
    c->s = S;
    c->cfl_bits = 0;
    c->n_clamped = 0;
    c->n_nonfinite = 0;
    c->n_flag_calls = 0;
    clear_ring(c);
}

__global__ void k_ctl_retarget(swe_ctl *c, double t_out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    swe_ctl_state S = c->s;
    S.t_out = t_out;
    S.done = 0;
    S.last_accepted = 0;
    ctl_clamp(S);
    c->s = S;
}

// Resolve the last of n attempts into ctl->s and clear the Courant slots.
__global__ void k_ctl_finish(swe_ctl *c, int n, double cfl_desired, double cfl_max)
{
    if (threadIdx.x != 0 || blockIdx.x != 0 || n < 1) return;
    unsigned long long bits = ring_bits(c, (n - 1) % 3);
    c->s = ctl_apply(c->slot[(n - 1) & 1], __longlong_as_double((long long)bits), cfl_desired, cfl_max);
    add_counts_if_accepted(c, (n - 1) % 3, c->s);
    c->cfl_bits = bits;
    clear_ring(c);
}

// ---------------------------------------------------------------------------
// Flagging pass: one thread per cell, coalesced across the row.
// ---------------------------------------------------------------------------
// Interpolation position of coordinate x on an axis of n cell centres
// x_lo + (c + 1/2) d: lower centre index i0 and weight w in [0, 1] (constant
// beyond the outermost centres); and the index of the cell containing x.
__device__ __forceinline__ void axis_weights(double x, double x_lo, double d, int n, int &i0, double &w, int &ic)
{
    const double u = (x - x_lo) / d;
    double c = floor(u);
    c = c < 0.0 ? 0.0 : (c > n - 1 ? (double)(n - 1) : c);
    ic = (int)c;
    const double xi = u - 0.5;
    double f = floor(xi);
    const double top = n >= 2 ? (double)(n - 2) : 0.0;
    f = f < 0.0 ? 0.0 : (f > top ? top : f);
    i0 = (int)f;
    double ww = n >= 2 ? xi - f : 0.0;
    w = ww < 0.0 ? 0.0 : (ww > 1.0 ? 1.0 : ww);
}

// Skipping snapshots that are exactly zero.  A snapshot contributes
// |<q, 0>| = 0 wherever it is zero, which leaves the maximum as it is (q
// finite).  The decision is taken per wavefront, for the rectangle of
// snapshot-grid indices its 64 cells read: a snapshot whose non-zero box
// misses the rectangle is skipped by the whole wavefront, the others are read
// by every lane (reading zeros where a lane lies outside the box).  Lane l
// tests snapshot base + l, so one ballot covers 64 snapshots of the window.
struct IdxRect { int i0, i1, j0, j1; };

__device__ __forceinline__ unsigned long long window_mask(const int *bounds, int base, int k_hi, const IdxRect &r)
{
    const int f = base + (int)(threadIdx.x & (WAVE - 1));
    bool hit = false;
    if (f <= k_hi) {
        const int *b = bounds + 4 * f;
        const int b0 = b[0], b1 = b[1], b2 = b[2], b3 = b[3];   // four loads in flight together
        hit = (r.i1 >= b0) & (r.i0 <= b1) & (r.j1 >= b2) & (r.j0 <= b3);
    }
    return __ballot(hit);
}

// m = max(m, |dot(f)|) over the snapshots f = base + s of the bits s of
// `mask`, in increasing order, four at a time so that their loads are in
// flight together; a short last group repeats its last snapshot, which leaves
// the maximum as it is.
template <class Dot>
__device__ __forceinline__ double max_over_mask(unsigned long long mask, int base, const Dot &dot, double m)
{
    while (mask) {
        int f[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (mask) {
                f[u] = base + __ffsll((long long)mask) - 1;
                mask &= mask - 1;
            } else {
                f[u] = f[u > 0 ? u - 1 : 0];
            }
        }
        double ip[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) ip[u] = dot(f[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) m = dmax(m, fabs(ip[u]));
    }
    return m;
}

// m = max over the window's snapshots of |<q, q^_k>| at cell (i, j) (storage
// index k), 0 where the forward or the adjoint cell is dry.  With snapshots on
// their own grid (INTERP), q^_k is interpolated (bilinear in 2D, linear in 1D)
// at the cell centre and the adjoint cell is the one containing the centre.
// Called by every lane of the wavefront (`live` false past the last cell,
// with k a valid index); with boxes, r is the wavefront's rectangle.  The
// snapshots are visited in increasing order either way.
template <bool TWOD, bool INTERP>
__device__ __forceinline__ double flag_m(const FlagParams &F, int i, int j, size_t k, bool live, IdxRect r)
{
    const double B = F.B[k];
    const double q0 = F.q0[k];
    const double eta = F.nonlinear ? (q0 + B) - F.sea_level : q0;
    double m = 0.0;
    const size_t plane = INTERP ? (size_t)F.any * F.apitch : (size_t)F.ny * F.pitch;
    const size_t fstride = (size_t)F.ncomp * plane;
    bool adj_wet;
    // cell offsets in the snapshot planes: the cell itself, or the four
    // interpolation corners and their weights
    size_t k00 = k, k10 = k, k01 = k, k11 = k;
    double ux = 1.0, wx = 0.0, uy = 1.0, wy = 0.0;
    if (!INTERP) {
        adj_wet = dmax(0.0, F.sea_level - B) > F.dry_tol;
    } else {
        const double x = F.x_lo + (i + 0.5) * F.dx;
        int i0, ic, j0 = 0, jc = 0;
        axis_weights(x, F.ax_lo, F.adx, F.anx, i0, wx, ic);
        if (TWOD) {
            const double y = F.y_lo + (j + 0.5) * F.dy;
            axis_weights(y, F.ay_lo, F.ady, F.any, j0, wy, jc);
        }
        adj_wet = dmax(0.0, F.sea_level - F.aB[(size_t)jc * F.apitch + ic]) > F.dry_tol;
        const int i1 = F.anx >= 2 ? i0 + 1 : i0;
        const int j1 = TWOD && F.any >= 2 ? j0 + 1 : j0;
        k00 = (size_t)j0 * F.apitch + i0;
        k10 = (size_t)j0 * F.apitch + i1;
        k01 = (size_t)j1 * F.apitch + i0;
        k11 = (size_t)j1 * F.apitch + i1;
        ux = 1.0 - wx;
        uy = 1.0 - wy;
    }
    const bool fwd_wet = F.nonlinear ? (q0 > F.dry_tol)
                                     : (INTERP ? dmax(0.0, F.sea_level - B) > F.dry_tol : adj_wet);
    const bool go = live && adj_wet && fwd_wet;
    const double q1 = go ? F.q1[k] : 0.0;
    const double q2 = TWOD && go ? F.q2[k] : 0.0;
    auto dot = [&](int f) {
        const double *fr = F.frames + (size_t)f * fstride;
        double v[3];
#pragma unroll
        for (int c = 0; c < (TWOD ? 3 : 2); ++c) {
            const double *p = fr + (size_t)c * plane;
            if (!INTERP)
                v[c] = p[k00];
            else if (TWOD)
                v[c] = uy * (ux * p[k00] + wx * p[k10]) + wy * (ux * p[k01] + wx * p[k11]);
            else
                v[c] = ux * p[k00] + wx * p[k10];
        }
        double ip = eta * v[0] + q1 * v[1];
        if (TWOD) ip = ip + q2 * v[2];
        return ip;
    };
    for (int base = F.k_lo; base <= F.k_hi; base += WAVE) {
        unsigned long long mask;
        if (F.bounds) {
            mask = window_mask(F.bounds, base, F.k_hi, r);
        } else {
            const int nb = F.k_hi - base + 1;
            mask = nb >= WAVE ? ~0ull : (1ull << nb) - 1;
        }
        if (go) m = max_over_mask(mask, base, dot, m);
    }
    return m;
}

// The rectangle of snapshot-grid indices read by the wavefront whose cells
// are the flat indices wb .. min(wb + 63, n - 1) (row-major, nx per row): the
// cells themselves, or with snapshots on their own grid the interpolation
// corners of those cells (monotone in the cell centre along each axis).
__device__ __forceinline__ IdxRect wave_rect(const FlagParams &F, long long wb, long long n)
{
    const long long last = (wb + WAVE < n ? wb + WAVE : n) - 1;
    IdxRect r;
    r.j0 = (int)(wb / F.nx);
    r.j1 = (int)(last / F.nx);
    if (r.j0 == r.j1) {
        r.i0 = (int)(wb - (long long)r.j0 * F.nx);
        r.i1 = (int)(last - (long long)r.j1 * F.nx);
    } else {
        r.i0 = 0;
        r.i1 = F.nx - 1;
    }
    if (!F.interp) return r;
    int a, c;
    double w;
    IdxRect s;
    axis_weights(F.x_lo + (r.i0 + 0.5) * F.dx, F.ax_lo, F.adx, F.anx, s.i0, w, c);
    axis_weights(F.x_lo + (r.i1 + 0.5) * F.dx, F.ax_lo, F.adx, F.anx, a, w, c);
    s.i1 = F.anx >= 2 ? a + 1 : a;
    s.j0 = s.j1 = 0;
    if (F.twod) {
        axis_weights(F.y_lo + (r.j0 + 0.5) * F.dy, F.ay_lo, F.ady, F.any, s.j0, w, c);
        axis_weights(F.y_lo + (r.j1 + 0.5) * F.dy, F.ay_lo, F.ady, F.any, a, w, c);
        s.j1 = F.any >= 2 ? a + 1 : a;
    }
    return s;
}

// Bounding box (i_lo, i_hi, j_lo, j_hi) of the cells of snapshot
// blockIdx.y with a non-zero value in any plane (a NaN counts as non-zero);
// an empty snapshot keeps (nx, -1, ny, -1) from k_bounds_init.
__global__ void __launch_bounds__(256) k_bounds_init(int *bounds, int n_frames, int nx, int ny)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * n_frames) return;
    const int w = t & 3;
    bounds[t] = w == 0 ? nx : (w == 2 ? ny : -1);
}

__global__ void __launch_bounds__(256) k_frame_bounds(const double *frames, int nx, int ny, int pitch, int ncomp,
                                                      int *bounds)
{
    const int k = blockIdx.y;
    const size_t plane = (size_t)ny * pitch;
    const double *f = frames + (size_t)k * ncomp * plane;
    int ilo = nx, ihi = -1, jlo = ny, jhi = -1;
    const long long n = (long long)nx * ny;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        const int j = (int)(idx / nx), i = (int)(idx - (long long)j * nx);
        const size_t o = (size_t)j * pitch + i;
        bool nz = false;
        for (int c = 0; c < ncomp; ++c) nz = nz || !(f[c * plane + o] == 0.0);
        if (nz) {
            ilo = min(ilo, i); ihi = max(ihi, i);
            jlo = min(jlo, j); jhi = max(jhi, j);
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        ilo = min(ilo, __shfl_xor(ilo, off, WAVE));
        ihi = max(ihi, __shfl_xor(ihi, off, WAVE));
        jlo = min(jlo, __shfl_xor(jlo, off, WAVE));
        jhi = max(jhi, __shfl_xor(jhi, off, WAVE));
    }
    // the workgroup's four wavefronts meet in LDS, then one thread updates
    // the snapshot's box (one set of atomics per workgroup: the workgroups of
    // a snapshot all update the same four words)
    __shared__ int box[4][4];
    const int w = threadIdx.x / WAVE;
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        box[w][0] = ilo;
        box[w][1] = ihi;
        box[w][2] = jlo;
        box[w][3] = jhi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < (int)(blockDim.x / WAVE); ++v) {
            ilo = min(ilo, box[v][0]);
            ihi = max(ihi, box[v][1]);
            jlo = min(jlo, box[v][2]);
            jhi = max(jhi, box[v][3]);
        }
        if (ihi >= 0) {
            atomicMin(&bounds[4 * k + 0], ilo);
            atomicMax(&bounds[4 * k + 1], ihi);
            atomicMin(&bounds[4 * k + 2], jlo);
            atomicMax(&bounds[4 * k + 3], jhi);
        }
    }
}

template <bool TWOD, bool INTERP>
__global__ void __launch_bounds__(256) k_flag(FlagParams F)
{
    const long long n = (long long)F.nx * F.ny;
    const int lane = threadIdx.x & (WAVE - 1);
    // whole wavefronts step through the cells (the snapshot masks are ballots)
    for (long long wb = (long long)blockIdx.x * blockDim.x + (threadIdx.x - lane); wb < n;
         wb += (long long)gridDim.x * blockDim.x) {
        const bool live = wb + lane < n;
        const long long idx = live ? wb + lane : wb;
        int j = (int)(idx / F.nx), i = (int)(idx - (long long)j * F.nx);
        size_t k = (size_t)j * F.pitch + i;
        const double m = flag_m<TWOD, INTERP>(F, i, j, k, live, F.bounds ? wave_rect(F, wb, n) : IdxRect{0, 0, 0, 0});
        if (!live) continue;
        int8_t fl = m > F.tol ? 1 : 0;
        if (F.flags) F.flags[k] = fl;
        if (F.maxip) F.maxip[k] = m;
        if (F.flag_acc) F.flag_acc[k] = (int8_t)(F.flag_acc[k] | fl);
        if (F.maxip_acc) F.maxip_acc[k] = dmax(F.maxip_acc[k], m);
    }
}

// Window of eq. (ip_timerange) on the device (same arithmetic as adj_window).
__device__ __forceinline__ double dev_snap(double r)
{
    double rr = rint(r);
    return fabs(r - rr) <= 1e-9 ? rr : r;
}

__device__ __forceinline__ bool dev_window(double t, double t0, double ts, double tf, int K, int &lo, int &hi)
{
    double ds = (tf - t0) / K;
    double T = fmin(t + (tf - ts), tf);
    double sa = tf - T, sb = tf - t;
    if (sb < 0.0) {
        lo = 1;
        hi = 0;
        return false;
    }
    double l = floor(dev_snap(sa / ds)), h = ceil(dev_snap(sb / ds));
    if (l < 0.0) l = 0.0;
    if (h > K) h = K;
    lo = (int)l;
    hi = (int)h;
    return true;
}

// Flagging after step attempt `attempt` of a device-controlled sequence: the
// attempt's outcome is derived from its state slot and its (now complete)
// Courant number; if it was accepted and either reached the segment's output
// time or its accepted-step count is a multiple of flag_every, flag the new
// state (in plane set a or b according to the new cur) at the new time.
template <bool TWOD, bool INTERP>
__global__ void __launch_bounds__(256) k_flag_ctl(FlagParams F, FlagCtl C)
{
    swe_ctl *c = C.ctl;
    swe_ctl_state S = ctl_apply(c->slot[C.attempt & 1],
                                __longlong_as_double((long long)ring_bits(c, C.attempt % 3)), C.cfl_desired,
                                C.cfl_max);
    if (!S.last_accepted) return;
    if (!(S.done || S.n_accepted % C.flag_every == 0)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) c->n_flag_calls = c->n_flag_calls + 1;
    int lo, hi;
    dev_window(S.t, C.t0, C.ts, C.tf, C.K, lo, hi);
    F.k_lo = lo;
    F.k_hi = hi;
    if (S.cur) { F.q0 = C.b0; F.q1 = C.b1; F.q2 = C.b2; }
    else       { F.q0 = C.a0; F.q1 = C.a1; F.q2 = C.a2; }
    F.flags = S.done ? C.flags_final : nullptr;
    const long long n = (long long)F.nx * F.ny;
    const int lane = threadIdx.x & (WAVE - 1);
    for (long long wb = (long long)blockIdx.x * blockDim.x + (threadIdx.x - lane); wb < n;
         wb += (long long)gridDim.x * blockDim.x) {
        const bool live = wb + lane < n;
        const long long idx = live ? wb + lane : wb;
        int j = (int)(idx / F.nx), i = (int)(idx - (long long)j * F.nx);
        size_t k = (size_t)j * F.pitch + i;
        const double m = flag_m<TWOD, INTERP>(F, i, j, k, live, F.bounds ? wave_rect(F, wb, n) : IdxRect{0, 0, 0, 0});
        if (!live) continue;
        int8_t fl = m > F.tol ? 1 : 0;
        if (F.flags) F.flags[k] = fl;
        if (F.flag_acc) F.flag_acc[k] = (int8_t)(F.flag_acc[k] | fl);
        if (F.maxip_acc) F.maxip_acc[k] = dmax(F.maxip_acc[k], m);
    }
}

// The recorded states of a 1D forward launch: m of record blockIdx.y at every
// cell (window from the record's time, as k_flag_ctl takes it) ...
template <bool INTERP>
__global__ void __launch_bounds__(256) k_hist_flag(FlagParams F, HistArgs H)
{
    const int r = blockIdx.y;
    if (r >= *H.n_rec) return;
    int lo, hi;
    dev_window(H.hist_t[r], H.t0, H.ts, H.tf, H.K, lo, hi);
    F.k_lo = lo;
    F.k_hi = hi;
    F.q0 = H.hist + (size_t)r * 2 * F.nx;
    F.q1 = F.q0 + F.nx;
    F.q2 = nullptr;
    const long long n = F.nx;
    const int lane = threadIdx.x & (WAVE - 1);
    for (long long wb = (long long)blockIdx.x * blockDim.x + (threadIdx.x - lane); wb < n;
         wb += (long long)gridDim.x * blockDim.x) {
        const bool live = wb + lane < n;
        const int i = (int)(live ? wb + lane : wb);
        const double m = flag_m<false, INTERP>(F, i, 0, (size_t)i, live, F.bounds ? wave_rect(F, wb, n) : IdxRect{0, 0, 0, 0});
        if (live) H.m[(size_t)r * F.nx + i] = m;
    }
}

// ... then per cell the records in order: flags of the record that ends the
// segment, the running OR of the flags and maximum of m.
__global__ void __launch_bounds__(256) k_hist_fold(FlagParams F, HistArgs H)
{
    const int nrec = *H.n_rec;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < F.nx; i += gridDim.x * blockDim.x) {
        int8_t acc = F.flag_acc ? F.flag_acc[i] : 0;
        double macc = F.maxip_acc ? F.maxip_acc[i] : 0.0;
        for (int r0 = 0; r0 < nrec; r0 += 8) {
            // eight records' loads in flight together, folded in order
            double mv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) mv[u] = r0 + u < nrec ? H.m[(size_t)(r0 + u) * F.nx + i] : 0.0;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (r0 + u >= nrec) break;
                const double m = mv[u];
                const int8_t fl = m > F.tol ? 1 : 0;
                if (H.hist_done[r0 + u] && H.flags_final) H.flags_final[i] = fl;
                acc = (int8_t)(acc | fl);
                macc = dmax(macc, m);
            }
        }
        if (F.flag_acc) F.flag_acc[i] = acc;
        if (F.maxip_acc) F.maxip_acc[i] = macc;
    }
}

// Target data, initial state, maximum speed: per-cell helpers.
__global__ void __launch_bounds__(256) k_target(CellParams C, double xc, double yc, double R, int shape)
{
    const long long n = (long long)C.nx * C.ny;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        int j = (int)(idx / C.nx), i = (int)(idx - (long long)j * C.nx);
        size_t k = (size_t)j * C.pitch + i;
        double x = C.x_lo + (i + 0.5) * C.dx;
        double ddx = x - xc;
        double r2 = ddx * ddx;
        if (C.ny > 1) {
            double y = C.y_lo + (j + 0.5) * C.dy;
            double ddy = y - yc;
            r2 = r2 + ddy * ddy;
        }
        double v = shape == 0 ? exp(-r2 / (R * R)) : (r2 <= R * R ? 1.0 : 0.0);
        double hb = dmax(0.0, C.sea_level - C.B[k]);
        C.o0[k] = hb > C.dry_tol ? v : 0.0;
        C.o1[k] = 0.0;
        if (C.o2) C.o2[k] = 0.0;
    }
}

__global__ void __launch_bounds__(256) k_init(CellParams C, const double *eta0, int nonlinear)
{
    const long long n = (long long)C.nx * C.ny;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        int j = (int)(idx / C.nx), i = (int)(idx - (long long)j * C.nx);
        size_t k = (size_t)j * C.pitch + i;
        double B = C.B[k];
        if (nonlinear) {
            C.o0[k] = dmax(0.0, eta0[k] - B);
        } else {
            double hb = dmax(0.0, C.sea_level - B);
            C.o0[k] = hb > C.dry_tol ? eta0[k] : 0.0;
        }
        C.o1[k] = 0.0;
        if (C.o2) C.o2[k] = 0.0;
    }
}

// Surface criterion: flag = wet && |eta| > tol, eta relative to sea level.
__global__ void __launch_bounds__(256) k_surface_flag(CellParams C, const double *q0, double tol, int nonlinear,
                                                      int8_t *flags, int8_t *flag_acc)
{
    const long long n = (long long)C.nx * C.ny;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        int j = (int)(idx / C.nx), i = (int)(idx - (long long)j * C.nx);
        size_t k = (size_t)j * C.pitch + i;
        double B = C.B[k], h = q0[k];
        bool wet;
        double eta;
        if (nonlinear) {
            wet = h > C.dry_tol;
            eta = (h + B) - C.sea_level;
        } else {
            wet = dmax(0.0, C.sea_level - B) > C.dry_tol;
            eta = h;
        }
        const int8_t fl = (wet && fabs(eta) > tol) ? 1 : 0;
        if (flags) flags[k] = fl;
        if (flag_acc) flag_acc[k] = (int8_t)(flag_acc[k] | fl);
    }
}

__global__ void __launch_bounds__(256) k_max_speed(CellParams C, const double *q0, const double *q1,
                                                   const double *q2, int mode, unsigned long long *out)
{
    // mode 0: nonlinear state; 1: static linear coefficients
    const long long n = (long long)C.nx * C.ny;
    double m = 0.0;
    for (long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
         idx += (long long)gridDim.x * blockDim.x) {
        int j = (int)(idx / C.nx), i = (int)(idx - (long long)j * C.nx);
        size_t k = (size_t)j * C.pitch + i;
        double a, b;
        if (mode == 0) {
            double h = q0[k];
            if (!(h > C.dry_tol)) continue;
            double c = sqrt(C.g * h);
            a = (fabs(q1[k] / h) + c) / C.dx;
            b = C.ny > 1 ? (fabs(q2[k] / h) + c) / C.dy : 0.0;
        } else {
            double hb = dmax(0.0, C.sea_level - C.B[k]);
            if (!(hb > C.dry_tol)) continue;
            double c = sqrt(C.g * hb);
            a = c / C.dx;
            b = C.ny > 1 ? c / C.dy : 0.0;
        }
        m = dmax(m, dmax(a, b));
    }
    m = wave_max(m);
    if ((threadIdx.x & (WAVE - 1)) == 0) atomicMax(out, (unsigned long long)__double_as_longlong(m));
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static int grid_cells(long long n)
{
    long long b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (int)b;
}

hipError_t launch_step(int model, const KParams &P, hipStream_t s)
{
    dim3 block(WAVE);
    if (P.ny == 1) {
        dim3 grid((P.nx + STRIP - 1) / STRIP);
        if (model == MODEL_ADJ) hipLaunchKernelGGL(k_step1d<ADJ<false>>, grid, block, 0, s, P);
        else if (model == MODEL_LIN) hipLaunchKernelGGL(k_step1d<LIN1>, grid, block, 0, s, P);
        else return hipErrorInvalidValue;
    } else {
        KParams Q = P;
        Q.nstrips = (P.nx + STRIP - 1) / STRIP;
        Q.nchunks = P.lyr > 0 ? (P.ny - P.lyr) / P.ly : (P.ny + P.ly - 1) / P.ly;
        dim3 grid(Q.nstrips * Q.nchunks);
        if (model == MODEL_NL) hipLaunchKernelGGL(k_march2d<NL>, grid, block, 0, s, Q);
        else if (model == MODEL_ADJ) hipLaunchKernelGGL(k_march2d<ADJ<true>>, grid, block, 0, s, Q);
        else if (model == MODEL_LIN) hipLaunchKernelGGL(k_march2d<LIN2>, grid, block, 0, s, Q);
        else return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_ctl_set(swe_ctl *c, double t, double dt, double t_out, int cur, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_set, dim3(1), dim3(1), 0, s, c, t, dt, t_out, cur);
    return hipGetLastError();
}

hipError_t launch_ctl_retarget(swe_ctl *c, double t_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_retarget, dim3(1), dim3(1), 0, s, c, t_out);
    return hipGetLastError();
}

hipError_t launch_ctl_finish(swe_ctl *c, int n, double cfl_desired, double cfl_max, hipStream_t s)
{
    hipLaunchKernelGGL(k_ctl_finish, dim3(1), dim3(1), 0, s, c, n, cfl_desired, cfl_max);
    return hipGetLastError();
}

hipError_t launch_level_step(const KParams &P, const LevelArgs &L, hipStream_t s)
{
    hipLaunchKernelGGL(k_level_step, dim3(L.n_passes), dim3(WAVE), 0, s, P, L);
    return hipGetLastError();
}

int level_persistent_capacity()
{
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_level_persistent, WAVE * LVL_WAVES, 0) != hipSuccess)
        return 0;
    return std::min(cus * per, LVL_MAX_BLOCKS);
}

hipError_t launch_level_persistent(const KParams &P, const LevelArgs &L, int n_steps, int nw, hipStream_t s)
{
    KParams p = P;
    LevelArgs l = L;
    int n = n_steps;
    void *args[] = {&p, &l, &n};
    return hipLaunchCooperativeKernel((const void *)k_level_persistent, dim3(nw), dim3(WAVE * LVL_WAVES), args, 0, s);
}

// Count elements whose bit patterns differ (schedule-invariance checks).
__global__ void __launch_bounds__(256) k_count_diff(const double *a, const double *b, long long n, int *out)
{
    int local = 0;
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
         k += (long long)gridDim.x * blockDim.x)
        local += __double_as_longlong(a[k]) != __double_as_longlong(b[k]);
    for (int off = 32; off > 0; off >>= 1) local += __shfl_xor(local, off, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0 && local) atomicAdd(out, local);
}

hipError_t launch_count_diff(const double *a, const double *b, long long n, int *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_count_diff, dim3(grid_cells(n)), dim3(256), 0, s, a, b, n, out);
    return hipGetLastError();
}

hipError_t launch_flag_ctl(const FlagParams &F, const FlagCtl &C, hipStream_t s)
{
    const dim3 grid(grid_cells((long long)F.nx * F.ny));
    switch ((F.twod ? 2 : 0) + (F.interp ? 1 : 0)) {
    case 0: hipLaunchKernelGGL((k_flag_ctl<false, false>), grid, dim3(256), 0, s, F, C); break;
    case 1: hipLaunchKernelGGL((k_flag_ctl<false, true>), grid, dim3(256), 0, s, F, C); break;
    case 2: hipLaunchKernelGGL((k_flag_ctl<true, false>), grid, dim3(256), 0, s, F, C); break;
    default: hipLaunchKernelGGL((k_flag_ctl<true, true>), grid, dim3(256), 0, s, F, C); break;
    }
    return hipGetLastError();
}

hipError_t launch_frame_bounds(const double *frames, int nx, int ny, int pitch, int ncomp, int K, int *bounds,
                               hipStream_t s)
{
    const int nf = K + 1;
    hipLaunchKernelGGL(k_bounds_init, dim3((4 * nf + 255) / 256), dim3(256), 0, s, bounds, nf, nx, ny);
    long long blocks = ((long long)nx * ny + 255) / 256;
    if (blocks > 64) blocks = 64;
    hipLaunchKernelGGL(k_frame_bounds, dim3((unsigned)blocks, (unsigned)nf), dim3(256), 0, s, frames, nx, ny, pitch,
                       ncomp, bounds);
    return hipGetLastError();
}

hipError_t launch_flag(const FlagParams &F, hipStream_t s)
{
    const dim3 grid(grid_cells((long long)F.nx * F.ny));
    switch ((F.twod ? 2 : 0) + (F.interp ? 1 : 0)) {
    case 0: hipLaunchKernelGGL((k_flag<false, false>), grid, dim3(256), 0, s, F); break;
    case 1: hipLaunchKernelGGL((k_flag<false, true>), grid, dim3(256), 0, s, F); break;
    case 2: hipLaunchKernelGGL((k_flag<true, false>), grid, dim3(256), 0, s, F); break;
    default: hipLaunchKernelGGL((k_flag<true, true>), grid, dim3(256), 0, s, F); break;
    }
    return hipGetLastError();
}

size_t run1d_lds_bytes(int nx)
{
    if (nx < 2 || nx > RUN1D_MAX_NX) return 0;
    const size_t bytes = (size_t)4 * nx * sizeof(double) + 2 * RUN1D_WAVES * (sizeof(unsigned long long) + sizeof(int));
    int dev = 0, lim = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&lim, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
    if (bytes > (size_t)lim) return 0;
    if (bytes > 65536) {
        // beyond 64 KiB the kernels must be allowed the larger allocation;
        // where that is refused the step-by-step launches are used instead
        if (hipFuncSetAttribute((const void *)k_adj_run1d<ADJ<false>>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)bytes) != hipSuccess ||
            hipFuncSetAttribute((const void *)k_fwd_run1d<LIN1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)bytes) != hipSuccess) {
            (void)hipGetLastError();
            return 0;
        }
    }
    return bytes;
}

hipError_t launch_adj_run1d(const Run1dArgs &A, hipStream_t s)
{
    const size_t lds = run1d_lds_bytes(A.P.nx);
    if (!lds) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_adj_run1d<ADJ<false>>, dim3(1), dim3(RUN1D_THREADS), lds, s, A);
    return hipGetLastError();
}

hipError_t launch_fwd_run1d(const Run1dArgs &A, hipStream_t s)
{
    const size_t lds = run1d_lds_bytes(A.P.nx);
    if (!lds || A.max_attempts > RUN1D_RECORDS) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fwd_run1d<LIN1>, dim3(1), dim3(RUN1D_THREADS), lds, s, A);
    return hipGetLastError();
}

hipError_t launch_hist_flag(const FlagParams &F, const HistArgs &H, hipStream_t s)
{
    const unsigned bx = (unsigned)((F.nx + 255) / 256);
    const dim3 grid(bx, RUN1D_RECORDS);
    if (F.interp) hipLaunchKernelGGL((k_hist_flag<true>), grid, dim3(256), 0, s, F, H);
    else hipLaunchKernelGGL((k_hist_flag<false>), grid, dim3(256), 0, s, F, H);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_hist_fold, dim3(bx), dim3(256), 0, s, F, H);
    return hipGetLastError();
}

hipError_t launch_target(const CellParams &C, double xc, double yc, double R, int shape, hipStream_t s)
{
    hipLaunchKernelGGL(k_target, dim3(grid_cells((long long)C.nx * C.ny)), dim3(256), 0, s, C, xc, yc, R, shape);
    return hipGetLastError();
}

hipError_t launch_surface_flag(const CellParams &C, const double *q0, double tol, int nonlinear, int8_t *flags,
                               int8_t *flag_acc, hipStream_t s)
{
    hipLaunchKernelGGL(k_surface_flag, dim3(grid_cells((long long)C.nx * C.ny)), dim3(256), 0, s, C, q0, tol,
                       nonlinear, flags, flag_acc);
    return hipGetLastError();
}

hipError_t launch_init(const CellParams &C, const double *eta0, int nonlinear, hipStream_t s)
{
    hipLaunchKernelGGL(k_init, dim3(grid_cells((long long)C.nx * C.ny)), dim3(256), 0, s, C, eta0, nonlinear);
    return hipGetLastError();
}

hipError_t launch_max_speed(const CellParams &C, const double *q0, const double *q1, const double *q2,
                            int mode, unsigned long long *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_max_speed, dim3(grid_cells((long long)C.nx * C.ny)), dim3(256), 0, s, C, q0, q1,
                       q2, mode, out);
    return hipGetLastError();
}

} // namespace swe
