// push_deposit.hip -- FP64 push + deposit kernels and the charge kernel.
//
// Per particle and step (Sec. 2.2-2.3 of arXiv:2503.04558): CIC gather of the
// six staggered field components at x^n, a full-step generalised Boris kick
// at x^n, the geodesic predictor and `ncorr` trapezoid corrector passes, axis
// reflection, Esirkepov deposit of the move on a 3x3 vertex window, and
// removal at the radial edges.
//
// Two kernel shapes share that body, each in FP64 and in split precision
// (push_deposit_f64 / _split, push_deposit_f64_tiled / _split_tiled):
//   push_deposit_f64        one thread per particle, any particle order,
//                           deposit with global FP64 atomics;
//   push_deposit_f64_tiled  one workgroup per slice (up to 256 particles) of a
//                           cell-sorted tile (see grpic_launch.hpp), one
//                           particle per thread, deposit into an LDS window
//                           with LDS FP64 atomics, one flush of the window's
//                           non-zero entries to global memory.  (A loop over
//                           several particles per thread makes the compiler
//                           keep the loop-invariant FP64 constants in
//                           registers: 256 VGPRs and one wave per SIMD.)
#include "grpic_device.hpp"
#include "grpic_launch.hpp"
#include "grpic_qed.hpp"

#include <algorithm>
#include <climits>
#include <type_traits>

namespace grpic {

// Bilinear interpolation in index space of the grid array F at (f, h),
// where (f, h) are grid coordinates already shifted by the stagger.
// Two consecutive elements of a row as one vector load (8-byte aligned).
typedef double double2_a8 __attribute__((ext_vector_type(2), aligned(8)));
typedef float float2_a4 __attribute__((ext_vector_type(2), aligned(4)));

__device__ __forceinline__ double cic_f64(const double* __restrict__ F, const StepArgs& A, double f, double h) {
    const double ff = floor(f), fh = floor(h);
    const int i = (int)ff, j = (int)fh;
    const double wf = f - ff, wh = h - fh;
    const uint32_t o = grid_index(A, i, j);
    const double2_a8 lo = *reinterpret_cast<const double2_a8*>(elem(F, o));
    const double2_a8 hi = *reinterpret_cast<const double2_a8*>(elem(F, o + (uint32_t)A.pitch));
    return (1.0 - wf) * (1.0 - wh) * lo.x + wf * (1.0 - wh) * hi.x + (1.0 - wf) * wh * lo.y + wf * wh * hi.y;
}

// Gather with the cubic shape: the 4 x 4 vertices around (f, h) =
// (xi - sr, eta - st) of the component's own stagger (guard rows and the
// columns beyond the axes included; the grid has guard >= 3).
__device__ __forceinline__ double spline3_f64(const double* __restrict__ F, const StepArgs& A, double f, double h) {
    const int i = (int)floor(f), j = (int)floor(h);
    double wx[4], wy[4];
    for (int a = 0; a < 4; ++a) {
        wx[a] = shape3(f - (double)(i - 1 + a));
        wy[a] = shape3(h - (double)(j - 1 + a));
    }
    double sum = 0.0;
    for (int a = 0; a < 4; ++a) {
        const uint32_t o = grid_index(A, i - 1 + a, j - 1);
        double row = 0.0;
        for (int b = 0; b < 4; ++b) row = fma(wy[b], *elem(F, o + (uint32_t)b), row);
        sum = fma(wx[a], row, sum);
    }
    // an empty asm that takes the sum and clobbers memory: the next
    // component's 16 loads are not hoisted above this one's sum, so at most
    // one component's loads are in flight (issued all together, the 96
    // loads' results outlived the register file: 256 VGPRs and spills)
    asm volatile("" : "+v"(sum) : : "memory");
    return sum;
}

// Minimum (MAX: maximum) of v over the 64 lanes of a wave, all of them
// active, returned wave-uniform.  DPP lane permutations combine pairs,
// quads, half rows and rows of 16; the row broadcasts of lanes 15 and 31
// then fold rows 0 and 2 into 1 and 3, and rows 0-1 into 2-3, so lane 63
// holds the result.  Lanes a broadcast does not write keep the operation's
// identity, so each step is one DPP min or max.
template <bool MAX>
__device__ __forceinline__ int wave_reduce(int v) {
    const int identity = MAX ? INT_MIN : INT_MAX;
    auto op = [](int a, int b) { return MAX ? max(a, b) : min(a, b); };
    v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0xB1, 0xF, 0xF, false));    // quad_perm [1,0,3,2]
    v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x4E, 0xF, 0xF, false));    // quad_perm [2,3,0,1]
    v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x141, 0xF, 0xF, false));   // row_half_mirror
    v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x140, 0xF, 0xF, false));   // row_mirror
    v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x142, 0xA, 0xF, false));   // row_bcast:15 to rows 1, 3
    v = op(v, __builtin_amdgcn_update_dpp(identity, v, 0x143, 0xC, 0xF, false));   // row_bcast:31 to rows 2, 3
    return __builtin_amdgcn_readlane(v, 63);
}

struct Events {
    int live, out, bad, refl, spill;
};

// Anchors (r at a row's corner, sin and cos at a column's) of one tile and
// the drift margin around it (rows ti - kMarginRows .. ti + kMarginRows,
// columns j_lo - kMarginCols .. j_lo + kTileCells + kMarginCols), copied
// once per workgroup into LDS from the launch's anchor table; particles that
// have drifted further evaluate their own (same functions, same values).
constexpr int kAnchorRows = 2 * kMarginRows + 1;
constexpr int kAnchorCols = kTileCells + 2 * kMarginCols + 1;
struct TileAnchors {
    int i_lo, j_lo;                           // grid indices of r[0] and s[0], c[0]
    double r[kAnchorRows];
    double s[kAnchorCols], c[kAnchorCols];
};

static_assert(kSliceThreads >= 64 + kAnchorCols && kSliceThreads3 >= 64 + kAnchorCols,
              "waves 1 and 2 fill the anchor table's columns");

template <class R>
__device__ __forceinline__ Anchor<R> anchor_for(const StepArgs& A, int ci, int cj, const TileAnchors* T) {
    if (T && A.small_steps) {
        const int di = ci - T->i_lo, dj = cj - T->j_lo;
        if (di >= 0 && di < kAnchorRows && dj >= 0 && dj < kAnchorCols) {
            Anchor<R> an;
            an.ci = ci;
            an.cj = cj;
            an.r = R(T->r[di]);
            an.s = R(T->s[dj]);
            an.c = R(T->c[dj]);
            return an;
        }
    }
    return make_anchor<R>(A, ci, cj);
}

// A particle's state as read at the start of a step (element type T: double,
// or float in split precision); the weight is read by the step itself, after
// the input checks.  The tiled kernel issues these loads before its LDS
// set-up so that their latency overlaps it.
template <class T>
struct ParticleIn {
    int cell, s;
    T dxr, dxt, u[3];
};

// Particle base + k of the particle arrays: base is uniform across the
// workgroup (its slice's or block's first particle), so each access is a
// scalar base register plus a 32-bit lane offset.
struct PIdx {
    int64_t base;
    uint32_t k;
    template <class T>
    __device__ __forceinline__ T* at(T* arr) const { return elem(arr + base, k); }
    template <class T>
    __device__ __forceinline__ T* at(void* arr) const { return at(static_cast<T*>(arr)); }
    template <class T>
    __device__ __forceinline__ const T* at(const void* arr) const { return at(static_cast<const T*>(arr)); }
};

template <class T>
__device__ __forceinline__ ParticleIn<T> load_particle(const StepArgs& A, const PIdx& p) {
    ParticleIn<T> in;
    in.cell = *p.at(A.cell);
    in.s = *p.at(A.sp);
    in.dxr = *p.at<T>(A.xr);
    in.dxt = *p.at<T>(A.xth);
    in.u[0] = *p.at<T>(A.ur);
    in.u[1] = *p.at<T>(A.uth);
    in.u[2] = *p.at<T>(A.uph);
    return in;
}

// A particle's state after a step, for the caller to store: kind 0 nothing
// (it was removed before the step), 1 removed now (cell = -1, the rest
// unchanged), 2 the new cell, offsets and momenta in x = (xr, xth, ur, uth,
// uph).
template <class T>
struct ParticleOut {
    int kind, cell;
    T x[5];
};

template <class T>
__device__ __forceinline__ void store_particle(const StepArgs& A, const PIdx& p, const ParticleOut<T>& o) {
    if (o.kind == 0) return;
    *p.at(A.cell) = o.kind == 2 ? o.cell : -1;
    if (o.kind != 2) return;
    *p.at<T>(A.xr) = o.x[0];
    *p.at<T>(A.xth) = o.x[1];
    *p.at<T>(A.ur) = o.x[2];
    *p.at<T>(A.uth) = o.x[3];
    *p.at<T>(A.uph) = o.x[4];
}

// Advances live particle p by one step; its new state goes to out.  Returns
// true when the move is to be deposited (mv filled), false when the particle
// was or became removed without a deposit.
// EARLY_QW: read the move's charge before the correctors (the monopole
// kernel, whose emission test holds more values live, reads it at the end).
template <bool SHORT, int KICK, int ORDER, bool EARLY_QW = true>
__device__ __forceinline__ bool advance_f64(const StepArgs& A, const PIdx& p, const ParticleIn<double>& in, Move& mv,
                                            Events& ev, const TileAnchors* T, ParticleOut<double>& out) {
    out.kind = 0;
    const int cell = in.cell;
    if (cell < 0) return false;
    ev.live = 1;
    out.kind = 1;
    const double* w = static_cast<const double*>(A.w);
    const double dxr = in.dxr, dxt = in.dxt;
    const int s = in.s;
    // Inputs that would index outside the grid arrays are removed as bad.
    if (cell >= A.nr * A.nth || s >= A.nsp || !(dxr >= 0.0 && dxr <= 1.0 && dxt >= 0.0 && dxt <= 1.0)) {
        ev.bad = 1;
        return false;
    }
    // the kick's q/m, a per-lane read of the argument block: issued here so
    // that it completes during the gather (it is live until the kick anyway)
    const double qm = A.qm[s];
    const int ci = div_by(cell, A.nth, A.inv_nth), cj = cell - ci * A.nth;
    const double xi0 = (double)ci + dxr, eta0 = (double)cj + dxt;
    double u[3] = {in.u[0], in.u[1], in.u[2]};
    const double* const* F = reinterpret_cast<const double* const*>(A.F);
    auto gather = [&](int c, double f, double h) {
        if constexpr (ORDER == 3) return spline3_f64(F[c], A, f, h);
        else return cic_f64(F[c], A, f, h);
    };
    const double D[3] = {gather(0, xi0 - 0.5, eta0), gather(1, xi0, eta0 - 0.5), gather(2, xi0, eta0)};
    const double B[3] = {gather(3, xi0, eta0 - 0.5), gather(4, xi0 - 0.5, eta0), gather(5, xi0 - 0.5, eta0 - 0.5)};
    const bool massless = A.massless[s] != 0;
    const double dt = A.dt;
    const double eps = massless ? 0.0 : 1.0;
    // one exp and one sincos per particle, at its start cell's corner
    const Anchor<double> an = anchor_for<double>(A, ci, cj, T);
    double f0[5], f1[5], yt[5];
    {
        // the kick takes the metric at x^n; the first RHS is evaluated from
        // r, sin, cos after it (the metric's derivatives and the six field
        // values are then never live together)
        double r0, s0, c0;
        point_at<SHORT>(A, an, xi0, eta0, r0, s0, c0);
        Metric<double> k0;
        ks_metric<double>(A.a, A.M, r0, s0, c0, k0);
        if (!massless) kick<KICK>(k0, qm, dt, D, B, u);
        geodesic_rhs_point(A, eps, r0, s0, c0, u[0], u[1], u[2], f0);
    }
    // geodesic predictor-corrector on y = (xi, eta, phi, u_r, u_th); u_ph is constant
    // The corrector sums f0 + f1 before adding y0: forming y0 + dt/2 f0 once
    // would round the absolute position (xi and eta run up to the grid size,
    // so an ulp is ~2e-13 cells) once more per corrector, and the momentum
    // picks that up through the metric and field gradients.
    const double y0[5] = {xi0, eta0, 0.0, u[0], u[1]};
    // the move's charge q w, read here so that its loads complete during the
    // correctors (before the kick they would raise the register peak)
    double qw = 0.0;
    if constexpr (EARLY_QW) qw = A.q[s] * *p.at(w);
    for (int c = 0; c < 5; ++c) yt[c] = y0[c] + dt * f0[c];
    for (int it = 0; it < A.ncorr; ++it) {
        geodesic_rhs<SHORT>(A, an, eps, yt[0], yt[1], yt[3], yt[4], u[2], f1);
        for (int c = 0; c < 5; ++c) yt[c] = y0[c] + 0.5 * dt * (f1[c] + f0[c]);
    }
    double xi1 = yt[0], eta1 = yt[1];
    double u1t = yt[4];
    const bool finite = isfinite(xi1) && isfinite(eta1) && isfinite(yt[2]) && isfinite(yt[3])
                      && isfinite(yt[4]) && isfinite(u[2]);
    if (!finite || fabs(xi1 - xi0) >= 1.0 || fabs(eta1 - eta0) >= 1.0) {
        ev.bad = 1;
        return false;
    }
    if (eta1 < 0.0) { eta1 = -eta1; u1t = -u1t; ev.refl = 1; }
    else if (eta1 > (double)A.nth) { eta1 = 2.0 * A.nth - eta1; u1t = -u1t; ev.refl = 1; }
    if constexpr (!EARLY_QW) qw = A.q[s] * *p.at(w);
    mv = make_move(qw, xi0, eta0, xi1, eta1, yt[2]);
    if (A.phi) *p.at<double>(A.phi) += yt[2];
    if (xi1 < 0.0 || xi1 >= (double)A.nr) {
        ev.out = 1;
    } else {
        const int i1 = (int)floor(xi1);
        int j1 = (int)floor(eta1);
        if (j1 >= A.nth) j1 = A.nth - 1;
        out.kind = 2;
        out.cell = i1 * A.nth + j1;
        out.x[0] = xi1 - (double)i1;
        out.x[1] = eta1 - (double)j1;
        out.x[2] = yt[3];
        out.x[3] = u1t;
        out.x[4] = u[2];
    }
    return true;
}

// ---------------------------------------------------------------- split precision
// Position as int32 cell + float offset, float momenta, weight and fields.
// The kick and the predictor-corrector run in float on offsets relative to
// the start cell, except in rows with r < 2M (fp64_rows) and in columns
// within ~5.7 degrees of the axis (pole_cols), where they run in double.
// The deposit is FP64 on the stored end point (int + float offsets are exact
// in double), so discrete charge continuity holds at FP64 round-off.

// Bilinear interpolation of a float grid array around cell (ci, cj) at
// offsets (fx, fy) already shifted by the stagger (fx, fy in [-1/2, 1]).
__device__ __forceinline__ float cic_f32(const float* __restrict__ F, const StepArgs& A, int ci, int cj,
                                         float fx, float fy) {
    const float fi = floorf(fx), fj = floorf(fy);
    const float wf = fx - fi, wh = fy - fj;
    const uint32_t o = grid_index(A, ci + (int)fi, cj + (int)fj);
    const float2_a4 lo = *reinterpret_cast<const float2_a4*>(elem(F, o));
    const float2_a4 hi = *reinterpret_cast<const float2_a4*>(elem(F, o + (uint32_t)A.pitch));
    return (1.0f - wf) * (1.0f - wh) * lo.x + wf * (1.0f - wh) * hi.x + (1.0f - wf) * wh * lo.y + wf * wh * hi.y;
}

// Kick and predictor-corrector in precision R on offsets from the start
// cell; y = (dxi, deta, phi, u_r, u_th) on return, u[2] = u_ph.
template <bool SHORT, class R>
__device__ __forceinline__ void split_core(const StepArgs& A, int ci, int cj, R dxr, R dxt, R eps, R qm,
                                           bool massless, const R D[3], const R B[3], R u[3], R yt[5],
                                           const TileAnchors* T) {
    const Anchor<R> an = anchor_for<R>(A, ci, cj, T);
    const R dt = R(A.dt);
    R f0[5], f1[5];
    {
        R r0, s0, c0;
        point_rel<SHORT>(A, an, dxr, dxt, r0, s0, c0);
        Metric<R> k0;
        ks_metric<R>(R(A.a), R(A.M), r0, s0, c0, k0);
        if (!massless) boris_kick(k0, qm, dt, D, B, u);
        geodesic_rhs_point(A, eps, r0, s0, c0, u[0], u[1], u[2], f0);
    }
    const R y0[5] = {dxr, dxt, R(0), u[0], u[1]};
    const R hdt = R(0.5) * dt;
    R yh[5];
    for (int c = 0; c < 5; ++c) {
        yt[c] = y0[c] + dt * f0[c];
        yh[c] = y0[c] + hdt * f0[c];
    }
    for (int it = 0; it < A.ncorr; ++it) {
        R r, sn, cs;
        point_rel<SHORT>(A, an, yt[0], yt[1], r, sn, cs);
        geodesic_rhs_point(A, eps, r, sn, cs, yt[3], yt[4], u[2], f1);
        for (int c = 0; c < 5; ++c) yt[c] = yh[c] + hdt * f1[c];
    }
}

// A float offset in [0, 1): values that round up to 1 take the largest float below 1.
__device__ __forceinline__ float offset_f32(double x) {
    const float f = (float)x;
    return f < 1.0f ? f : 0.99999994f;
}

template <bool SHORT>
__device__ __forceinline__ bool advance_split(const StepArgs& A, const PIdx& p, const ParticleIn<float>& in, Move& mv,
                                              Events& ev, const TileAnchors* T, ParticleOut<float>& out) {
    out.kind = 0;
    const int cell = in.cell;
    if (cell < 0) return false;
    ev.live = 1;
    out.kind = 1;
    const float* w = static_cast<const float*>(A.w);
    const float fxr = in.dxr, fxt = in.dxt;
    const int s = in.s;
    if (cell >= A.nr * A.nth || s >= A.nsp || !(fxr >= 0.0f && fxr <= 1.0f && fxt >= 0.0f && fxt <= 1.0f)) {
        ev.bad = 1;
        return false;
    }
    const double qw = A.q[s] * (double)*p.at(w);          // read early, as in the FP64 step
    const bool massless = A.massless[s] != 0;
    const double qm = A.qm[s];
    const int ci = div_by(cell, A.nth, A.inv_nth), cj = cell - ci * A.nth;
    const float* const* F = reinterpret_cast<const float* const*>(A.F);
    const float Df[3] = {cic_f32(F[0], A, ci, cj, fxr - 0.5f, fxt), cic_f32(F[1], A, ci, cj, fxr, fxt - 0.5f),
                         cic_f32(F[2], A, ci, cj, fxr, fxt)};
    const float Bf[3] = {cic_f32(F[3], A, ci, cj, fxr, fxt - 0.5f), cic_f32(F[4], A, ci, cj, fxr - 0.5f, fxt),
                         cic_f32(F[5], A, ci, cj, fxr - 0.5f, fxt - 0.5f)};
    double y[5], uph1;
    const bool fp64 = ci < A.fp64_rows || cj < A.pole_cols || cj >= A.nth - A.pole_cols;
    if (fp64) {
        const double D[3] = {Df[0], Df[1], Df[2]}, B[3] = {Bf[0], Bf[1], Bf[2]};
        double u[3] = {in.u[0], in.u[1], in.u[2]};
        split_core<SHORT, double>(A, ci, cj, (double)fxr, (double)fxt, massless ? 0.0 : 1.0, qm, massless, D, B, u, y, T);
        uph1 = u[2];
    } else {
        float u[3] = {in.u[0], in.u[1], in.u[2]};
        float yf[5];
        split_core<SHORT, float>(A, ci, cj, fxr, fxt, massless ? 0.0f : 1.0f, (float)qm, massless, Df, Bf, u, yf, T);
        for (int c = 0; c < 5; ++c) y[c] = yf[c];
        uph1 = u[2];
    }
    const double xi0 = (double)ci + (double)fxr, eta0 = (double)cj + (double)fxt;
    double xi1 = (double)ci + y[0], eta1 = (double)cj + y[1];
    double u1t = y[4];
    const bool finite = isfinite(xi1) && isfinite(eta1) && isfinite(y[2]) && isfinite(y[3]) && isfinite(y[4])
                      && isfinite(uph1);
    if (!finite || fabs(xi1 - xi0) >= 1.0 || fabs(eta1 - eta0) >= 1.0) {
        ev.bad = 1;
        return false;
    }
    if (eta1 < 0.0) { eta1 = -eta1; u1t = -u1t; ev.refl = 1; }
    else if (eta1 > (double)A.nth) { eta1 = 2.0 * A.nth - eta1; u1t = -u1t; ev.refl = 1; }
    // the end point as stored (cell + float offset), exact in double
    const int i1 = (int)floor(xi1);
    int j1 = (int)floor(eta1);
    if (j1 >= A.nth) j1 = A.nth - 1;
    const float ox = offset_f32(xi1 - (double)i1), oy = offset_f32(eta1 - (double)j1);
    mv = make_move(qw, xi0, eta0, (double)i1 + (double)ox, (double)j1 + (double)oy, y[2]);
    if (A.phi) *p.at<float>(A.phi) += (float)y[2];
    if (xi1 < 0.0 || xi1 >= (double)A.nr) {
        ev.out = 1;
    } else {
        out.kind = 2;
        out.cell = i1 * A.nth + j1;
        out.x[0] = ox;
        out.x[1] = oy;
        out.x[2] = (float)y[3];
        out.x[3] = (float)u1t;
        out.x[4] = (float)uph1;
    }
    return true;
}

template <bool SPLIT>
using Elem = typename std::conditional<SPLIT, float, double>::type;

// SHORT: the short Taylor series, for grids fine enough for them
// (small_steps == 2); the launch picks the kernel variant.
// KICK: the momentum kick (kBoris, or kVay for the FP64 path only).
// ORDER: the shape, 1 (CIC) or 3 (cubic spline, FP64 only).  QED: the
// monopole step's kernels (the charge is read at the end there).
template <bool SPLIT, bool SHORT, int KICK, int ORDER = 1, bool QED = false>
__device__ __forceinline__ bool advance(const StepArgs& A, const PIdx& p, const ParticleIn<Elem<SPLIT>>& in, Move& mv,
                                        Events& ev, const TileAnchors* T, ParticleOut<Elem<SPLIT>>& out) {
    static_assert(!SPLIT || (KICK == kBoris && ORDER == 1), "the split form runs the Boris kick and CIC only");
    if constexpr (SPLIT) return advance_split<SHORT>(A, p, in, mv, ev, T, out);
    else return advance_f64<SHORT, KICK, ORDER, !QED>(A, p, in, mv, ev, T, out);
}

template <int ORDER = 1>
__device__ __forceinline__ void scatter_global(const StepArgs& A, const Move& mv) {
    double* const J[3] = {A.Fr, A.Fth, A.Gph};
    auto add = [&](int c, int i, int j, double v) { atomicAdd(elem(J[c], grid_index(A, i, j)), v); };
    if constexpr (ORDER == 3) esirkepov3(mv, A.idt, A.nth, add);
    else esirkepov(mv, A.idt, add);
}

// Event counts of a workgroup: each wave adds its ballot counts to five LDS
// words (cnt, zeroed before the first barrier); after a later barrier one
// thread adds the non-zero totals to the global counters, so the counters
// see one atomic per workgroup instead of one per wave.
__device__ __forceinline__ void wave_events_to_lds(const Events& ev, int* cnt) {
    const unsigned long long b[5] = {__ballot(ev.out), __ballot(ev.bad), __ballot(ev.refl), __ballot(ev.live),
                                     __ballot(ev.spill)};
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 5; ++k)
            if (b[k]) atomicAdd(cnt + k, __popcll(b[k]));
}

__device__ __forceinline__ void workgroup_events_to_global(const StepArgs& A, const int* cnt) {
    if (threadIdx.x == 0)
        for (int k = 0; k < 5; ++k)
            if (cnt[k]) atomicAdd(A.counters + k, (unsigned long long)cnt[k]);
}

template <bool SPLIT, bool SHORT, int KICK, int ORDER = 1>
__device__ __forceinline__ void push_deposit_body(const StepArgs& A) {
    __shared__ int cnt[5];
    if (threadIdx.x < 5) cnt[threadIdx.x] = 0;
    const PIdx pi{(int64_t)blockIdx.x * blockDim.x, threadIdx.x};
    const int64_t p = pi.base + pi.k;
    Events ev = {0, 0, 0, 0, 0};
    if (p < A.n) {
        Move mv;
        ParticleOut<Elem<SPLIT>> out;
        const bool dep =
            advance<SPLIT, SHORT, KICK, ORDER>(A, pi, load_particle<Elem<SPLIT>>(A, pi), mv, ev, nullptr, out);
        store_particle(A, pi, out);
        if (dep && mv.qw != 0.0) scatter_global<ORDER>(A, mv);   // an uncharged move adds only zeros
    }
    if (!A.counters) return;                                 // uniform
    __syncthreads();
    wave_events_to_lds(ev, cnt);
    __syncthreads();
    workgroup_events_to_global(A, cnt);
}

template <bool SHORT, int KICK, int ORDER>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void push_deposit_f64(const StepArgs A) {
    push_deposit_body<false, SHORT, KICK, ORDER>(A);
}
// The cubic shape's kernel (96 gather loads, a 5 x 5 deposit), at three
// waves per SIMD like the CIC kernel (its gather loads one component at a
// time).
template <bool SHORT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void push_deposit_f64_spline3(const StepArgs A) {
    push_deposit_body<false, SHORT, kBoris, 3>(A);
}
template <bool SHORT>
__global__ __launch_bounds__(256) void push_deposit_split(const StepArgs A) {
    push_deposit_body<true, SHORT, kBoris>(A);
}

// QED: photon emission and pair conversion after the push (FP64, Boris,
// CIC), with the created particles appended after the elements in use.
template <int THREADS, bool SPLIT, bool SHORT, int KICK, int ORDER = 1, bool QED = false>
__device__ __forceinline__ void push_deposit_tiled_body(const StepArgs& A, const Slice* __restrict__ slices,
                                                        int64_t slice_cap,
                                                        int32_t* __restrict__ slice_live,
                                                        const double* __restrict__ anchors,
                                                        const QedArgs& Q = QedArgs{}) {
    __shared__ double win[3][kWinRows][kWinCols];
    __shared__ TileAnchors tab;
    __shared__ int cnt[5];
    __shared__ int touched[4];                           // lowest, highest window row; lowest, highest column
    __shared__ unsigned q_total, q_ev[2];                // QED, staged: the slice's created particles, events
    // the slice's new particle states, by slot (one pad element per 32 keeps
    // the permuted lanes' writes on distinct banks): written back in slot
    // order after the deposit, so that consecutive lanes store consecutive
    // particles (the loads stay in the pushing lanes: staging them too would
    // make each wave wait for its loads before the first barrier)
    constexpr int kStage = THREADS + THREADS / 32;
    __shared__ int st_cell[kStage];                       // new cell; -1: removed; -2: nothing to store
    __shared__ Elem<SPLIT> st_x[5][kStage];
    // the slice table is in dispatch order (XCD-aware bands, written so by
    // the sort): one load finds this workgroup's slice
    const int64_t logical = blockIdx.x;
    if (logical >= slice_cap) return;
    const Slice sl = slices[logical];
    if (sl.start < 0 || sl.len <= 0) {
        if (A.counters && threadIdx.x == 0) slice_live[logical] = 0;
        if constexpr (QED) {
            if (Q.staged && threadIdx.x == 0) {
                Q.st.count[logical] = 0;
                Q.st.ev[logical] = 0;
                Q.st.ev[Q.slices + logical] = 0;
            }
        }
        return;
    }
    const int tpr = (A.nth + kTileCells - 1) / kTileCells;
    const int ti = div_by(sl.tile, tpr, A.inv_tpr);
    const int j_lo = (sl.tile - ti * tpr) * kTileCells;
    const int wi0 = ti - kMarginRows - 1;                // window origin (vertex indices)
    const int wj0 = j_lo - kMarginCols - 1;
    // one particle per thread; with S = ceil(len / 8), thread t < 8 S pushes
    // particle (t % 8) S + t / 8 of the slice (a bijection of [0, 8 S)), so a
    // wave's 64 lanes cover 8 runs of 8 particles spread over the slice's
    // cells and their LDS atomics rarely hit one address, and the threads of
    // a short slice's particles are the first ones (the waves after them skip
    // the push).  Its state is loaded before the LDS set-up and the barrier
    // (which waits for LDS accesses only), so the loads overlap them.
    const int t = threadIdx.x;
    const int run = (sl.len + kLaneGroups - 1) / kLaneGroups;
    const int slot = (t % kLaneGroups) * run + t / kLaneGroups;
    const PIdx pi{sl.start, (uint32_t)slot};
    const int64_t p = sl.start + slot;
    const bool mine = t / kLaneGroups < run && slot < sl.len && p < A.n;
    ParticleIn<Elem<SPLIT>> in;
    if (mine) in = load_particle<Elem<SPLIT>>(A, pi);

    double2* wflat = reinterpret_cast<double2*>(&win[0][0][0]);
    static_assert((3 * kWinRows * kWinCols) % 2 == 0, "the window is cleared in pairs");
    for (int e = threadIdx.x; e < 3 * kWinRows * kWinCols / 2; e += THREADS) wflat[e] = make_double2(0.0, 0.0);
    if (threadIdx.x < 5) cnt[threadIdx.x] = 0;
    if constexpr (QED) {
        if (threadIdx.x == 0) {
            q_total = 0;
            q_ev[0] = q_ev[1] = 0;
        }
    }
    if (threadIdx.x == 0) {
        touched[0] = kWinRows;
        touched[1] = -1;
        touched[2] = kWinCols;
        touched[3] = -1;
    }
    if (A.small_steps) {
        // table entry of row i is anchors[i + kMarginRows], of column j
        // S[j + kMarginCols] and C[j + kMarginCols]
        const double* S = anchors + (A.nr + 2 * kMarginRows);
        const double* C = S + (tpr * kTileCells + 2 * kMarginCols + 1);
        const int t0 = threadIdx.x;
        if (t0 == 0) {
            tab.i_lo = ti - kMarginRows;
            tab.j_lo = j_lo - kMarginCols;
        }
        if (t0 < kAnchorRows) tab.r[t0] = anchors[ti + t0];
        const int k = t0 - 64;                                // columns: from the second wave on
        if (k >= 0 && k < kAnchorCols) {
            tab.s[k] = S[j_lo + k];
            tab.c[k] = C[j_lo + k];
        }
    }
    __syncthreads();

    Events ev = {0, 0, 0, 0, 0};
    int row_lo = kWinRows, row_hi = -1;                  // window rows and columns this lane deposited on
    int col_lo = kWinCols, col_hi = -1;
    Created cr;
    QedEvents qe = {0, 0};
    cr.n = 0;
    if (mine) {
        Move mv;
        ParticleOut<Elem<SPLIT>> out;
        const bool dep = advance<SPLIT, SHORT, KICK, ORDER, QED>(A, pi, in, mv, ev, &tab, out);
        if constexpr (QED) qed_after_step(A, Q, in.s, *pi.at(Q.tag), *pi.at<double>(A.w), out, cr, qe);
        const int si = slot + slot / 32;
        st_cell[si] = out.kind == 2 ? out.cell : out.kind - 2;
        for (int k = 0; k < 5; ++k) st_x[k][si] = out.x[k];
        if (dep && mv.qw != 0.0) {                           // an uncharged move (a photon) adds only zeros
            if constexpr (ORDER == 3) {
                // the cubic window: rows i3 .. i3 + 4, columns j3 .. j3 + 4
                // folded across the axes (vertex and face columns)
                const int i3 = (int)floor(fmin(mv.xi0, mv.xi1)) - 1, j3 = (int)floor(fmin(mv.eta0, mv.eta1)) - 1;
                int jlo = kWinCols + wj0, jhi = wj0 - 1;
                for (int b = 0; b < 5; ++b) {
                    double sg;
                    const int jv = fold_vertex(j3 + b, A.nth), jf = fold_face(j3 + b, A.nth, sg);
                    jlo = min(jlo, min(jv, jf));
                    jhi = max(jhi, max(jv, jf));
                }
                const int li = i3 - wi0, ljl = jlo - wj0, ljh = jhi - wj0;
                if (li >= 0 && li + 4 < kWinRows && ljl >= 0 && ljh < kWinCols) {
                    esirkepov3(mv, A.idt, A.nth,
                               [&](int c, int i, int j, double v) { atomicAdd(&win[c][i - wi0][j - wj0], v); });
                    row_lo = li;
                    row_hi = li + 4;
                    col_lo = ljl;
                    col_hi = ljh;
                } else {
                    scatter_global<3>(A, mv);            // drifted out of the window
                    ev.spill = 1;
                }
            } else {
                const int li = mv.i0 - wi0, lj = mv.j0 - wj0;
                if (li >= 0 && li + 2 < kWinRows && lj >= 0 && lj + 2 < kWinCols) {
                    esirkepov(mv, A.idt,
                              [&](int c, int i, int j, double v) { atomicAdd(&win[c][i - wi0][j - wj0], v); });
                    row_lo = li;
                    row_hi = li + 2;
                    col_lo = lj;
                    col_hi = lj + 2;
                } else {
                    scatter_global(A, mv);               // drifted out of the window
                    ev.spill = 1;
                }
            }
        }
    }
    row_lo = wave_reduce<false>(row_lo);                 // every lane of the wave is active here
    row_hi = wave_reduce<true>(row_hi);
    col_lo = wave_reduce<false>(col_lo);
    col_hi = wave_reduce<true>(col_hi);
    if constexpr (QED) {
        if (Q.staged) qed_stage(A, Q, logical, cr, qe, &q_total, q_ev);
        else qed_append<double>(A, Q, Q.n_used[0], cr, qe);
    }
    if ((threadIdx.x & 63) == 0 && row_hi >= 0) {
        atomicMin(&touched[0], row_lo);
        atomicMax(&touched[1], row_hi);
        atomicMin(&touched[2], col_lo);
        atomicMax(&touched[3], col_hi);
    }
    if (A.counters) wave_events_to_lds(ev, cnt);
    __syncthreads();
    // the new particle states, thread t storing slot t (before the flush, so
    // that the stores' latency overlaps it)
    if (t < sl.len && sl.start + t < A.n) {
        const int si = t + t / 32;
        ParticleOut<Elem<SPLIT>> o;
        const int sc = st_cell[si];
        o.kind = sc >= 0 ? 2 : sc + 2;
        o.cell = sc;
        for (int k = 0; k < 5; ++k) o.x[k] = st_x[k][si];
        store_particle(A, PIdx{sl.start, (uint32_t)t}, o);
    }
    // flush the window's non-zero entries that lie inside the grid arrays
    double* const J[3] = {A.Fr, A.Fth, A.Gph};
    const int rows_lo = -A.guard, rows_hi = A.nr + A.guard;             // inclusive vertex rows
    const int cols_lo = -A.guard, cols_hi = A.pitch - A.guard - 1;      // inclusive vertex columns
    // only the rectangle of rows and columns that received deposits (a
    // slice covers a few cells of its tile; empty when nothing was deposited)
    const bool any = touched[1] >= 0;                    // then all four bounds are set
    const int r0 = touched[0], nrow = any ? touched[1] - touched[0] + 1 : 0;
    const int c0 = touched[2], ncol = any ? touched[3] - touched[2] + 1 : 1;
    // rows to groups of 32 threads, columns to the threads of a group
    for (int rr = threadIdx.x >> 5; rr < nrow; rr += THREADS >> 5) {
        for (int cc = threadIdx.x & 31; cc < ncol; cc += 32) {
            const int r = r0 + rr, c = c0 + cc;
            const int gi = wi0 + r, gj = wj0 + c;
            if (gi < rows_lo || gi > rows_hi || gj < cols_lo || gj > cols_hi) continue;
            const uint32_t g = grid_index(A, gi, gj);
            for (int a = 0; a < 3; ++a) {
                const double v = win[a][r][c];
                if (v != 0.0) atomicAdd(elem(J[a], g), v);
            }
        }
    }
    if (A.counters && threadIdx.x == 0) {
        // the live count goes to the slice's own word (summed by slice_live_sum);
        // the rare events take one atomic each when non-zero
        slice_live[logical] = cnt[3];
        for (int k = 0; k < 5; ++k)
            if (k != 3 && cnt[k]) atomicAdd(A.counters + k, (unsigned long long)cnt[k]);
    }
    if constexpr (QED) {
        // the slice's staged count and events, final after the barrier above
        if (Q.staged && threadIdx.x == 0) {
            Q.st.count[logical] = min(q_total, (unsigned)kQedStage);
            Q.st.ev[logical] = q_ev[0];
            Q.st.ev[Q.slices + logical] = q_ev[1];
        }
    }
}

// counters[LIVE] += sum of the per-slice live counts of one tiled push.
__global__ __launch_bounds__(256) void slice_live_sum(const int32_t* __restrict__ live, int64_t slice_cap,
                                                      unsigned long long* __restrict__ counters) {
    const int64_t n = slice_cap;                         // every entry is written by the push
    unsigned long long v = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v += (unsigned long long)live[i];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __shared__ unsigned long long part[4];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = part[0] + part[1] + part[2] + part[3];
        if (t) atomicAdd(counters + 3, t);
    }
}

// THREADS: the tiling's slice size (kSliceThreads).  With the short series
// the CIC kernels run at four waves per SIMD (at most 128 VGPRs; four
// workgroups' LDS fit a CU); the long series needs more registers and runs
// at three.
template <int THREADS, bool SHORT, int KICK>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(SHORT ? 4 : 3))) void push_deposit_f64_tiled(
    const StepArgs A, const Slice* __restrict__ slices, int64_t slice_cap,
    int32_t* slice_live, const double* anchors) {
    push_deposit_tiled_body<THREADS, false, SHORT, KICK>(A, slices, slice_cap, slice_live, anchors);
}
// The cubic shape's tiled kernel, at three or more waves per SIMD.
template <int THREADS, bool SHORT>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(3))) void push_deposit_f64_tiled_spline3(
    const StepArgs A, const Slice* __restrict__ slices, int64_t slice_cap, int32_t* slice_live,
    const double* anchors) {
    push_deposit_tiled_body<THREADS, false, SHORT, kBoris, 3>(A, slices, slice_cap, slice_live, anchors);
}
template <int THREADS, bool SHORT>
__global__ __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(SHORT ? 4 : 3))) void push_deposit_f64_tiled_qed(
    const StepArgs A, const Slice* __restrict__ slices, int64_t slice_cap, int32_t* slice_live,
    const double* anchors, const QedArgs Q) {
    push_deposit_tiled_body<THREADS, false, SHORT, kBoris, 1, true>(A, slices, slice_cap, slice_live, anchors, Q);
}

// The QED step of one block of particles b .. b + 255 below `end`: one
// particle per thread, global atomics.
template <bool SHORT>
__device__ __forceinline__ void qed_block(const StepArgs& A, const QedArgs& Q, int64_t b, int64_t end, int* cnt) {
    if (threadIdx.x < 5) cnt[threadIdx.x] = 0;
    const PIdx pi{b, threadIdx.x};
    Events ev = {0, 0, 0, 0, 0};
    Created cr;
    QedEvents qe = {0, 0};
    cr.n = 0;
    if (b + threadIdx.x < end) {
        Move mv;
        ParticleOut<double> out;
        const ParticleIn<double> in = load_particle<double>(A, pi);
        const bool dep = advance<false, SHORT, kBoris, 1, true>(A, pi, in, mv, ev, nullptr, out);
        qed_after_step(A, Q, in.s, *pi.at(Q.tag), *pi.at<double>(A.w), out, cr, qe);
        store_particle(A, pi, out);
        if (dep && mv.qw != 0.0) scatter_global(A, mv);
    }
    qed_append<double>(A, Q, end, cr, qe);
    if (A.counters) {                                       // uniform
        __syncthreads();
        wave_events_to_lds(ev, cnt);
        __syncthreads();
        workgroup_events_to_global(A, cnt);
    }
}

// Without a tiling: block b takes particles 256 b .. 256 b + 255 of those in
// use (the grid covers the capacity; blocks beyond the elements in use
// return at once).
template <bool SHORT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void push_deposit_f64_qed(
    const StepArgs A, const QedArgs Q) {
    __shared__ int cnt[5];
    const int64_t end = Q.n_used[0];
    const int64_t b = (int64_t)blockIdx.x * blockDim.x;
    if (b >= end) return;
    qed_block<SHORT>(A, Q, b, end, cnt);
}

// With a tiling: the particles appended since the sort, [n_sorted,
// n_used[0]), which no slice covers; a few blocks loop over them (a short
// range, so the loop's register spills cost little).
template <bool SHORT>
__global__ __launch_bounds__(256) void push_deposit_f64_qed_tail(const StepArgs A, const QedArgs Q) {
    __shared__ int cnt[5];
    const int64_t end = Q.n_used[0];
    const int64_t start = min(*Q.tail_start, end);
    for (int64_t b = start + (int64_t)blockIdx.x * blockDim.x; b < end; b += (int64_t)gridDim.x * blockDim.x) {
        qed_block<SHORT>(A, Q, b, end, cnt);
        __syncthreads();                                    // cnt is cleared again next pass
    }
}

// Before a QED step: the elements in use cover the tiling's sorted
// particles, the append counter starts at zero, and so does the staged
// counts' scan sentinel.
__global__ void qed_begin(int64_t* n_used, const int64_t* tail_start, int64_t cap, unsigned long long* sentinel) {
    int64_t n0 = n_used[0];
    if (tail_start && *tail_start > n0) n0 = *tail_start;
    n_used[0] = n0 < 0 ? 0 : (n0 > cap ? cap : n0);
    n_used[1] = 0;
    if (sentinel) *sentinel = 0ull;
}
// After it: the appended and the placed staged particles join the elements
// in use (staged_total: the scan's total, NULL without staging).
__global__ void qed_end(int64_t* n_used, int64_t cap, const unsigned long long* staged_total) {
    const int64_t n = n_used[0] + n_used[1] + (staged_total ? (int64_t)*staged_total : 0);
    n_used[0] = n > cap ? cap : n;
    n_used[1] = 0;
}

// Staged path: particle k of slice s goes to the elements after those in
// use and those appended directly, at the slice's scanned offset (so in
// slice order); those beyond the capacity are dropped.
__global__ __launch_bounds__(256) void qed_place(const StepArgs A, const QedArgs Q) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t s = t / kQedStage;
    const int k = (int)(t - s * kQedStage);
    if (s >= Q.slices) return;
    const unsigned long long o0 = Q.st.count[s], o1 = Q.st.count[s + 1];
    if ((unsigned long long)k >= o1 - o0) return;
    const int64_t q = Q.n_used[0] + Q.n_used[1] + (int64_t)(o0 + (unsigned long long)k);
    if (q >= Q.cap) {
        if (Q.qcounters) atomicAdd(Q.qcounters + 2, 1ull);
        return;
    }
    const int64_t e = s * kQedStage + k;
    A.cell[q] = Q.st.cell[e];
    static_cast<double*>(A.xr)[q] = Q.st.xr[e];
    static_cast<double*>(A.xth)[q] = Q.st.xth[e];
    static_cast<double*>(A.ur)[q] = Q.st.ur[e];
    static_cast<double*>(A.uth)[q] = Q.st.uth[e];
    static_cast<double*>(A.uph)[q] = Q.st.uph[e];
    static_cast<double*>(A.w)[q] = Q.st.w[e];
    const_cast<uint8_t*>(A.sp)[q] = Q.st.sp[e];
    Q.tag[q] = Q.st.tag[e];
    if (A.phi) static_cast<double*>(A.phi)[q] = 0.0;
}

// Staged path: the slices' event counts summed into the counters.
__global__ __launch_bounds__(256) void qed_event_sum(const unsigned* __restrict__ ev, int64_t slices,
                                                     unsigned long long* __restrict__ qcounters) {
    unsigned long long v[2] = {0, 0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < slices; i += (int64_t)gridDim.x * blockDim.x) {
        v[0] += ev[i];
        v[1] += ev[slices + i];
    }
    __shared__ unsigned long long part[2][4];
    for (int c = 0; c < 2; ++c) {
        for (int off = 32; off > 0; off >>= 1) v[c] += __shfl_xor(v[c], off);
        if ((threadIdx.x & 63) == 0) part[c][threadIdx.x >> 6] = v[c];
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const unsigned long long t = part[threadIdx.x][0] + part[threadIdx.x][1] + part[threadIdx.x][2] +
                                     part[threadIdx.x][3];
        if (t) atomicAdd(qcounters + threadIdx.x, t);
    }
}

// Workspace of the staged path, each array 256-byte aligned:
// count (slices + 1) and scan block sums (u64), events (2 x u32 per slice),
// then the staging SoA (kQedStage entries per slice).
namespace {
inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }
struct QedLayout {
    size_t count, blocksums, ev, cell, real[6], sp, tag, total;
};
inline QedLayout qed_layout(int64_t slices) {
    QedLayout L;
    const size_t S = (size_t)slices * kQedStage;
    size_t o = 0;
    L.count = o; o += align256(8 * ((size_t)slices + 1));
    L.blocksums = o; o += align256(8 * ((size_t)sort_scan_blocks(slices + 1) + 1));
    L.ev = o; o += align256(4 * 2 * (size_t)slices);
    L.cell = o; o += align256(4 * S);
    for (int k = 0; k < 6; ++k) { L.real[k] = o; o += align256(8 * S); }
    L.sp = o; o += align256(S);
    L.tag = o; o += align256(8 * S);
    L.total = o;
    return L;
}
}  // namespace

size_t qed_workspace_bytes(int64_t slice_cap) { return qed_layout(slice_cap).total; }

template <int THREADS, bool SHORT>
__global__ __launch_bounds__(THREADS) void push_deposit_split_tiled(const StepArgs A, const Slice* __restrict__ slices,
                                                                    int64_t slice_cap, int32_t* slice_live,
                                                                    const double* anchors) {
    push_deposit_tiled_body<THREADS, true, SHORT, kBoris>(A, slices, slice_cap, slice_live, anchors);
}

// The anchor table of a tiling (layout in grpic_launch.hpp), from the same
// anchor_r / anchor_sc as the untiled kernels' anchors.
__global__ __launch_bounds__(256) void tile_anchor_table(const StepArgs A, double* __restrict__ anchors, int rows,
                                                         int cols) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < rows) anchors[t] = anchor_r(A, t - kMarginRows);
    if (t < cols) {
        double s, c;
        anchor_sc(A, t - kMarginCols, s, c);
        anchors[rows + t] = s;
        anchors[rows + cols + t] = c;
    }
}

hipError_t launch_anchor_table(double lnr0, double dlnr, double dth, int nr, int nth, double* anchors,
                               hipStream_t stream) {
    StepArgs A{};
    A.lnr0 = lnr0;
    A.dlnr = dlnr;
    A.dth = dth;
    A.nr = nr;
    A.nth = nth;
    const int rows = anchor_table_rows(nr), cols = anchor_table_cols(nth);
    hipLaunchKernelGGL(tile_anchor_table, dim3((unsigned)((std::max(rows, cols) + 255) / 256)), dim3(256), 0, stream,
                       A, anchors, rows, cols);
    return hipGetLastError();
}

// Q_ij += q w S_ij(x_p) over live particles (FP64 or split offsets).
template <class T>
__global__ __launch_bounds__(256) void charge_kernel(const StepArgs A, double* __restrict__ Q) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.n) return;
    const int cell = A.cell[p];
    const int s = A.sp[p];
    if (cell < 0 || cell >= A.nr * A.nth || s >= A.nsp) return;
    const double fx = (double)static_cast<const T*>(A.xr)[p];
    const double fy = (double)static_cast<const T*>(A.xth)[p];
    if (!(fx >= 0.0 && fx <= 1.0 && fy >= 0.0 && fy <= 1.0)) return;
    const double qw = A.q[s] * (double)static_cast<const T*>(A.w)[p];
    const int ci = cell / A.nth, cj = cell - ci * A.nth;
    double* q = Q + grid_index(A, ci, cj);
    atomicAdd(q, qw * (1.0 - fx) * (1.0 - fy));
    atomicAdd(q + A.pitch, qw * fx * (1.0 - fy));
    atomicAdd(q + 1, qw * (1.0 - fx) * fy);
    atomicAdd(q + A.pitch + 1, qw * fx * fy);
}

// Charge with the cubic shape, folded across the axes like the deposit.
template <class T>
__global__ __launch_bounds__(256) void charge3_kernel(const StepArgs A, double* __restrict__ Q) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.n) return;
    const int cell = A.cell[p];
    const int s = A.sp[p];
    if (cell < 0 || cell >= A.nr * A.nth || s >= A.nsp) return;
    const double fx = (double)static_cast<const T*>(A.xr)[p];
    const double fy = (double)static_cast<const T*>(A.xth)[p];
    if (!(fx >= 0.0 && fx <= 1.0 && fy >= 0.0 && fy <= 1.0)) return;
    const double qw = A.q[s] * (double)static_cast<const T*>(A.w)[p];
    const int ci = cell / A.nth, cj = cell - ci * A.nth;
    for (int a = -1; a <= 2; ++a) {
        const double wx = qw * shape3(fx - (double)a);
        for (int b = -1; b <= 2; ++b)
            atomicAdd(elem(Q, grid_index(A, ci + a, fold_vertex(cj + b, A.nth))), wx * shape3(fy - (double)b));
    }
}

static inline dim3 blocks_for(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_push_deposit(const StepArgs& A, bool split, hipStream_t stream, int kick, int order) {
    if (A.n <= 0) return hipSuccess;
    const bool sh = A.small_steps == 2;
    const dim3 g = blocks_for(A.n), b(256);
    if (order == 3) {                                    // FP64, Boris kick (checked by the caller)
        if (sh) hipLaunchKernelGGL(push_deposit_f64_spline3<true>, g, b, 0, stream, A);
        else hipLaunchKernelGGL(push_deposit_f64_spline3<false>, g, b, 0, stream, A);
        return hipGetLastError();
    }
    if (split && sh) hipLaunchKernelGGL(push_deposit_split<true>, g, b, 0, stream, A);
    else if (split) hipLaunchKernelGGL(push_deposit_split<false>, g, b, 0, stream, A);
    else if (kick == kVay && sh) hipLaunchKernelGGL((push_deposit_f64<true, kVay, 1>), g, b, 0, stream, A);
    else if (kick == kVay) hipLaunchKernelGGL((push_deposit_f64<false, kVay, 1>), g, b, 0, stream, A);
    else if (sh) hipLaunchKernelGGL((push_deposit_f64<true, kBoris, 1>), g, b, 0, stream, A);
    else hipLaunchKernelGGL((push_deposit_f64<false, kBoris, 1>), g, b, 0, stream, A);
    return hipGetLastError();
}

hipError_t launch_push_deposit_qed(const StepArgs& A, QedArgs Q, void* tiling, int64_t slice_cap, void* ws,
                                   hipStream_t stream) {
    const bool sh = A.small_steps == 2;
    Q.tail_start = nullptr;
    Q.staged = 0;
    if (tiling) {
        const TilingHeader* hdr = static_cast<const TilingHeader*>(tiling);
        Q.tail_start = &hdr->n_sorted;
        if (ws) {
            const QedLayout L = qed_layout(slice_cap);
            char* b = static_cast<char*>(ws);
            Q.staged = 1;
            Q.slices = slice_cap;
            Q.st.count = reinterpret_cast<unsigned long long*>(b + L.count);
            Q.st.blocksums = reinterpret_cast<unsigned long long*>(b + L.blocksums);
            Q.st.ev = reinterpret_cast<unsigned*>(b + L.ev);
            Q.st.cell = reinterpret_cast<int32_t*>(b + L.cell);
            double** real[6] = {&Q.st.xr, &Q.st.xth, &Q.st.ur, &Q.st.uth, &Q.st.uph, &Q.st.w};
            for (int k = 0; k < 6; ++k) *real[k] = reinterpret_cast<double*>(b + L.real[k]);
            Q.st.sp = reinterpret_cast<uint8_t*>(b + L.sp);
            Q.st.tag = reinterpret_cast<uint64_t*>(b + L.tag);
        }
    }
    hipLaunchKernelGGL(qed_begin, dim3(1), dim3(1), 0, stream, Q.n_used, Q.tail_start, Q.cap,
                       Q.staged ? Q.st.count + slice_cap : nullptr);
    if (tiling) {
        const TilingLayout L = tiling_layout(A.n, A.nr, A.nth);     // slice_cap == L.cap
        const Slice* slices = tiling_at<const Slice>(tiling, L.slices);
        int32_t* live = tiling_at<int32_t>(tiling, L.live);
        const double* anchors = tiling_at<const double>(tiling, L.anchors);   // written by the sort
        const dim3 g((unsigned)((slice_cap + 7) / 8 * 8));
        const dim3 b(kSliceThreads);
        if (sh) hipLaunchKernelGGL((push_deposit_f64_tiled_qed<kSliceThreads, true>), g, b, 0, stream, A, slices,
                                   slice_cap, live, anchors, Q);
        else hipLaunchKernelGGL((push_deposit_f64_tiled_qed<kSliceThreads, false>), g, b, 0, stream, A, slices,
                                slice_cap, live, anchors, Q);
        if (A.counters)
            hipLaunchKernelGGL(slice_live_sum, dim3(64), dim3(256), 0, stream, live, slice_cap, A.counters);
    }
    if (tiling) {                                        // the particles appended since the sort
        const dim3 g((unsigned)std::min<int64_t>((A.n + 255) / 256, 1024));
        if (sh) hipLaunchKernelGGL(push_deposit_f64_qed_tail<true>, g, dim3(256), 0, stream, A, Q);
        else hipLaunchKernelGGL(push_deposit_f64_qed_tail<false>, g, dim3(256), 0, stream, A, Q);
    } else {                                             // every element in use
        const dim3 g((unsigned)((A.n + 255) / 256));
        if (sh) hipLaunchKernelGGL(push_deposit_f64_qed<true>, g, dim3(256), 0, stream, A, Q);
        else hipLaunchKernelGGL(push_deposit_f64_qed<false>, g, dim3(256), 0, stream, A, Q);
    }
    if (Q.staged) {                                      // place the staged particles after all others
        scan_exclusive(Q.st.count, slice_cap + 1, Q.st.blocksums, stream);
        const int64_t threads = slice_cap * kQedStage;
        hipLaunchKernelGGL(qed_place, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, stream, A, Q);
        if (Q.qcounters)
            hipLaunchKernelGGL(qed_event_sum, dim3(64), dim3(256), 0, stream, Q.st.ev, slice_cap, Q.qcounters);
    }
    hipLaunchKernelGGL(qed_end, dim3(1), dim3(1), 0, stream, Q.n_used, Q.cap,
                       Q.staged ? Q.st.count + slice_cap : nullptr);
    return hipGetLastError();
}

// The tiled kernel for the launch's shape, precision, kick and order: the
// cubic shape runs the tiling's cubic cut, the CIC kernels the other one.
hipError_t launch_push_deposit_tiled(const StepArgs& A, bool split, void* tiling, hipStream_t stream, int kick,
                                     int order) {
    if (A.n <= 0) return hipSuccess;
    const TilingLayout L = tiling_layout(A.n, A.nr, A.nth);
    const double* anchors = tiling_at<const double>(tiling, L.anchors);   // written by the sort
    const bool sh = A.small_steps == 2;
    const bool cubic = order == 3;                       // FP64, Boris kick (checked by the caller)
    const int64_t cap = cubic ? L.cap3 : L.cap;
    const Slice* slices = tiling_at<const Slice>(tiling, cubic ? L.slices3 : L.slices);
    int32_t* live = tiling_at<int32_t>(tiling, cubic ? L.live3 : L.live);
    const dim3 g((unsigned)((cap + 7) / 8 * 8));
    if (cubic) {
        const dim3 b(kSliceThreads3);
        if (sh)
            hipLaunchKernelGGL((push_deposit_f64_tiled_spline3<kSliceThreads3, true>), g, b, 0, stream, A, slices, cap,
                               live, anchors);
        else
            hipLaunchKernelGGL((push_deposit_f64_tiled_spline3<kSliceThreads3, false>), g, b, 0, stream, A, slices,
                               cap, live, anchors);
    } else {
        const dim3 b(kSliceThreads);
        if (split && sh)
            hipLaunchKernelGGL((push_deposit_split_tiled<kSliceThreads, true>), g, b, 0, stream, A, slices, cap, live,
                               anchors);
        else if (split)
            hipLaunchKernelGGL((push_deposit_split_tiled<kSliceThreads, false>), g, b, 0, stream, A, slices, cap, live,
                               anchors);
        else if (kick == kVay && sh)
            hipLaunchKernelGGL((push_deposit_f64_tiled<kSliceThreads, true, kVay>), g, b, 0, stream, A, slices, cap,
                               live, anchors);
        else if (kick == kVay)
            hipLaunchKernelGGL((push_deposit_f64_tiled<kSliceThreads, false, kVay>), g, b, 0, stream, A, slices, cap,
                               live, anchors);
        else if (sh)
            hipLaunchKernelGGL((push_deposit_f64_tiled<kSliceThreads, true, kBoris>), g, b, 0, stream, A, slices, cap,
                               live, anchors);
        else
            hipLaunchKernelGGL((push_deposit_f64_tiled<kSliceThreads, false, kBoris>), g, b, 0, stream, A, slices, cap,
                               live, anchors);
    }
    if (A.counters)
        hipLaunchKernelGGL(slice_live_sum, dim3(256), dim3(256), 0, stream, live, cap, A.counters);
    return hipGetLastError();
}

hipError_t launch_charge(const StepArgs& A, bool split, double* Q, hipStream_t stream, int order) {
    if (A.n <= 0) return hipSuccess;
    if (order == 3 && split) hipLaunchKernelGGL(charge3_kernel<float>, blocks_for(A.n), dim3(256), 0, stream, A, Q);
    else if (order == 3) hipLaunchKernelGGL(charge3_kernel<double>, blocks_for(A.n), dim3(256), 0, stream, A, Q);
    else if (split) hipLaunchKernelGGL(charge_kernel<float>, blocks_for(A.n), dim3(256), 0, stream, A, Q);
    else hipLaunchKernelGGL(charge_kernel<double>, blocks_for(A.n), dim3(256), 0, stream, A, Q);
    return hipGetLastError();
}

}  // namespace grpic
