// fields.hip -- the field solver of Sec. 2.1 and App. B of arXiv:2503.04558:
// the integral form of the 3+1 Maxwell equations on the staggered Yee grid,
// advanced by a predictor and ncorr semi-implicit corrector passes.
//
// One evaluation of the circulations is one stencil kernel (HBM-bound, no
// matrix work), field_eval_kernel: a workgroup takes a tile of kTileR x
// kTileC grid points, forms the auxiliary fields E_i, H_i of eqs. auxE /
// auxH over the tile and a one-point halo in LDS -- metric coefficients
// first (evaluated on the fly from tabulated r and sin, cos theta), then
// averaged to the auxiliary field's location -- and then takes their
// circulations (eqs. D-update, B-update; the axis rows of D^r by eq.
// Dr-axis) and writes the predictor or corrector value of its points.
// Guard rows are refilled (zero gradient) and the axis values of D^ph, B^th
// set to zero by every pass; a damping layer scales the outer rows on the
// last pass, and the columns beyond the axes are refreshed after the step.
//
// Locations, array element (i, j) of each component (r_x = exp(lnr0 + x
// dlnr), theta_y = y dth): D^r, B^th, E_r, H_th at (i+1/2, j); D^th, B^r,
// E_th, H_r at (i, j+1/2); D^ph, E_ph at (i, j); B^ph, H_ph at (i+1/2, j+1/2).
// Areas and volumes are per unit phi (the deposit's flux-form currents are
// J^r A^D_r, J^th A^D_th, J^ph A^D_ph).
#include "grpic_device.hpp"
#include "grpic_fields.hpp"

#include <algorithm>

namespace grpic {
namespace {

constexpr int kTileR = 8, kTileC = 64;                  // grid points per workgroup (2 per thread)
constexpr int kAuxR = kTileR + 2, kAuxC = kTileC + 2;   // with a one-point halo

__device__ __forceinline__ double rad(const FieldArgs& F, double x) { return exp(F.lnr0 + x * F.dlnr); }

// sqrt(det gamma) of the Kerr-Schild 3-metric (App. A, M reinstated).
__device__ __forceinline__ double sqrt_gamma(double a, double M, double r, double th) {
    const double s = sin(th), c = cos(th);
    const double rho2 = r * r + a * a * c * c;
    return rho2 * fabs(s) * sqrt(1.0 + 2.0 * M * r / rho2);
}

struct Coef {
    double aGrr, aGrp, aGtt, aGpp, sgB;                 // alpha gamma_ij, sqrt(gamma) beta^r
};

// Coefficients at radius r and polar angle with sine s, cosine c, with
// alpha = 1/sqrt(1 + z), z = 2 M r / rho^2: alpha gamma_rr = sqrt(1 + z),
// alpha gamma_rph = -a sin^2 sqrt(1 + z), alpha gamma_thth = rho^2 alpha,
// alpha gamma_phph = alpha Sigma sin^2 / rho^2, sqrt(gamma) beta^r =
// rho^2 |sin| sqrt(1 + z) z / (1 + z) = 2 M r |sin| alpha.  One reciprocal
// and one reciprocal square root per point.
__device__ __forceinline__ Coef coef_at(double a, double M, double r, double s, double c) {
    const double s2 = s * s, a2 = a * a, r2 = r * r;
    const double rho2 = r2 + a2 * (c * c);
    const double irho2 = rcp(rho2);
    const double tMr = 2.0 * M * r;
    double sq, alpha;
    sqrt_rsqrt(1.0 + tMr * irho2, sq, alpha);
    const double ra2 = r2 + a2;
    const double Sigma = ra2 * ra2 - a2 * (ra2 - tMr) * s2;
    Coef k;
    k.aGrr = sq;
    k.aGrp = -a * s2 * sq;
    k.aGtt = alpha * rho2;
    k.aGpp = alpha * Sigma * s2 * irho2;
    k.sgB = tMr * fabs(s) * alpha;
    return k;
}

// At grid position (x, y) = (hx / 2, hy / 2), hx >= -4 (x = -2), hy >= 0.
__device__ __forceinline__ Coef coef_grid(const FieldArgs& F, int hx, int hy) {
    return coef_at(F.a, F.M, F.rad[hx + 4], F.sn[hy], F.sn[field_nang(F.nth) + hy]);
}

struct Quad {
    double x[10], w[10];
};

__device__ __forceinline__ double int_th(const FieldArgs& F, const Quad& Q, double r, double t0, double t1) {
    double s = 0.0;
    for (int k = 0; k < 10; ++k) s += Q.w[k] * sqrt_gamma(F.a, F.M, r, 0.5 * (t0 + t1) + 0.5 * (t1 - t0) * Q.x[k]);
    return 0.5 * (t1 - t0) * s;
}
__device__ __forceinline__ double int_r(const FieldArgs& F, const Quad& Q, double th, double r0, double r1) {
    double s = 0.0;
    for (int k = 0; k < 10; ++k) s += Q.w[k] * sqrt_gamma(F.a, F.M, 0.5 * (r0 + r1) + 0.5 * (r1 - r0) * Q.x[k], th);
    return 0.5 * (r1 - r0) * s;
}
__device__ __forceinline__ double int_rth(const FieldArgs& F, const Quad& Q, double r0, double r1, double t0,
                                          double t1) {
    double s = 0.0;
    for (int k = 0; k < 10; ++k) s += Q.w[k] * int_th(F, Q, 0.5 * (r0 + r1) + 0.5 * (r1 - r0) * Q.x[k], t0, t1);
    return 0.5 * (r1 - r0) * s;
}

__device__ __forceinline__ double inv_or_zero(double v) { return v != 0.0 ? 1.0 / v : 0.0; }

// Tables: inverse areas of the six components over the physical rows and
// columns (zero in the other rows -2, -1, nr + 1 that the table covers),
// radial edge lengths per row, radii and sin, cos at half-integer steps.
__global__ __launch_bounds__(256) void field_tables_kernel(FieldArgs F, Quad Q) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int ncol = F.nth + 1;
    if (t < field_nrad(F.nr)) F.rad[t] = rad(F, -2.0 + 0.5 * (double)t);
    if (t < field_nang(F.nth)) {
        F.sn[t] = sin(0.5 * (double)t * F.dth);
        F.sn[field_nang(F.nth) + t] = cos(0.5 * (double)t * F.dth);
    }
    if (t >= (int64_t)ncol * F.nrow) return;
    const int i = (int)(t / ncol) + kTableRowLo, j = (int)(t % ncol);
    const uint32_t e = F.at(i, j);
    const double th_j = j * F.dth, th_h = (j + 0.5) * F.dth;
    const double r_i = rad(F, i), r_h = rad(F, i + 0.5);
    auto clamp_th = [&](double y) { return fmin(fmax(y, 0.0), (double)F.nth) * F.dth; };
    double iADr = 0.0, iADt = 0.0, iADp = 0.0, iABr = 0.0, iABt = 0.0, iABp = 0.0;
    if (i >= 0 && i <= F.nr) {
        const double r_m = rad(F, i - 0.5), r_p = rad(F, i + 1.0);
        if (i < F.nr) iADr = inv_or_zero(int_th(F, Q, r_h, clamp_th(j - 0.5), clamp_th(j + 0.5)));
        if (j < F.nth) iADt = inv_or_zero(int_r(F, Q, th_h, r_m, r_h));
        if (j > 0 && j < F.nth) iADp = inv_or_zero(int_rth(F, Q, r_m, r_h, clamp_th(j - 0.5), clamp_th(j + 0.5)));
        if (j < F.nth) iABr = inv_or_zero(int_th(F, Q, r_i, th_j, (j + 1) * F.dth));
        if (i < F.nr && j > 0 && j < F.nth) iABt = inv_or_zero(int_r(F, Q, th_j, r_i, r_p));
        if (i < F.nr && j < F.nth) iABp = inv_or_zero(int_rth(F, Q, r_i, r_p, th_j, (j + 1) * F.dth));
    }
    double* T = F.tab;
    const size_t S = F.plane;
    T[kT_iADr * S + e] = iADr;
    T[kT_iADt * S + e] = iADt;
    T[kT_iADp * S + e] = iADp;
    T[kT_iABr * S + e] = iABr;
    T[kT_iABt * S + e] = iABt;
    T[kT_iABp * S + e] = iABp;
    if (j == 0) {                                       // radial edge lengths of row i
        F.drow[kDrPrimal * F.nrow + (i - kTableRowLo)] = rad(F, i + 1.0) - r_i;
        F.drow[kDrDual * F.nrow + (i - kTableRowLo)] = r_h - rad(F, i - 0.5);
    }
}

// Axis values of D^ph and B^th set to zero (every row), then (second
// launch) zero-gradient guard rows of the six components, all pitch
// columns: rows -guard .. -1 copy row 0, rows above the last physical one
// (nr for D^th, D^ph, B^r; nr - 1 for the components at i + 1/2) copy it.
__global__ __launch_bounds__(256) void field_axis_kernel(FieldArgs F, FieldPtrs X) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int rows = F.nr + 1 + 2 * F.guard;
    if (t >= (int64_t)rows * 2) return;
    const int i = (int)(t >> 1) - F.guard, j = (t & 1) ? F.nth : 0;
    X.c[2][F.at(i, j)] = 0.0;
    X.c[4][F.at(i, j)] = 0.0;
}

__global__ __launch_bounds__(256) void field_guard_rows_kernel(FieldArgs F, FieldPtrs X) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int nrows = 2 * F.guard + 1;                  // -guard .. -1, nr .. nr + guard
    if (t >= (int64_t)nrows * F.pitch) return;
    const int r = (int)(t / F.pitch), jj = (int)(t % F.pitch) - F.guard;
    const int i = r < F.guard ? r - F.guard : F.nr + (r - F.guard);
    for (int c = 0; c < 6; ++c) {
        const bool half = c == 0 || c == 4 || c == 5;
        const int last = half ? F.nr - 1 : F.nr;
        if (i >= 0 && i <= last) continue;              // row nr of D^th, D^ph, B^r is physical
        const int src = i < 0 ? 0 : last;
        X.c[c][F.at(i, jj)] = X.c[c][F.at(src, jj)];
    }
}

// Columns beyond the axes, which the particles' CIC gather reads within
// half a cell of an axis.  By axisymmetry (the extended chart's point
// (r, -theta, phi) is (r, theta, phi + pi), where only the theta basis
// vector is reversed) a component there is its value at the mirrored
// location, negated for D^th and B^th.  Mirror pairs: integer columns
// -m <-> m and nth + m <-> nth - m; columns at j + 1/2 (D^th, B^r, B^ph)
// -m <-> m - 1 and nth - 1 + m <-> nth - m; every row, m = 1 .. guard.
// Written columns and read columns are disjoint (nth > guard).
__global__ __launch_bounds__(256) void field_axis_ghosts_kernel(FieldArgs F, FieldPtrs X) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int rows = F.nr + 1 + 2 * F.guard;
    if (t >= (int64_t)rows * F.guard * 2) return;
    const bool far = (t & 1) != 0;
    const int m = (int)((t >> 1) % F.guard) + 1;
    const int i = (int)((t >> 1) / F.guard) - F.guard;
    for (int c = 0; c < 6; ++c) {
        const double p = (c == 1 || c == 4) ? -1.0 : 1.0;
        const bool half = c == 1 || c == 3 || c == 5;
        const int dst = far ? (half ? F.nth - 1 + m : F.nth + m) : -m;
        const int src = far ? F.nth - m : (half ? m - 1 : m);
        X.c[c][F.at(i, dst)] = p * X.c[c][F.at(i, src)];
    }
}

// The six auxiliary fields at grid point (i, j), -1 <= i <= nr, 0 <= j <=
// nth, from the state X (guard rows filled): o[0..2] = E_r, E_th, E_ph,
// o[3..5] = H_r, H_th, H_ph (E_th, H_r, H_ph only for j < nth, else 0).
__device__ __forceinline__ void aux_at(const FieldArgs& F, const FieldPtrs& X, int i, int j, double o[6]) {
    const uint32_t e = F.at(i, j), em = F.at(i - 1, j), ep = F.at(i + 1, j);
    const double *Dr = X.c[0], *Dt = X.c[1], *Dp = X.c[2], *Br = X.c[3], *Bt = X.c[4], *Bp = X.c[5];
    const int hx = 2 * i, hy = 2 * j;
    // coefficients at (i +- 1/2, j), (i, j), (i + 1, j)
    const Coef cRh = coef_grid(F, hx + 1, hy), cRm = coef_grid(F, hx - 1, hy);
    const Coef cP = coef_grid(F, hx, hy), cPp = coef_grid(F, hx + 2, hy);
    o[0] = cRh.aGrr * Dr[e] + 0.5 * (cP.aGrp * Dp[e] + cPp.aGrp * Dp[ep]);
    o[2] = cP.aGpp * Dp[e] + 0.5 * (cRh.aGrp * Dr[e] + cRm.aGrp * Dr[em]) +
           0.5 * (cRh.sgB * Bt[e] + cRm.sgB * Bt[em]);
    o[4] = cRh.aGtt * Bt[e] + 0.5 * (cP.sgB * Dp[e] + cPp.sgB * Dp[ep]);
    if (j < F.nth) {
        // coefficients at (i, j + 1/2), (i + 1, j + 1/2), (i +- 1/2, j + 1/2)
        const Coef cT = coef_grid(F, hx, hy + 1), cTp = coef_grid(F, hx + 2, hy + 1);
        const Coef cBh = coef_grid(F, hx + 1, hy + 1), cBm = coef_grid(F, hx - 1, hy + 1);
        o[1] = cT.aGtt * Dt[e] - 0.5 * (cBh.sgB * Bp[e] + cBm.sgB * Bp[em]);
        o[3] = cT.aGrr * Br[e] + 0.5 * (cBh.aGrp * Bp[e] + cBm.aGrp * Bp[em]);
        o[5] = cBh.aGpp * Bp[e] + 0.5 * (cT.aGrp * Br[e] + cTp.aGrp * Br[ep]) -
               0.5 * (cT.sgB * Dt[e] + cTp.sgB * Dt[ep]);
    } else {
        o[1] = o[3] = o[5] = 0.0;
    }
}

// One evaluation: the auxiliary fields of X over the tile and its halo in
// LDS, then for each point of the tile the circulations C and the pass's
// value of all six components.  The terms of a corrector that do not change
// between passes are formed once: FIRST (the predictor, X = x0) writes
// R = x0 + dt (w0 C - J) and the value x0 + dt (C - J); a corrector's value
// is R + dt w1 C.  Elements a component does not update take x0 (R holds
// it for the correctors; zero on the axes for D^ph, B^th); with L > 0 the
// values at radial position x >= nr - L are scaled by 1 - d ((x - nr + L) /
// L)^2 (the damping layer, on the step's last pass).  The zero-gradient
// guard rows of out are written from the rows they copy.  out must not
// alias X (other workgroups read X in their halo).
//
// Tile order: workgroup w runs on XCD w mod 8 (the dispatcher's round
// robin), so logical tile (w mod 8) per + w / 8 gives each XCD a contiguous
// band of tile rows in row-major order; the halo rows a tile shares with its
// neighbours are then read through the same L2.
template <bool FIRST>
__global__ __launch_bounds__(256) void field_eval_kernel(FieldArgs F, FieldPtrs X, FieldPtrs x0, FieldPtrs R,
                                                         FieldPtrs out, int L, double d, unsigned ntiles,
                                                         unsigned per_xcd) {
    __shared__ double aux[6][kAuxR][kAuxC];
    const unsigned tile = (blockIdx.x & 7u) * per_xcd + (blockIdx.x >> 3);
    if (tile >= ntiles) return;                          // whole workgroup: before any barrier
    const int tiles_c = (F.nth + kTileC) / kTileC;      // columns 0 .. nth
    const int i0 = (int)(tile / tiles_c) * kTileR, j0 = (int)(tile % tiles_c) * kTileC;
    for (int e = threadIdx.x; e < kAuxR * kAuxC; e += blockDim.x) {
        const int li = e / kAuxC, lj = e - li * kAuxC;
        const int i = i0 - 1 + li, j = j0 - 1 + lj;
        double o[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (i >= -1 && i <= F.nr && j >= 0 && j <= F.nth) aux_at(F, X, i, j, o);
        for (int c = 0; c < 6; ++c) aux[c][li][lj] = o[c];
    }
    __syncthreads();
    const double* T = F.tab;
    const size_t S = F.plane;
    for (int k = threadIdx.x; k < kTileR * kTileC; k += blockDim.x) {
        const int li = k / kTileC, lj = k - li * kTileC;
        const int i = i0 + li, j = j0 + lj;
        if (i > F.nr || j > F.nth) continue;
        const int a = li + 1, b = lj + 1;                // this point in the aux tile
        const uint32_t e = F.at(i, j);
        const double dr = F.drow[kDrPrimal * F.nrow + (i - kTableRowLo)];
        const double drd = F.drow[kDrDual * F.nrow + (i - kTableRowLo)];
        double f_i = 1.0, f_h = 1.0;                     // damping at x = i, i + 1/2
        if (L > 0) {
            const double x_in = (double)(F.nr - L);
            auto damp = [&](double x) {
                const double s = (x - x_in) / L;
                return x < x_in ? 1.0 : 1.0 - d * s * s;
            };
            f_i = damp((double)i);
            f_h = damp(i + 0.5);
        }
        auto put = [&](int c, double v) {
            const bool half = c == 0 || c == 4 || c == 5;
            const int last = half ? F.nr - 1 : F.nr;
            v *= half ? f_h : f_i;
            out.c[c][e] = v;
            if (i == 0)
                for (int g = 1; g <= F.guard; ++g) out.c[c][F.at(-g, j)] = v;
            if (i == last)
                for (int r = last + 1; r <= F.nr + F.guard; ++r) out.c[c][F.at(r, j)] = v;
        };
        auto next = [&](int c, double C, double J) {
            if (FIRST) {
                const double x = x0.c[c][e];
                R.c[c][e] = x + F.dt * (F.w0 * C - J);
                return x + F.dt * (C - J);
            }
            return R.c[c][e] + F.dt * F.w1 * C;
        };
        auto keep = [&](int c) {                         // an element the component does not update
            if (FIRST) {
                const double x = x0.c[c][e];
                R.c[c][e] = x;
                return x;
            }
            return R.c[c][e];
        };
        auto cur = [&](int c, int t) { return FIRST && F.J[c] ? F.J[c][e] * T[t * S + e] : 0.0; };
        const bool axis = j == 0 || j == F.nth;
        if (i < F.nr) {                                  // D^r at (i+1/2, j), axes included
            const double hp = j < F.nth ? aux[5][a][b] : 0.0, hm = j > 0 ? aux[5][a][b - 1] : 0.0;
            put(0, next(0, (hp - hm) * T[kT_iADr * S + e], cur(0, kT_iADr)));
        }
        // D^th at (i, j+1/2), B^r at (i, j+1/2)
        put(1, j < F.nth ? next(1, (aux[5][a - 1][b] - aux[5][a][b]) * T[kT_iADt * S + e], cur(1, kT_iADt))
                         : keep(1));
        put(3, j < F.nth ? next(3, -(aux[2][a][b + 1] - aux[2][a][b]) * T[kT_iABr * S + e], 0.0) : keep(3));
        // D^ph at (i, j), B^th at (i+1/2, j)
        put(2, axis ? 0.0
                    : next(2,
                           ((aux[4][a][b] - aux[4][a - 1][b]) * F.dth + (aux[3][a][b - 1] - aux[3][a][b]) * drd) *
                               T[kT_iADp * S + e],
                           cur(2, kT_iADp)));
        if (i < F.nr) {
            put(4, axis ? 0.0 : next(4, -(aux[2][a][b] - aux[2][a + 1][b]) * T[kT_iABt * S + e], 0.0));
            // B^ph at (i+1/2, j+1/2)
            put(5, j < F.nth ? next(5,
                                    -((aux[1][a + 1][b] - aux[1][a][b]) * F.dth +
                                      (aux[0][a][b] - aux[0][a][b + 1]) * dr) *
                                        T[kT_iABp * S + e],
                                    0.0)
                             : keep(5));
        }
    }
}

__global__ __launch_bounds__(256) void field_copy_kernel(FieldPtrs dst, FieldPtrs src, int64_t n) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    for (int c = 0; c < 6; ++c) dst.c[c][t] = src.c[c][t];
}

inline unsigned nb(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t launch_field_tables(const FieldArgs& F, const double* gx, const double* gw, hipStream_t stream) {
    Quad Q;
    for (int k = 0; k < 10; ++k) {
        Q.x[k] = gx[k];
        Q.w[k] = gw[k];
    }
    const int64_t n = std::max<int64_t>((int64_t)(F.nth + 1) * F.nrow,
                                        std::max(field_nrad(F.nr), field_nang(F.nth)));
    hipLaunchKernelGGL(field_tables_kernel, dim3(nb(n)), dim3(256), 0, stream, F, Q);
    return hipGetLastError();
}

// The step.  X's guard rows and axis values are set first; the predictor
// reads X (iterate and start state) and writes W1 and the corrector's
// constant part R; corrector passes alternate between W1 and W2 (a pass's
// workgroups read their neighbours' halo of the previous iterate) and the
// last writes X with the damping layer applied; then X's columns beyond the
// axes are refreshed.  With no corrector the predictor writes X from a copy
// of it in W2.
hipError_t launch_field_step(const FieldArgs& F, FieldPtrs X, FieldPtrs R, FieldPtrs W1, FieldPtrs W2, int ncorr,
                             int damp_cells, double damp_max, hipStream_t stream) {
    const int64_t n_all = (int64_t)(F.nr + 1 + 2 * F.guard) * F.pitch;
    const int64_t n_axis = (int64_t)(F.nr + 1 + 2 * F.guard) * 2, n_grow = (int64_t)(2 * F.guard + 1) * F.pitch;
    const int64_t n_ghost = (int64_t)(F.nr + 1 + 2 * F.guard) * F.guard * 2;
    const unsigned tiles = (unsigned)(((F.nr + kTileR) / kTileR) * ((F.nth + kTileC) / kTileC));
    const unsigned per = (tiles + 7) / 8;
    const dim3 grid(8 * per), block(256);
    hipLaunchKernelGGL(field_axis_kernel, dim3(nb(n_axis)), block, 0, stream, F, X);
    hipLaunchKernelGGL(field_guard_rows_kernel, dim3(nb(n_grow)), block, 0, stream, F, X);
    if (ncorr == 0) {
        hipLaunchKernelGGL(field_copy_kernel, dim3(nb(n_all)), block, 0, stream, W2, X, n_all);
        hipLaunchKernelGGL(field_eval_kernel<true>, grid, block, 0, stream, F, W2, W2, R, X, damp_cells, damp_max,
                           tiles, per);
        hipLaunchKernelGGL(field_axis_ghosts_kernel, dim3(nb(n_ghost)), block, 0, stream, F, X);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(field_eval_kernel<true>, grid, block, 0, stream, F, X, X, R, W1, 0, 0.0, tiles, per);
    for (int it = 0; it < ncorr; ++it) {
        const bool last = it == ncorr - 1;
        const FieldPtrs cur = it % 2 == 0 ? W1 : W2;
        const FieldPtrs nxt = last ? X : (it % 2 == 0 ? W2 : W1);
        hipLaunchKernelGGL(field_eval_kernel<false>, grid, block, 0, stream, F, cur, X, R, nxt,
                           last ? damp_cells : 0, damp_max, tiles, per);
    }
    hipLaunchKernelGGL(field_axis_ghosts_kernel, dim3(nb(n_ghost)), block, 0, stream, F, X);
    return hipGetLastError();
}

}  // namespace grpic
