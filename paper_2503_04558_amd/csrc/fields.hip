// fields.hip -- the field solver of Sec. 2.1 and App. B of arXiv:2503.04558:
// the integral form of the 3+1 Maxwell equations on the staggered Yee grid,
// advanced by a predictor and ncorr semi-implicit corrector passes.
//
// One evaluation of the circulations is two stencil kernels over the grid
// (HBM-bound, no matrix work): field_aux forms the auxiliary fields E_i, H_i
// of eqs. auxE / auxH (metric coefficients first, then averaged to the
// auxiliary field's location), field_update takes their circulations
// (eqs. D-update, B-update; the axis rows of D^r by eq. Dr-axis) and writes
// the predictor or corrector value.  Guard rows are refilled (zero
// gradient) and the axis values of D^ph, B^th set to zero after every pass;
// a damping layer scales the outer rows after the step.
//
// Locations, array element (i, j) of each component (r_x = exp(lnr0 + x
// dlnr), theta_y = y dth): D^r, B^th, E_r, H_th at (i+1/2, j); D^th, B^r,
// E_th, H_r at (i, j+1/2); D^ph, E_ph at (i, j); B^ph, H_ph at (i+1/2, j+1/2).
// Areas and volumes are per unit phi (the deposit's flux-form currents are
// J^r A^D_r, J^th A^D_th, J^ph A^D_ph).
#include "grpic_fields.hpp"

#include <algorithm>

namespace grpic {
namespace {

__device__ __forceinline__ double rad(const FieldArgs& F, double x) { return exp(F.lnr0 + x * F.dlnr); }

// sqrt(det gamma) of the Kerr-Schild 3-metric (App. A, M reinstated).
__device__ __forceinline__ double sqrt_gamma(double a, double M, double r, double th) {
    const double s = sin(th), c = cos(th);
    const double rho2 = r * r + a * a * c * c;
    return rho2 * fabs(s) * sqrt(1.0 + 2.0 * M * r / rho2);
}

struct Coef {
    double aGrr, aGrp, aGtt, aGpp, sgB;       // alpha gamma_ij, sqrt(gamma) beta^r
};

__device__ __forceinline__ Coef coef_at(double a, double M, double r, double th) {
    const double s = sin(th), c = cos(th), s2 = s * s;
    const double rho2 = r * r + a * a * c * c;
    const double z = 2.0 * M * r / rho2;
    const double opz = 1.0 + z;
    const double alpha = 1.0 / sqrt(opz);
    const double Delta = r * r + a * a - 2.0 * M * r;
    const double Sigma = (r * r + a * a) * (r * r + a * a) - a * a * Delta * s2;
    Coef k;
    k.aGrr = alpha * opz;
    k.aGrp = -alpha * a * s2 * opz;
    k.aGtt = alpha * rho2;
    k.aGpp = alpha * Sigma * s2 / rho2;
    k.sgB = rho2 * fabs(s) * sqrt(opz) * (z / opz);
    return k;
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

// Tables: coefficients at the six locations and inverse areas, for the
// physical rows and columns (0 .. nr, 0 .. nth) and the guard rows -2, -1
// and nr + 1 that the auxiliary fields of rows -1 and nr reach.
__global__ __launch_bounds__(256) void field_tables_kernel(FieldArgs F, Quad Q) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int ncol = F.nth + 1;
    if (t >= (int64_t)ncol * F.nrow) return;
    const int i = (int)(t / ncol) + kTableRowLo, j = (int)(t % ncol);
    const uint32_t e = F.at(i, j);
    const double th_j = j * F.dth, th_h = (j + 0.5) * F.dth;
    const double r_i = rad(F, i), r_h = rad(F, i + 0.5);
    auto clamp_th = [&](double y) { return fmin(fmax(y, 0.0), (double)F.nth) * F.dth; };
    // coefficients: D^r and B^th at (i+1/2, j), D^th and B^r at (i, j+1/2),
    // D^ph at (i, j), B^ph at (i+1/2, j+1/2)
    const Coef cDr = coef_at(F.a, F.M, r_h, th_j), cDt = coef_at(F.a, F.M, r_i, th_h);
    const Coef cDp = coef_at(F.a, F.M, r_i, th_j), cBp = coef_at(F.a, F.M, r_h, th_h);
    double* T = F.tab;
    const size_t S = F.plane;
    T[kT_Dr_aGrr * S + e] = cDr.aGrr;
    T[kT_Dr_aGrp * S + e] = cDr.aGrp;
    T[kT_Dr_sgB * S + e] = cDr.sgB;                // B^th shares the location
    T[kT_Dr_aGtt * S + e] = cDr.aGtt;
    T[kT_Dt_aGtt * S + e] = cDt.aGtt;
    T[kT_Dt_sgB * S + e] = cDt.sgB;
    T[kT_Dt_aGrr * S + e] = cDt.aGrr;              // B^r shares the location
    T[kT_Dt_aGrp * S + e] = cDt.aGrp;
    T[kT_Dp_aGpp * S + e] = cDp.aGpp;
    T[kT_Dp_aGrp * S + e] = cDp.aGrp;
    T[kT_Dp_sgB * S + e] = cDp.sgB;
    T[kT_Bp_aGpp * S + e] = cBp.aGpp;
    T[kT_Bp_aGrp * S + e] = cBp.aGrp;
    T[kT_Bp_sgB * S + e] = cBp.sgB;
    // inverse areas (per unit phi), zero where a component is not updated
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
    T[kT_iADr * S + e] = iADr;
    T[kT_iADt * S + e] = iADt;
    T[kT_iADp * S + e] = iADp;
    T[kT_iABr * S + e] = iABr;
    T[kT_iABt * S + e] = iABt;
    T[kT_iABp * S + e] = iABp;
    if (j == 0) {                                   // radial edge lengths of row i
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
    const int nrows = 2 * F.guard + 1;                 // -guard .. -1, nr .. nr + guard
    if (t >= (int64_t)nrows * F.pitch) return;
    const int r = (int)(t / F.pitch), jj = (int)(t % F.pitch) - F.guard;
    const int i = r < F.guard ? r - F.guard : F.nr + (r - F.guard);
    for (int c = 0; c < 6; ++c) {
        const bool half = c == 0 || c == 4 || c == 5;
        const int last = half ? F.nr - 1 : F.nr;
        if (i >= 0 && i <= last) continue;             // row nr of D^th, D^ph, B^r is physical
        const int src = i < 0 ? 0 : last;
        X.c[c][F.at(i, jj)] = X.c[c][F.at(src, jj)];
    }
}

// Auxiliary fields of the state X (eqs. auxE, auxH) over rows -1 .. nr and
// columns 0 .. nth: aux.c[0..2] = E_r, E_th, E_ph; aux.c[3..5] = H_r, H_th, H_ph.
__global__ __launch_bounds__(256) void field_aux_kernel(FieldArgs F, FieldPtrs X, FieldPtrs aux) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int ncol = F.nth + 1;
    if (t >= (int64_t)ncol * (F.nr + 2)) return;
    const int i = (int)(t / ncol) - 1, j = (int)(t % ncol);
    const uint32_t e = F.at(i, j), em = F.at(i - 1, j), ep = F.at(i + 1, j);
    const double* T = F.tab;
    const size_t S = F.plane;
    const double *Dr = X.c[0], *Dt = X.c[1], *Dp = X.c[2], *Br = X.c[3], *Bt = X.c[4], *Bp = X.c[5];
    auto tb = [&](int k, uint32_t x) { return T[k * S + x]; };
    // E_r at (i+1/2, j)
    aux.c[0][e] = tb(kT_Dr_aGrr, e) * Dr[e] + 0.5 * (tb(kT_Dp_aGrp, e) * Dp[e] + tb(kT_Dp_aGrp, ep) * Dp[ep]);
    // E_ph at (i, j)
    aux.c[2][e] = tb(kT_Dp_aGpp, e) * Dp[e] + 0.5 * (tb(kT_Dr_aGrp, e) * Dr[e] + tb(kT_Dr_aGrp, em) * Dr[em]) +
                  0.5 * (tb(kT_Dr_sgB, e) * Bt[e] + tb(kT_Dr_sgB, em) * Bt[em]);
    // H_th at (i+1/2, j)
    aux.c[4][e] = tb(kT_Dr_aGtt, e) * Bt[e] + 0.5 * (tb(kT_Dp_sgB, e) * Dp[e] + tb(kT_Dp_sgB, ep) * Dp[ep]);
    if (j < F.nth) {
        // E_th at (i, j+1/2)
        aux.c[1][e] = tb(kT_Dt_aGtt, e) * Dt[e] - 0.5 * (tb(kT_Bp_sgB, e) * Bp[e] + tb(kT_Bp_sgB, em) * Bp[em]);
        // H_r at (i, j+1/2)
        aux.c[3][e] = tb(kT_Dt_aGrr, e) * Br[e] + 0.5 * (tb(kT_Bp_aGrp, e) * Bp[e] + tb(kT_Bp_aGrp, em) * Bp[em]);
        // H_ph at (i+1/2, j+1/2)
        aux.c[5][e] = tb(kT_Bp_aGpp, e) * Bp[e] + 0.5 * (tb(kT_Dt_aGrp, e) * Br[e] + tb(kT_Dt_aGrp, ep) * Br[ep]) -
                      0.5 * (tb(kT_Dt_sgB, e) * Dt[e] + tb(kT_Dt_sgB, ep) * Dt[ep]);
    }
}

// Circulations of the auxiliary fields and the pass's update, rows 0 .. nr,
// columns 0 .. nth.  first: C0 <- C and out = x0 + dt (C - J); else
// out = x0 + dt (w0 C0 + w1 C) - dt J.  Elements a component does not
// update are left alone.
__global__ __launch_bounds__(256) void field_update_kernel(FieldArgs F, FieldPtrs aux, FieldPtrs x0, FieldPtrs C0,
                                                           FieldPtrs out, int first) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int ncol = F.nth + 1;
    if (t >= (int64_t)ncol * (F.nr + 1)) return;
    const int i = (int)(t / ncol), j = (int)(t % ncol);
    const uint32_t e = F.at(i, j), em = F.at(i - 1, j), ep = F.at(i + 1, j);
    const uint32_t ejm = F.at(i, j - 1), ejp = F.at(i, j + 1);
    const double* T = F.tab;
    const size_t S = F.plane;
    const double *Er = aux.c[0], *Et = aux.c[1], *Ep = aux.c[2], *Hr = aux.c[3], *Ht = aux.c[4], *Hp = aux.c[5];
    const double dth = F.dth;
    const double dr = F.drow[kDrPrimal * F.nrow + (i - kTableRowLo)];
    const double drd = F.drow[kDrDual * F.nrow + (i - kTableRowLo)];
    auto apply = [&](int c, double C, double J) {
        if (first) {
            C0.c[c][e] = C;
            out.c[c][e] = x0.c[c][e] + F.dt * (C - J);
        } else {
            out.c[c][e] = x0.c[c][e] + F.dt * (F.w0 * C0.c[c][e] + F.w1 * C) - F.dt * J;
        }
    };
    auto cur = [&](int c, int k) { return F.J[c] ? F.J[c][e] * T[k * S + e] : 0.0; };
    if (i < F.nr) {                                       // D^r at (i+1/2, j), axes included
        const double hp = j < F.nth ? Hp[e] : 0.0, hm = j > 0 ? Hp[ejm] : 0.0;
        apply(0, (hp - hm) * T[kT_iADr * S + e], cur(0, kT_iADr));
    }
    if (j < F.nth) {                                      // D^th at (i, j+1/2)
        apply(1, (Hp[em] - Hp[e]) * T[kT_iADt * S + e], cur(1, kT_iADt));
        apply(3, -(Ep[ejp] - Ep[e]) * T[kT_iABr * S + e], 0.0);   // B^r at (i, j+1/2)
    }
    if (j > 0 && j < F.nth) {                             // D^ph at (i, j)
        apply(2, ((Ht[e] - Ht[em]) * dth + (Hr[ejm] - Hr[e]) * drd) * T[kT_iADp * S + e], cur(2, kT_iADp));
        if (i < F.nr) apply(4, -(Ep[e] - Ep[ep]) * T[kT_iABt * S + e], 0.0);   // B^th at (i+1/2, j)
    }
    if (i < F.nr && j < F.nth)                            // B^ph at (i+1/2, j+1/2)
        apply(5, -((Et[ep] - Et[e]) * dth + (Er[e] - Er[ejp]) * dr) * T[kT_iABp * S + e], 0.0);
}

// Damping layer: component values at radial position x >= nr - L scaled
// by 1 - d ((x - nr + L) / L)^2.
__global__ __launch_bounds__(256) void field_damp_kernel(FieldArgs F, FieldPtrs X, int L, double d) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int ncol = F.nth + 1;
    if (t >= (int64_t)ncol * (L + 1)) return;
    const int i = F.nr - L + (int)(t / ncol), j = (int)(t % ncol);
    if (i < 0) return;
    const double x_in = (double)(F.nr - L);
    for (int c = 0; c < 6; ++c) {
        const bool half = c == 0 || c == 4 || c == 5;
        if (half && i >= F.nr) continue;
        const double x = i + (half ? 0.5 : 0.0);
        if (x < x_in) continue;
        const double s = (x - x_in) / L;
        X.c[c][F.at(i, j)] *= 1.0 - d * s * s;
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
    hipLaunchKernelGGL(field_tables_kernel, dim3(nb((int64_t)(F.nth + 1) * F.nrow)), dim3(256), 0, stream, F, Q);
    return hipGetLastError();
}

hipError_t launch_field_step(const FieldArgs& F, FieldPtrs X, FieldPtrs x0, FieldPtrs C0, FieldPtrs aux, int ncorr,
                             int damp_cells, double damp_max, hipStream_t stream) {
    const int64_t n_all = (int64_t)(F.nr + 1 + 2 * F.guard) * F.pitch;
    const int64_t n_aux = (int64_t)(F.nth + 1) * (F.nr + 2), n_upd = (int64_t)(F.nth + 1) * (F.nr + 1);
    const int64_t n_axis = (int64_t)(F.nr + 1 + 2 * F.guard) * 2, n_grow = (int64_t)(2 * F.guard + 1) * F.pitch;
    auto guards = [&](FieldPtrs P) {
        hipLaunchKernelGGL(field_axis_kernel, dim3(nb(n_axis)), dim3(256), 0, stream, F, P);
        hipLaunchKernelGGL(field_guard_rows_kernel, dim3(nb(n_grow)), dim3(256), 0, stream, F, P);
    };
    guards(X);
    hipLaunchKernelGGL(field_copy_kernel, dim3(nb(n_all)), dim3(256), 0, stream, x0, X, n_all);
    hipLaunchKernelGGL(field_aux_kernel, dim3(nb(n_aux)), dim3(256), 0, stream, F, x0, aux);
    hipLaunchKernelGGL(field_update_kernel, dim3(nb(n_upd)), dim3(256), 0, stream, F, aux, x0, C0, X, 1);
    guards(X);
    for (int it = 0; it < ncorr; ++it) {
        hipLaunchKernelGGL(field_aux_kernel, dim3(nb(n_aux)), dim3(256), 0, stream, F, X, aux);
        hipLaunchKernelGGL(field_update_kernel, dim3(nb(n_upd)), dim3(256), 0, stream, F, aux, x0, C0, X, 0);
        guards(X);
    }
    if (damp_cells > 0) {
        hipLaunchKernelGGL(field_damp_kernel, dim3(nb((int64_t)(F.nth + 1) * (damp_cells + 1))), dim3(256), 0, stream,
                           F, X, damp_cells, damp_max);
        guards(X);
    }
    return hipGetLastError();
}

}  // namespace grpic
