// grpic_adjoint.hpp -- reverse-mode derivative of one GRPIC particle step
// (arXiv:2503.04558 Sec. 2.2-2.3, App. A): the vector-Jacobian product of
//   (xi, eta, u_r, u_th, u_ph, gathered D^i, B^i) -> (end point, u, deposit)
// needed by the adjoint of K push + deposit steps.
//
// Structure of one step (the forward replay records a tape of it):
//   gather D, B at x^n -> Boris kick at x^n -> geodesic predictor + ncorr
//   trapezoid correctors -> axis reflection -> Esirkepov deposit.
// The reverse sweep runs the same stages backwards.  The right-hand side and
// the Boris kick are differentiated by hand; the metric quantities they use
// are differentiated with respect to (r, theta) by forward mode (Dual2 below)
// on the same App. A formulas, which gives the second derivatives of the
// metric that the geodesic right-hand side's derivative needs.
//
// Everything here is plain double arithmetic (host or device), apart from the
// reciprocal and square root below, which take the hardware's estimates on
// the GPU.
#pragma once

#include <math.h>
#include <stdint.h>

namespace grpic {
namespace adj {

// 1/x and sqrt(x).  Compiled for the GPU: the hardware estimates refined by
// two Newton steps (1-2 ulp; the IEEE-rounded division and square root take
// twice the instructions and more registers, which this register-bound sweep
// spills).  Compiled for the host (the same per-particle sweep run on the
// CPU): the library's.
#if defined(__HIP_DEVICE_COMPILE__)
__device__ inline double inv_(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ inline double sqrt_(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    r = fma(-g, h, 0.5);
    return fma(g, r, g);
}
#else
inline double inv_(double x) { return 1.0 / x; }
inline double sqrt_(double x) { return ::sqrt(x); }
#endif

constexpr int kMaxCorr = 8;            // predictor-corrector passes the adjoint supports

// value and partial derivatives along r and theta
struct Dual2 {
    double v, r, t;
};
__host__ __device__ inline Dual2 dconst(double x) { return {x, 0.0, 0.0}; }
__host__ __device__ inline Dual2 operator+(Dual2 a, Dual2 b) { return {a.v + b.v, a.r + b.r, a.t + b.t}; }
__host__ __device__ inline Dual2 operator-(Dual2 a, Dual2 b) { return {a.v - b.v, a.r - b.r, a.t - b.t}; }
__host__ __device__ inline Dual2 operator-(Dual2 a) { return {-a.v, -a.r, -a.t}; }
__host__ __device__ inline Dual2 operator*(Dual2 a, Dual2 b) {
    return {a.v * b.v, a.r * b.v + a.v * b.r, a.t * b.v + a.v * b.t};
}
__host__ __device__ inline Dual2 operator/(Dual2 a, Dual2 b) {
    const double ib = inv_(b.v);
    const double q = a.v * ib;
    return {q, (a.r - q * b.r) * ib, (a.t - q * b.t) * ib};
}
__host__ __device__ inline Dual2 operator+(double a, Dual2 b) { return {a + b.v, b.r, b.t}; }
__host__ __device__ inline Dual2 operator+(Dual2 a, double b) { return {a.v + b, a.r, a.t}; }
__host__ __device__ inline Dual2 operator-(double a, Dual2 b) { return {a - b.v, -b.r, -b.t}; }
__host__ __device__ inline Dual2 operator-(Dual2 a, double b) { return {a.v - b, a.r, a.t}; }
__host__ __device__ inline Dual2 operator*(double a, Dual2 b) { return {a * b.v, a * b.r, a * b.t}; }
__host__ __device__ inline Dual2 operator*(Dual2 a, double b) { return {a.v * b, a.r * b, a.t * b}; }
__host__ __device__ inline Dual2 operator/(double a, Dual2 b) {
    const double ib = inv_(b.v);
    const double q = a * ib;
    return {q, -q * b.r * ib, -q * b.t * ib};
}
__host__ __device__ inline Dual2 sqrt(Dual2 a) {
    const double s = sqrt_(a.v);
    const double h = 0.5 * inv_(s);
    return {s, a.r * h, a.t * h};
}
using ::sqrt;          // the double overload stays visible next to the Dual2 one
// The same for the metric's template argument (double or Dual2).
__host__ __device__ inline double inv_any(double x) { return inv_(x); }
__host__ __device__ inline Dual2 inv_any(Dual2 b) { return 1.0 / b; }
__host__ __device__ inline double sqrt_any(double x) { return sqrt_(x); }
__host__ __device__ inline Dual2 sqrt_any(Dual2 a) { return sqrt(a); }

// Metric quantities of App. A (mass M reinstated) as one array, so that an
// adjoint can hold one cotangent per entry.
enum {
    M_ALPHA, M_IALPHA, M_BETA, M_GRR, M_GRP, M_GTT, M_GPP, M_HRR, M_HRP, M_HTT, M_HPP, M_SQRTG,
    M_DAL0, M_DAL1, M_DBE0, M_DBE1, M_DHRR0, M_DHRR1, M_DHRP0, M_DHRP1, M_DHTT0, M_DHTT1, M_DHPP0, M_DHPP1,
    M_N
};

// The quantities are handed to out(index, value) as they are formed, so a
// caller can contract their derivatives without storing them all.
template <class T, class Out>
__host__ __device__ inline void metric_emit(double a, double M, T r, T s, T c, Out&& out) {
    const double a2 = a * a;
    const T r2 = r * r, s2 = s * s, sc = s * c;
    const T rho2 = r2 + a2 * (c * c);
    const T irho2 = inv_any(rho2);
    const T z = 2.0 * M * r * irho2;
    const T opz = 1.0 + z;
    const T sq = sqrt_any(opz);
    const T iopz = inv_any(opz);
    const T is2 = inv_any(s2);
    const T ra2 = r2 + a2;
    const T Delta = ra2 - 2.0 * M * r;
    const T Sigma = ra2 * ra2 - a2 * Delta * s2;
    const T alpha = sq * iopz;
    const T beta = z * iopz;
    out(M_IALPHA, sq);
    out(M_ALPHA, alpha);
    out(M_BETA, beta);
    out(M_GRR, opz);
    out(M_GRP, -a * s2 * opz);
    out(M_GTT, rho2);
    out(M_GPP, Sigma * s2 * irho2);
    out(M_HRR, ra2 * irho2 - beta);
    out(M_HRP, a * irho2);
    out(M_HTT, irho2);
    out(M_HPP, irho2 * is2);
    out(M_SQRTG, rho2 * s * sq);
    const T irho4 = irho2 * irho2;
    const T dr_rho2 = 2.0 * r;
    const T dt_rho2 = -2.0 * a2 * sc;
    const T dz_r = 2.0 * M * (rho2 - 2.0 * r2) * irho4;
    const T dz_t = 4.0 * M * a2 * r * sc * irho4;
    const T al3 = alpha * iopz;
    const T al4 = iopz * iopz;
    out(M_DAL0, -0.5 * al3 * dz_r);
    out(M_DAL1, -0.5 * al3 * dz_t);
    const T dbe0 = al4 * dz_r, dbe1 = al4 * dz_t;
    out(M_DBE0, dbe0);
    out(M_DBE1, dbe1);
    out(M_DHRP0, -a * dr_rho2 * irho4);
    out(M_DHRP1, -a * dt_rho2 * irho4);
    out(M_DHTT0, -dr_rho2 * irho4);
    out(M_DHTT1, -dt_rho2 * irho4);
    out(M_DHRR0, -2.0 * r * a2 * s2 * irho4 - dbe0);
    out(M_DHRR1, 2.0 * a2 * ra2 * sc * irho4 - dbe1);
    out(M_DHPP0, -2.0 * r * irho4 * is2);
    out(M_DHPP1, -(dt_rho2 * s2 + 2.0 * rho2 * sc) * irho4 * is2 * is2);
}

template <class T>
__host__ __device__ inline void metric(double a, double M, T r, T s, T c, T m[M_N]) {
    metric_emit<T>(a, M, r, s, c, [&](int i, const T& v) { m[i] = v; });
}

// Grid and metric constants of a step.
struct Geo {
    double a, M, lnr0, dlnr, dth;
    int nr, nth, guard, pitch;
    double idlnr, idth;                        // 1/dlnr, 1/dth
    __host__ __device__ long index(int i, int j) const { return (long)(i + guard) * pitch + (j + guard); }
};

// r, sin(theta), cos(theta) at grid point (xi, eta): the only transcendental
// functions the metric needs.  The reverse forms them once per point for both
// the metric and its derivatives (they are not kept in the step's tape: the
// register file is the reverse sweep's limit, not its arithmetic).
struct Trig {
    double r, s, c;
};
__host__ __device__ inline Trig trig_at(const Geo& G, double xi, double eta) {
    const double th = eta * G.dth;
    return {::exp(G.lnr0 + xi * G.dlnr), ::sin(th), ::cos(th)};
}

__host__ __device__ inline void metric_at(const Geo& G, const Trig& t, double m[M_N]) {
    metric<double>(G.a, G.M, t.r, t.s, t.c, m);
}

// Cotangents mb of the metric quantities at a point -> cotangents of r and
// theta: the quantities' r and theta derivatives (forward mode, Dual2)
// contracted with mb as they are formed.
__host__ __device__ inline void metric_vjp_at(const Geo& G, const Trig& t, const double mb[M_N], double& rb,
                                              double& thb) {
    double ar = 0.0, at = 0.0;
    metric_emit<Dual2>(G.a, G.M, Dual2{t.r, 1.0, 0.0}, Dual2{t.s, 0.0, t.c}, Dual2{t.c, 0.0, -t.s},
                       [&](int i, const Dual2& v) {
        ar += mb[i] * v.r;
        at += mb[i] * v.t;
    });
    rb += ar;
    thb += at;
}

// ---------------------------------------------------------------- RHS
// Geodesic right-hand side (eq. particle-eom without the Lorentz force) in
// grid units: f = (dxi/dt, deta/dt, dphi/dt, du_r/dt, du_th/dt).
__host__ __device__ inline void rhs(const Geo& G, double eps, const double m[M_N], double r, double ur, double ut,
                                    double up, double f[5]) {
    const double uu = m[M_HRR] * ur * ur + 2.0 * m[M_HRP] * ur * up + m[M_HTT] * ut * ut + m[M_HPP] * up * up;
    const double u0 = sqrt_(eps + uu) * m[M_IALPHA];
    const double iu0 = inv_(u0);
    f[0] = ((m[M_HRR] * ur + m[M_HRP] * up) * iu0 - m[M_BETA]) * (G.idlnr * inv_(r));
    f[1] = m[M_HTT] * ut * iu0 * G.idth;
    f[2] = (m[M_HRP] * ur + m[M_HPP] * up) * iu0;
    for (int q = 0; q < 2; ++q) {
        const double quad = ur * ur * m[M_DHRR0 + q] + 2.0 * ur * up * m[M_DHRP0 + q]
                          + ut * ut * m[M_DHTT0 + q] + up * up * m[M_DHPP0 + q];
        f[3 + q] = -m[M_ALPHA] * u0 * m[M_DAL0 + q] + ur * m[M_DBE0 + q] - 0.5 * quad * iu0;
    }
}

// Cotangent g of f at point (xi, eta, ur, ut, up), t = trig_at(xi, eta) ->
// cotangents of the point (added to yb[0..1] = xi, eta and ub[0..2] = u_r,
// u_th, u_ph).
__host__ __device__ inline void rhs_vjp(const Geo& G, double eps, const Trig& t, double ur, double ut, double up,
                                        const double g[5], double yb[2], double ub[3]) {
    double m[M_N], mb[M_N];
    const double r = t.r;
    metric_at(G, t, m);
    for (int i = 0; i < M_N; ++i) mb[i] = 0.0;
    const double uu = m[M_HRR] * ur * ur + 2.0 * m[M_HRP] * ur * up + m[M_HTT] * ut * ut + m[M_HPP] * up * up;
    const double S = sqrt_(eps + uu);
    const double u0 = S * m[M_IALPHA];
    const double iu0 = inv_(u0);
    const double ir = inv_(r);
    const double iS = inv_(S);
    const double A1 = m[M_HRR] * ur + m[M_HRP] * up;
    const double B1 = m[M_HRP] * ur + m[M_HPP] * up;
    double urb = 0.0, utb = 0.0, upb = 0.0, rb = 0.0, iu0b = 0.0, u0b = 0.0;
    // f0 = (A1 iu0 - beta) ir / dlnr
    {
        const double c = g[0] * ir * G.idlnr;
        const double A1b = c * iu0;
        iu0b += c * A1;
        mb[M_BETA] -= c;
        rb -= c * (A1 * iu0 - m[M_BETA]) * ir;
        mb[M_HRR] += A1b * ur;
        mb[M_HRP] += A1b * up;
        urb += A1b * m[M_HRR];
        upb += A1b * m[M_HRP];
    }
    // f1 = h_tt ut iu0 / dth
    {
        const double c = g[1] * G.idth;
        mb[M_HTT] += c * ut * iu0;
        utb += c * m[M_HTT] * iu0;
        iu0b += c * m[M_HTT] * ut;
    }
    // f2 = B1 iu0
    {
        const double B1b = g[2] * iu0;
        iu0b += g[2] * B1;
        mb[M_HRP] += B1b * ur;
        mb[M_HPP] += B1b * up;
        urb += B1b * m[M_HRP];
        upb += B1b * m[M_HPP];
    }
    // f3+q = -alpha u0 dal_q + ur dbe_q - quad_q iu0 / 2
    for (int q = 0; q < 2; ++q) {
        const double gq = g[3 + q];
        const double quad = ur * ur * m[M_DHRR0 + q] + 2.0 * ur * up * m[M_DHRP0 + q]
                          + ut * ut * m[M_DHTT0 + q] + up * up * m[M_DHPP0 + q];
        mb[M_ALPHA] -= gq * u0 * m[M_DAL0 + q];
        u0b -= gq * m[M_ALPHA] * m[M_DAL0 + q];
        mb[M_DAL0 + q] -= gq * m[M_ALPHA] * u0;
        urb += gq * m[M_DBE0 + q];
        mb[M_DBE0 + q] += gq * ur;
        const double qb = -0.5 * gq * iu0;
        iu0b -= 0.5 * gq * quad;
        mb[M_DHRR0 + q] += qb * ur * ur;
        mb[M_DHRP0 + q] += qb * 2.0 * ur * up;
        mb[M_DHTT0 + q] += qb * ut * ut;
        mb[M_DHPP0 + q] += qb * up * up;
        urb += qb * (2.0 * ur * m[M_DHRR0 + q] + 2.0 * up * m[M_DHRP0 + q]);
        utb += qb * 2.0 * ut * m[M_DHTT0 + q];
        upb += qb * (2.0 * ur * m[M_DHRP0 + q] + 2.0 * up * m[M_DHPP0 + q]);
    }
    // iu0 = 1/u0; u0 = S ialpha; S = sqrt(eps + uu)
    u0b -= iu0b * iu0 * iu0;
    const double Sb = u0b * m[M_IALPHA];
    mb[M_IALPHA] += u0b * S;
    const double uub = 0.5 * Sb * iS;
    mb[M_HRR] += uub * ur * ur;
    mb[M_HRP] += uub * 2.0 * ur * up;
    mb[M_HTT] += uub * ut * ut;
    mb[M_HPP] += uub * up * up;
    urb += uub * (2.0 * m[M_HRR] * ur + 2.0 * m[M_HRP] * up);
    utb += uub * 2.0 * m[M_HTT] * ut;
    upb += uub * (2.0 * m[M_HRP] * ur + 2.0 * m[M_HPP] * up);
    // metric quantities -> r, theta -> xi, eta
    double thb = 0.0;
    metric_vjp_at(G, t, mb, rb, thb);
    yb[0] += rb * r * G.dlnr;
    yb[1] += thb * G.dth;
    ub[0] += urb;
    ub[1] += utb;
    ub[2] += upb;
}

// ---------------------------------------------------------------- Boris
// o = sqrt(gamma) eps_ijk v^j w^k with v^j = gamma^jl a_l.
__host__ __device__ inline void cross(const double m[M_N], const double a[3], const double w[3], double o[3]) {
    const double v0 = m[M_HRR] * a[0] + m[M_HRP] * a[2], v1 = m[M_HTT] * a[1], v2 = m[M_HRP] * a[0] + m[M_HPP] * a[2];
    o[0] = m[M_SQRTG] * (v1 * w[2] - v2 * w[1]);
    o[1] = m[M_SQRTG] * (v2 * w[0] - v0 * w[2]);
    o[2] = m[M_SQRTG] * (v0 * w[1] - v1 * w[0]);
}

__host__ __device__ inline void cross_vjp(const double m[M_N], const double a[3], const double w[3],
                                          const double ob[3], double ab[3], double wb[3], double mb[M_N]) {
    const double sg = m[M_SQRTG];
    const double v0 = m[M_HRR] * a[0] + m[M_HRP] * a[2], v1 = m[M_HTT] * a[1], v2 = m[M_HRP] * a[0] + m[M_HPP] * a[2];
    mb[M_SQRTG] += ob[0] * (v1 * w[2] - v2 * w[1]) + ob[1] * (v2 * w[0] - v0 * w[2]) + ob[2] * (v0 * w[1] - v1 * w[0]);
    wb[0] += sg * (ob[1] * v2 - ob[2] * v1);
    wb[1] += sg * (ob[2] * v0 - ob[0] * v2);
    wb[2] += sg * (ob[0] * v1 - ob[1] * v0);
    const double v0b = sg * (ob[2] * w[1] - ob[1] * w[2]);
    const double v1b = sg * (ob[0] * w[2] - ob[2] * w[0]);
    const double v2b = sg * (ob[1] * w[0] - ob[0] * w[1]);
    ab[0] += v0b * m[M_HRR] + v2b * m[M_HRP];
    ab[1] += v1b * m[M_HTT];
    ab[2] += v0b * m[M_HRP] + v2b * m[M_HPP];
    mb[M_HRR] += v0b * a[0];
    mb[M_HRP] += v0b * a[2] + v2b * a[0];
    mb[M_HTT] += v1b * a[1];
    mb[M_HPP] += v2b * a[2];
}

struct BorisTape {
    double Dl[3], hk, um[3], S, u0b, tf, t[3], tt, x1[3], ut[3], sf, s[3];
};

// Full-step generalised Boris kick (eqs. boris-plus-minus, u0bar, boris-scheme).
__host__ __device__ inline void boris(const double m[M_N], double qm, double dt, const double D[3], const double B[3],
                                      const double u[3], double up[3], BorisTape& T) {
    T.Dl[0] = m[M_GRR] * D[0] + m[M_GRP] * D[2];
    T.Dl[1] = m[M_GTT] * D[1];
    T.Dl[2] = m[M_GRP] * D[0] + m[M_GPP] * D[2];
    T.hk = qm * m[M_ALPHA] * dt * 0.5;
    for (int i = 0; i < 3; ++i) T.um[i] = u[i] + T.hk * T.Dl[i];
    const double uu = m[M_HRR] * T.um[0] * T.um[0] + 2.0 * m[M_HRP] * T.um[0] * T.um[2]
                    + m[M_HTT] * T.um[1] * T.um[1] + m[M_HPP] * T.um[2] * T.um[2];
    T.S = sqrt_(1.0 + uu);
    T.u0b = T.S * m[M_IALPHA];
    T.tf = 0.5 * qm * dt * inv_(T.u0b);
    for (int i = 0; i < 3; ++i) T.t[i] = T.tf * B[i];
    T.tt = m[M_GRR] * T.t[0] * T.t[0] + 2.0 * m[M_GRP] * T.t[0] * T.t[2]
         + m[M_GTT] * T.t[1] * T.t[1] + m[M_GPP] * T.t[2] * T.t[2];
    cross(m, T.um, T.t, T.x1);
    for (int i = 0; i < 3; ++i) T.ut[i] = T.um[i] + T.x1[i];
    T.sf = 2.0 * inv_(1.0 + T.tt);
    for (int i = 0; i < 3; ++i) T.s[i] = T.sf * T.t[i];
    double x2[3];
    cross(m, T.ut, T.s, x2);
    for (int i = 0; i < 3; ++i) up[i] = T.um[i] + x2[i] + T.hk * T.Dl[i];
}

// Cotangent of the kicked momentum -> cotangents of u, D, B and the metric.
__host__ __device__ inline void boris_vjp(const double m[M_N], double qm, double dt, const double D[3],
                                          const double B[3], const BorisTape& T, const double upb[3], double ub[3],
                                          double Db[3], double Bb[3], double mb[M_N]) {
    double umb[3], Dlb[3], utb[3] = {0, 0, 0}, sb[3] = {0, 0, 0}, x1b[3], tb[3] = {0, 0, 0};
    double hkb = 0.0;
    for (int i = 0; i < 3; ++i) {
        umb[i] = upb[i];
        hkb += upb[i] * T.Dl[i];
        Dlb[i] = upb[i] * T.hk;
    }
    // x2 = cross(ut, s), x2b = upb
    cross_vjp(m, T.ut, T.s, upb, utb, sb, mb);
    // s = sf t
    double sfb = 0.0;
    for (int i = 0; i < 3; ++i) { sfb += sb[i] * T.t[i]; tb[i] += sb[i] * T.sf; }
    const double ttb = -0.5 * sfb * T.sf * T.sf;
    // ut = um + x1
    for (int i = 0; i < 3; ++i) { umb[i] += utb[i]; x1b[i] = utb[i]; }
    cross_vjp(m, T.um, T.t, x1b, umb, tb, mb);
    // tt = t . g . t
    mb[M_GRR] += ttb * T.t[0] * T.t[0];
    mb[M_GRP] += ttb * 2.0 * T.t[0] * T.t[2];
    mb[M_GTT] += ttb * T.t[1] * T.t[1];
    mb[M_GPP] += ttb * T.t[2] * T.t[2];
    tb[0] += ttb * (2.0 * m[M_GRR] * T.t[0] + 2.0 * m[M_GRP] * T.t[2]);
    tb[1] += ttb * 2.0 * m[M_GTT] * T.t[1];
    tb[2] += ttb * (2.0 * m[M_GRP] * T.t[0] + 2.0 * m[M_GPP] * T.t[2]);
    // t = tf B
    double tfb = 0.0;
    for (int i = 0; i < 3; ++i) { tfb += tb[i] * B[i]; Bb[i] += tb[i] * T.tf; }
    // tf = qm dt / (2 u0b); u0b = S ialpha; S = sqrt(1 + uu)
    const double u0bb = -tfb * T.tf * inv_(T.u0b);
    const double Sb = u0bb * m[M_IALPHA];
    mb[M_IALPHA] += u0bb * T.S;
    const double uub = 0.5 * Sb * inv_(T.S);
    mb[M_HRR] += uub * T.um[0] * T.um[0];
    mb[M_HRP] += uub * 2.0 * T.um[0] * T.um[2];
    mb[M_HTT] += uub * T.um[1] * T.um[1];
    mb[M_HPP] += uub * T.um[2] * T.um[2];
    umb[0] += uub * (2.0 * m[M_HRR] * T.um[0] + 2.0 * m[M_HRP] * T.um[2]);
    umb[1] += uub * 2.0 * m[M_HTT] * T.um[1];
    umb[2] += uub * (2.0 * m[M_HRP] * T.um[0] + 2.0 * m[M_HPP] * T.um[2]);
    // um = u + hk Dl
    for (int i = 0; i < 3; ++i) {
        ub[i] += umb[i];
        hkb += umb[i] * T.Dl[i];
        Dlb[i] += umb[i] * T.hk;
    }
    mb[M_ALPHA] += hkb * qm * dt * 0.5;
    // Dl = g . D
    Db[0] += Dlb[0] * m[M_GRR] + Dlb[2] * m[M_GRP];
    Db[1] += Dlb[1] * m[M_GTT];
    Db[2] += Dlb[0] * m[M_GRP] + Dlb[2] * m[M_GPP];
    mb[M_GRR] += Dlb[0] * D[0];
    mb[M_GRP] += Dlb[0] * D[2] + Dlb[2] * D[0];
    mb[M_GTT] += Dlb[1] * D[1];
    mb[M_GPP] += Dlb[2] * D[2];
}

// ---------------------------------------------------------------- gather
// Bilinear interpolation in index space at (f, h) (already shifted by the
// stagger) and its reverse: field cotangents are handed to add(e, value).
template <class FieldT>
__host__ __device__ inline double gather(const Geo& G, const FieldT* F, double f, double h) {
    const int i = (int)::floor(f), j = (int)::floor(h);
    const double wf = f - i, wh = h - j;
    const long e = G.index(i, j);
    return (1.0 - wf) * (1.0 - wh) * F[e] + wf * (1.0 - wh) * F[e + G.pitch] + (1.0 - wf) * wh * F[e + 1]
         + wf * wh * F[e + G.pitch + 1];
}

// The four field cotangents go to add(e, g00, g10, g01, g11): element e of
// the lower corner, then the values for e, e + pitch, e + 1, e + pitch + 1.
template <class FieldT, class Add>
__host__ __device__ inline void gather_vjp(const Geo& G, const FieldT* F, double f, double h, double gb,
                                           double& fb, double& hb, Add add) {
    const int i = (int)::floor(f), j = (int)::floor(h);
    const double wf = f - i, wh = h - j;
    const long e = G.index(i, j);
    const double F00 = F[e], F10 = F[e + G.pitch], F01 = F[e + 1], F11 = F[e + G.pitch + 1];
    fb += gb * ((1.0 - wh) * (F10 - F00) + wh * (F11 - F01));
    hb += gb * ((1.0 - wf) * (F01 - F00) + wf * (F11 - F10));
    add(e, gb * (1.0 - wf) * (1.0 - wh), gb * wf * (1.0 - wh), gb * (1.0 - wf) * wh, gb * wf * wh);
}

// ---------------------------------------------------------------- deposit
// d L / d(xi0, eta0, xi1, eta1, dphi) for L = lambda . (Esirkepov fluxes of
// the move) (eqs. esirkepov-decomp, j-phi-deposit with the local prefix sum).
// L is bilinear in the corner shape values S_xy[a][b] = wx_x[a] wy_y[b]
// (x, y = 0 start / 1 end); the prefix sums become suffix sums of lambda.
__host__ __device__ inline double shape_w(double x) {
    const double ax = ::fabs(x);
    return ax >= 1.0 ? 0.0 : 1.0 - ax;
}
__host__ __device__ inline double shape_dw(double x) {
    const double ax = ::fabs(x);
    return ax >= 1.0 ? 0.0 : (x > 0.0 ? -1.0 : 1.0);
}

template <class LamT>
__host__ __device__ inline void deposit_vjp(const Geo& G, const LamT* lr, const LamT* lt, const LamT* lp, double qw,
                                            double dt, double xi0, double eta0, double xi1, double eta1, double dphi,
                                            double pb[5]) {
    const int i0 = (int)::floor(fmin(xi0, xi1)), j0 = (int)::floor(fmin(eta0, eta1));
    double wx0[3], wx1[3], wy0[3], wy1[3], dx0[3], dx1[3], dy0[3], dy1[3];
    for (int a = 0; a < 3; ++a) {
        wx0[a] = shape_w(xi0 - (i0 + a)); dx0[a] = shape_dw(xi0 - (i0 + a));
        wx1[a] = shape_w(xi1 - (i0 + a)); dx1[a] = shape_dw(xi1 - (i0 + a));
        wy0[a] = shape_w(eta0 - (j0 + a)); dy0[a] = shape_dw(eta0 - (j0 + a));
        wy1[a] = shape_w(eta1 - (j0 + a)); dy1[a] = shape_dw(eta1 - (j0 + a));
    }
    const double idt = 1.0 / dt;
    const double cf = -qw * idt, cp = qw * dphi * idt;
    const double c3 = cp * (1.0 / 3.0), c6 = cp * (1.0 / 6.0);
    double L_dphi = 0.0;
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b) {
            // suffix sums of lambda over the face rows / columns of the window
            double Lr = 0.0, Lt = 0.0;
            for (int a2 = a; a2 < 2; ++a2) Lr += (double)lr[G.index(i0 + a2, j0 + b)];
            for (int b2 = b; b2 < 2; ++b2) Lt += (double)lt[G.index(i0 + a, j0 + b2)];
            const double lpab = (double)lp[G.index(i0 + a, j0 + b)];
            const double C11 = 0.5 * cf * (Lr + Lt) + c3 * lpab;
            const double C10 = 0.5 * cf * (Lr - Lt) + c6 * lpab;
            const double C01 = 0.5 * cf * (-Lr + Lt) + c6 * lpab;
            const double C00 = -0.5 * cf * (Lr + Lt) + c3 * lpab;
            pb[0] += (C01 * wy1[b] + C00 * wy0[b]) * dx0[a];
            pb[1] += (C10 * wx1[a] + C00 * wx0[a]) * dy0[b];
            pb[2] += (C11 * wy1[b] + C10 * wy0[b]) * dx1[a];
            pb[3] += (C11 * wx1[a] + C01 * wx0[a]) * dy1[b];
            L_dphi += lpab * ((wx1[a] * wy1[b] + wx0[a] * wy0[b]) * (1.0 / 3.0)
                              + (wx1[a] * wy0[b] + wx0[a] * wy1[b]) * (1.0 / 6.0));
        }
    }
    pb[4] += qw * idt * L_dphi;
}

// ---------------------------------------------------------------- one step
enum { ST_ALIVE = 0, ST_OUT = 1, ST_BAD = 2 };

// Stagger (s_r, s_th) of D^r, D^th, D^ph, B^r, B^th, B^ph (Fig. Yee).
__host__ __device__ inline double stag_r(int c) { return (c == 0 || c == 4 || c == 5) ? 0.5 : 0.0; }
__host__ __device__ inline double stag_t(int c) { return (c == 1 || c == 3 || c == 5) ? 0.5 : 0.0; }

template <int NC>                              // NC: bound on the corrector passes
struct StepTape {
    double xi0, eta0, u[3];
    double D[3], B[3];
    double up[3];                              // momentum after the kick
    double pts[NC + 1][5];                     // y0 and the corrector points f was evaluated at
    double y[5];                               // raw end of the predictor-corrector
    double xi1, eta1, dphi;                    // end point after reflection
    int refl, status;
};

// Forward replay of one step from (xi0, eta0, u); fills the tape and returns
// the status.  The same formulas as the plain reference (Sec. 2.2-2.3).
template <int NC, class FieldT>
__host__ __device__ inline int replay_step(const Geo& G, const FieldT* const F[6], double qm, bool massless,
                                           double dt, int ncorr, double xi0, double eta0, const double u[3],
                                           StepTape<NC>& T) {
    T.xi0 = xi0;
    T.eta0 = eta0;
    for (int c = 0; c < 3; ++c) T.u[c] = u[c];
    for (int c = 0; c < 3; ++c) {
        T.D[c] = gather(G, F[c], xi0 - stag_r(c), eta0 - stag_t(c));
        T.B[c] = gather(G, F[3 + c], xi0 - stag_r(3 + c), eta0 - stag_t(3 + c));
    }
    double m0[M_N];
    const Trig t0 = trig_at(G, xi0, eta0);
    metric_at(G, t0, m0);
    if (massless) {
        for (int c = 0; c < 3; ++c) T.up[c] = u[c];
    } else {
        BorisTape bt;
        boris(m0, qm, dt, T.D, T.B, u, T.up, bt);
    }
    const double eps = massless ? 0.0 : 1.0;
    double f0[5], f1[5];
    rhs(G, eps, m0, t0.r, T.up[0], T.up[1], T.up[2], f0);
    const double y0[5] = {xi0, eta0, 0.0, T.up[0], T.up[1]};
    for (int c = 0; c < 5; ++c) { T.pts[0][c] = y0[c]; T.y[c] = y0[c] + dt * f0[c]; }
    for (int it = 0; it < ncorr; ++it) {
        for (int c = 0; c < 5; ++c) T.pts[it + 1][c] = T.y[c];
        double m[M_N];
        const Trig t = trig_at(G, T.y[0], T.y[1]);
        metric_at(G, t, m);
        rhs(G, eps, m, t.r, T.y[3], T.y[4], T.up[2], f1);
        for (int c = 0; c < 5; ++c) T.y[c] = y0[c] + 0.5 * dt * (f1[c] + f0[c]);
    }
    bool finite = isfinite(T.y[0]) && isfinite(T.y[1]) && isfinite(T.y[2]) && isfinite(T.y[3]) &&
                  isfinite(T.y[4]) && isfinite(T.up[2]);
    if (!finite || ::fabs(T.y[0] - xi0) >= 1.0 || ::fabs(T.y[1] - eta0) >= 1.0) {
        T.status = ST_BAD;
        return T.status;
    }
    T.xi1 = T.y[0];
    T.eta1 = T.y[1];
    T.refl = 0;
    if (T.eta1 < 0.0) { T.eta1 = -T.eta1; T.refl = 1; }
    else if (T.eta1 > (double)G.nth) { T.eta1 = 2.0 * G.nth - T.eta1; T.refl = 2; }
    T.dphi = T.y[2];
    T.status = (T.xi1 < 0.0 || T.xi1 >= (double)G.nr) ? ST_OUT : ST_ALIVE;
    return T.status;
}

// Reverse of one step.  a[5] holds on entry the cotangent of the state after
// the step (xi, eta, u_r, u_th, u_ph; zero if the particle did not survive
// it) and on return the cotangent of the state before it.  Field
// cotangents go to addF(component, lower-corner element, four values) as in
// gather_vjp.
template <int NC, class FieldT, class LamT, class AddF>
__host__ __device__ inline void reverse_step(const Geo& G, const FieldT* const F[6], const LamT* const lam[3],
                                             double qm, bool massless, double qw, double dt, int ncorr,
                                             const StepTape<NC>& T, double a[5], AddF addF) {
    if (T.status == ST_BAD) {
        for (int c = 0; c < 5; ++c) a[c] = 0.0;
        return;
    }
    if (T.status == ST_OUT) for (int c = 0; c < 5; ++c) a[c] = 0.0;
    // deposit: d/d(xi0, eta0, xi1, eta1, dphi)
    double pb[5] = {0, 0, 0, 0, 0};
    deposit_vjp(G, lam[0], lam[1], lam[2], qw, dt, T.xi0, T.eta0, T.xi1, T.eta1, T.dphi, pb);
    // cotangent of the raw predictor-corrector output y = (xi, eta, phi, u_r, u_th) and u_ph
    double z[5];
    z[0] = a[0] + pb[2];
    double etab = a[1] + pb[3], utb = a[3];
    if (T.refl) { etab = -etab; utb = -utb; }
    z[1] = etab;
    z[2] = pb[4];
    z[3] = a[2];
    z[4] = utb;
    double upb[3] = {0.0, 0.0, a[4]};        // u_ph passes through the predictor-corrector
    double y0b[5] = {0, 0, 0, 0, 0}, f0b[5] = {0, 0, 0, 0, 0};
    const double eps = massless ? 0.0 : 1.0;
    const double h = 0.5 * dt;
    for (int m = ncorr; m >= 1; --m) {
        double g[5], pyb[2] = {0.0, 0.0}, pub[3] = {0.0, 0.0, 0.0};
        for (int c = 0; c < 5; ++c) { y0b[c] += z[c]; f0b[c] += h * z[c]; g[c] = h * z[c]; }
        const double* P = T.pts[m];
        rhs_vjp(G, eps, trig_at(G, P[0], P[1]), P[3], P[4], T.up[2], g, pyb, pub);
        z[0] = pyb[0];
        z[1] = pyb[1];
        z[2] = 0.0;                          // f does not depend on phi
        z[3] = pub[0];
        z[4] = pub[1];
        upb[2] += pub[2];
    }
    for (int c = 0; c < 5; ++c) { y0b[c] += z[c]; f0b[c] += dt * z[c]; }
    // f0 = f(y0) at x^n; its metric adjoint goes into the position
    const Trig t0 = trig_at(G, T.xi0, T.eta0);
    {
        double pyb[2] = {0.0, 0.0}, pub[3] = {0.0, 0.0, 0.0};
        rhs_vjp(G, eps, t0, T.up[0], T.up[1], T.up[2], f0b, pyb, pub);
        y0b[0] += pyb[0];
        y0b[1] += pyb[1];
        upb[0] += pub[0];
        upb[1] += pub[1];
        upb[2] += pub[2];
    }
    upb[0] += y0b[3];
    upb[1] += y0b[4];
    double xib = y0b[0] + pb[0], etab0 = y0b[1] + pb[1];
    double ub[3] = {0.0, 0.0, 0.0}, Db[3] = {0.0, 0.0, 0.0}, Bb[3] = {0.0, 0.0, 0.0};
    if (massless) {
        for (int c = 0; c < 3; ++c) ub[c] = upb[c];
    } else {
        double m0[M_N], mb[M_N];
        const double r0 = t0.r;
        metric_at(G, t0, m0);
        for (int i = 0; i < M_N; ++i) mb[i] = 0.0;
        BorisTape bt;
        double up[3];
        boris(m0, qm, dt, T.D, T.B, T.u, up, bt);
        boris_vjp(m0, qm, dt, T.D, T.B, bt, upb, ub, Db, Bb, mb);
        double rb = 0.0, thb = 0.0;
        metric_vjp_at(G, t0, mb, rb, thb);
        xib += rb * r0 * G.dlnr;
        etab0 += thb * G.dth;
    }
    // gather: fields and the interpolation weights' dependence on position
    for (int c = 0; c < 6; ++c) {
        const double gb = c < 3 ? Db[c] : Bb[c - 3];
        if (gb == 0.0) continue;
        double fb = 0.0, hb = 0.0;
        gather_vjp(G, F[c], T.xi0 - stag_r(c), T.eta0 - stag_t(c), gb, fb, hb,
                   [&](long e, double g00, double g10, double g01, double g11) { addF(c, e, g00, g10, g01, g11); });
        xib += fb;
        etab0 += hb;
    }
    a[0] = xib;
    a[1] = etab0;
    a[2] = ub[0];
    a[3] = ub[1];
    a[4] = ub[2];
}

}  // namespace adj
}  // namespace grpic
