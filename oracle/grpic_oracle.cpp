/*
 * grpic_oracle.cpp -- plain FP64 CPU oracle for the GRPIC particle step of
 * Chen, Luepker & Yuan, "Introducing APERTURE: A GPU-based General
 * Relativistic Particle-in-Cell Simulation Framework" (arXiv:2503.04558).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, obviously correct reference
 * the HIP library is checked against.  It shares no code, header, table or
 * helper with the HIP library, and nothing in the library calls it.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark load
 * it (through oracle/oracle.py).
 *
 * What one step computes, per particle, in the paper's order:
 *   1. Kerr-Schild 3+1 metric at the particle (App. A, eqs. ks-coefficients,
 *      ks-variables, gamma-inverse, ks-alpha-beta, with the mass M written
 *      back in) and its analytic first derivatives.
 *   2. First-order (cloud-in-cell) interpolation of the six staggered field
 *      components D^i, B^i (Sec. 2.1, Fig. Yee; CIC is the default shape of
 *      Sec. 2.3), bilinear in grid-index space.
 *   3. One full-step generalised Boris kick at x^n (Sec. 2.2, eqs.
 *      boris-step, boris-plus-minus, u0bar, boris-scheme; the two half kicks
 *      of the Strang split bundled into one, as the paper does).
 *   4. Geodesic predictor-corrector (eqs. geodesic-predictor,
 *      geodesic-corrector) on the right-hand sides of eq. particle-eom
 *      without the Lorentz force, iterated ncorr times (3 by default).
 *   5. Axis reflection and radial outflow (Sec. 2.1 boundary conditions).
 *   6. Esirkepov charge-conserving deposit (Sec. 2.3, eqs.
 *      esirkepov-decomp, J-integral-eqn, j-phi-deposit) with a local prefix
 *      sum, in flux form F^r = J^r A_r, F^th = J^th A_th, G^ph = J^ph dV.
 *
 * Readings where the paper is silent or garbled (each is also listed in the
 * design notes of the repository):
 *   - positions are integrated in grid units xi = (ln r - ln r0)/dlnr,
 *     eta = theta/dtheta; momenta are the covariant KS components u_i;
 *   - metric derivatives are analytic at the particle position;
 *   - "3 iterations" = predictor + 3 trapezoid corrector passes;
 *   - J^ph carries +q (a positive charge moving in +phi gives J^ph > 0, as
 *     dD/dt = curl H - J requires) and is stored multiplied by the cell
 *     volume, like the other two components;
 *   - the axis reflects the end point (eta -> -eta, u_th -> -u_th); a
 *     particle leaving [0, Nr) in xi deposits its full move into the guard
 *     vertices and is then removed (cell = -1);
 *   - a particle whose end point is not finite or that moved one cell or more
 *     in either direction is removed without depositing and counted, and so
 *     is a particle whose cell, offsets or species index lie outside their
 *     ranges (such input would index outside the arrays).
 *
 * Build: g++ -O2 -std=c++17 -fPIC -shared -ffp-contract=off -fopenmp
 */
#include <cmath>
#include <cstdint>
#include <cstring>
#include <algorithm>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

/* ------------------------------------------------------------------ */
/* Scalar type plumbing.  Every formula below is written once over a   */
/* scalar type T; T = double is the oracle.  T = Dual (forward-mode    */
/* dual numbers) gives exact directional derivatives of the same code. */
/* ------------------------------------------------------------------ */
inline double val(double x) { return x; }

struct Dual {
    double v, d;
    Dual(double x = 0.0, double dx = 0.0) : v(x), d(dx) {}
};
inline double val(const Dual& x) { return x.v; }
inline Dual operator+(const Dual& a, const Dual& b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(const Dual& a, const Dual& b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(const Dual& a) { return Dual(-a.v, -a.d); }
inline Dual operator*(const Dual& a, const Dual& b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(const Dual& a, const Dual& b) {
    return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v));
}
inline Dual operator+(double a, const Dual& b) { return Dual(a + b.v, b.d); }
inline Dual operator+(const Dual& a, double b) { return Dual(a.v + b, a.d); }
inline Dual operator-(double a, const Dual& b) { return Dual(a - b.v, -b.d); }
inline Dual operator-(const Dual& a, double b) { return Dual(a.v - b, a.d); }
inline Dual operator*(double a, const Dual& b) { return Dual(a * b.v, a * b.d); }
inline Dual operator*(const Dual& a, double b) { return Dual(a.v * b, a.d * b); }
inline Dual operator/(const Dual& a, double b) { return Dual(a.v / b, a.d / b); }
inline Dual operator/(double a, const Dual& b) { return Dual(a / b.v, -a * b.d / (b.v * b.v)); }
inline Dual& operator+=(Dual& a, const Dual& b) { a = a + b; return a; }
inline Dual sqrt(const Dual& a) { double s = std::sqrt(a.v); return Dual(s, a.d / (2.0 * s)); }
inline Dual exp(const Dual& a) { double e = std::exp(a.v); return Dual(e, e * a.d); }
inline Dual sin(const Dual& a) { return Dual(std::sin(a.v), std::cos(a.v) * a.d); }
inline Dual cos(const Dual& a) { return Dual(std::cos(a.v), -std::sin(a.v) * a.d); }
inline Dual fabs(const Dual& a) { return a.v < 0 ? -a : a; }
using std::sqrt; using std::exp; using std::sin; using std::cos; using std::fabs;

/* Counting scalar: a double that tallies the floating-point operations done
 * on it (+, -, *, / and sqrt, exp, sin, cos each count one), to measure the
 * algorithm's operation count per particle-step. */
struct OpCount {
    long add, mul, div, sqrt_, exp_, sin_, cos_;
};
thread_local OpCount g_ops = {0, 0, 0, 0, 0, 0, 0};

struct Cnt {
    double v;
    Cnt(double x = 0.0) : v(x) {}
};
inline double val(const Cnt& x) { return x.v; }
inline Cnt operator+(const Cnt& a, const Cnt& b) { ++g_ops.add; return Cnt(a.v + b.v); }
inline Cnt operator-(const Cnt& a, const Cnt& b) { ++g_ops.add; return Cnt(a.v - b.v); }
inline Cnt operator-(const Cnt& a) { return Cnt(-a.v); }
inline Cnt operator*(const Cnt& a, const Cnt& b) { ++g_ops.mul; return Cnt(a.v * b.v); }
inline Cnt operator/(const Cnt& a, const Cnt& b) { ++g_ops.div; return Cnt(a.v / b.v); }
inline Cnt operator+(double a, const Cnt& b) { ++g_ops.add; return Cnt(a + b.v); }
inline Cnt operator+(const Cnt& a, double b) { ++g_ops.add; return Cnt(a.v + b); }
inline Cnt operator-(double a, const Cnt& b) { ++g_ops.add; return Cnt(a - b.v); }
inline Cnt operator-(const Cnt& a, double b) { ++g_ops.add; return Cnt(a.v - b); }
inline Cnt operator*(double a, const Cnt& b) { ++g_ops.mul; return Cnt(a * b.v); }
inline Cnt operator*(const Cnt& a, double b) { ++g_ops.mul; return Cnt(a.v * b); }
inline Cnt operator/(const Cnt& a, double b) { ++g_ops.div; return Cnt(a.v / b); }
inline Cnt operator/(double a, const Cnt& b) { ++g_ops.div; return Cnt(a / b.v); }
inline Cnt sqrt(const Cnt& a) { ++g_ops.sqrt_; return Cnt(std::sqrt(a.v)); }
inline Cnt exp(const Cnt& a) { ++g_ops.exp_; return Cnt(std::exp(a.v)); }
inline Cnt sin(const Cnt& a) { ++g_ops.sin_; return Cnt(std::sin(a.v)); }
inline Cnt cos(const Cnt& a) { ++g_ops.cos_; return Cnt(std::cos(a.v)); }
inline Cnt fabs(const Cnt& a) { return Cnt(std::fabs(a.v)); }

/* ------------------------------------------------------------------ */
/* Problem description (mirrored by ctypes structures in oracle.py).   */
/* ------------------------------------------------------------------ */
struct Geom {
    double a, M;                    /* spin and mass of the hole            */
    int32_t nr, nth, guard, pitch;  /* cells in r and theta; guard vertices; row pitch */
    double lnr0, dlnr, dth;         /* ln r at vertex 0; ln r step; theta step */
};

struct Species {
    double q, m;
    int32_t massless, pad;
};

/* Array element holding grid point (i, j) of any staggered quantity:
 * rows run along r, theta is the contiguous direction.                 */
inline long idx(const Geom& g, int i, int j) {
    return (long)(i + g.guard) * g.pitch + (j + g.guard);
}

/* Stagger of each field component, Fig. Yee:
 * D^r, B^th at (i+1/2, j); D^th, B^r at (i, j+1/2); D^ph at (i, j);
 * B^ph at (i+1/2, j+1/2).  Order: D^r, D^th, D^ph, B^r, B^th, B^ph.   */
const double kStagR[6] = {0.5, 0.0, 0.0, 0.0, 0.5, 0.5};
const double kStagT[6] = {0.0, 0.5, 0.0, 0.5, 0.0, 0.5};

/* ------------------------------------------------------------------ */
/* 1. Kerr-Schild metric, App. A, with M reinstated.                   */
/* ------------------------------------------------------------------ */
template <class T>
struct KS {
    T alpha, beta;                      /* lapse; radial shift beta^r        */
    T g_rr, g_rp, g_tt, g_pp;           /* gamma_ij                          */
    T h_rr, h_rp, h_tt, h_pp;           /* gamma^ij                          */
    T sqrtg;                            /* sqrt(det gamma_ij)                */
    T dal[2], dbe[2];                   /* d/dr, d/dtheta of alpha, beta^r   */
    T dh_rr[2], dh_rp[2], dh_tt[2], dh_pp[2];   /* of gamma^ij               */
};

template <class T>
void ks_metric(double a, double M, const T& r, const T& th, KS<T>& k) {
    const T s = sin(th), c = cos(th);
    const T s2 = s * s, c2 = c * c;
    const T rho2 = r * r + a * a * c2;                      /* rho^2        */
    const T z = 2.0 * M * r / rho2;                         /* z = 2Mr/rho^2 */
    const T Delta = r * r + a * a - 2.0 * M * r;
    const T Sigma = (r * r + a * a) * (r * r + a * a) - a * a * Delta * s2;

    k.g_rr = 1.0 + z;
    k.g_rp = -a * s2 * (1.0 + z);
    k.g_tt = rho2;
    k.g_pp = Sigma * s2 / rho2;

    k.h_rr = (a * a + r * r) / rho2 - 2.0 * M * r / (rho2 + 2.0 * M * r);
    k.h_rp = a / rho2;
    k.h_tt = 1.0 / rho2;
    k.h_pp = 1.0 / (rho2 * s2);

    k.alpha = 1.0 / sqrt(1.0 + z);
    k.beta = z / (1.0 + z);
    /* det gamma_ij = (1+z) rho^4 sin^2(theta): not printed in the paper,
     * follows from the printed gamma_ij.                                  */
    k.sqrtg = rho2 * s * sqrt(1.0 + z);

    /* Analytic derivatives (the paper does not say how they are formed). */
    const T rho4 = rho2 * rho2;
    const T drho2[2] = {2.0 * r, -2.0 * a * a * s * c};
    const T dz[2] = {2.0 * M * (rho2 - 2.0 * r * r) / rho4,
                     4.0 * M * a * a * r * s * c / rho4};
    const T al3 = k.alpha * k.alpha * k.alpha;
    const T al4 = al3 * k.alpha;
    for (int d = 0; d < 2; ++d) {
        k.dal[d] = -0.5 * al3 * dz[d];              /* alpha = (1+z)^(-1/2) */
        k.dbe[d] = al4 * dz[d];                     /* beta = z/(1+z)       */
        k.dh_rp[d] = -a * drho2[d] / rho4;
        k.dh_tt[d] = -drho2[d] / rho4;
    }
    /* gamma^rr = (r^2+a^2)/rho^2 - beta^r */
    k.dh_rr[0] = -2.0 * r * a * a * s2 / rho4 - k.dbe[0];
    k.dh_rr[1] = 2.0 * a * a * (r * r + a * a) * s * c / rho4 - k.dbe[1];
    /* gamma^phph = 1/(rho^2 sin^2) */
    k.dh_pp[0] = -2.0 * r / (rho4 * s2);
    k.dh_pp[1] = -(drho2[1] * s2 + 2.0 * rho2 * s * c) / (rho4 * s2 * s2);
}

/* ------------------------------------------------------------------ */
/* 4a. Right-hand sides X^i, U_i of eq. particle-eom without F_i, in    */
/*     grid units: y = (xi, eta, phi, u_r, u_th, u_ph).                  */
/* ------------------------------------------------------------------ */
template <class T>
void geodesic_rhs(const Geom& g, double eps, const T y[6], T f[6]) {
    const T r = exp(g.lnr0 + y[0] * g.dlnr);
    const T th = y[1] * g.dth;
    KS<T> k;
    ks_metric(g.a, g.M, r, th, k);
    const T ur = y[3], ut = y[4], up = y[5];
    const T uu = k.h_rr * ur * ur + 2.0 * k.h_rp * ur * up + k.h_tt * ut * ut + k.h_pp * up * up;
    const T u0 = sqrt(eps + uu) / k.alpha;                  /* u^0 */
    /* dx^i/dt = gamma^ij u_j / u^0 - beta^i; xi = (ln r - ln r0)/dlnr */
    f[0] = ((k.h_rr * ur + k.h_rp * up) / u0 - k.beta) / (r * g.dlnr);
    f[1] = k.h_tt * ut / u0 / g.dth;
    f[2] = (k.h_rp * ur + k.h_pp * up) / u0;
    /* du_i/dt = -alpha u^0 d_i alpha + u_k d_i beta^k - u_j u_k d_i gamma^jk / (2 u^0) */
    for (int d = 0; d < 2; ++d) {
        const T quad = ur * ur * k.dh_rr[d] + 2.0 * ur * up * k.dh_rp[d]
                     + ut * ut * k.dh_tt[d] + up * up * k.dh_pp[d];
        f[3 + d] = -k.alpha * u0 * k.dal[d] + ur * k.dbe[d] - quad / (2.0 * u0);
    }
    f[5] = T(0.0);                                          /* d_phi of nothing */
}

/* ------------------------------------------------------------------ */
/* 2. CIC gather of one staggered component, bilinear in index space.  */
/* ------------------------------------------------------------------ */
template <class T, class Arr>
T cic_gather(const Geom& g, const Arr& arr, double sr, double st, const T& xi, const T& eta) {
    const T f = xi - sr, h = eta - st;
    const int i = (int)std::floor(val(f)), j = (int)std::floor(val(h));
    const T wf = f - (double)i, wh = h - (double)j;
    return (1.0 - wf) * (1.0 - wh) * arr[idx(g, i, j)]
         + wf * (1.0 - wh) * arr[idx(g, i + 1, j)]
         + (1.0 - wf) * wh * arr[idx(g, i, j + 1)]
         + wf * wh * arr[idx(g, i + 1, j + 1)];
}

/* ------------------------------------------------------------------ */
/* 3. Generalised Boris kick, full step, metric and fields at x^n.     */
/* ------------------------------------------------------------------ */
/* (v x w)_i = e_ijk v^j w^k with e_ijk = sqrt(gamma) eps_ijk; v given   */
/* covariant (raised with gamma^ij), w contravariant.                   */
template <class T>
void cross_lower(const KS<T>& k, const T v[3], const T w[3], T out[3]) {
    const T vr = k.h_rr * v[0] + k.h_rp * v[2];
    const T vt = k.h_tt * v[1];
    const T vp = k.h_rp * v[0] + k.h_pp * v[2];
    out[0] = k.sqrtg * (vt * w[2] - vp * w[1]);
    out[1] = k.sqrtg * (vp * w[0] - vr * w[2]);
    out[2] = k.sqrtg * (vr * w[1] - vt * w[0]);
}

template <class T>
void boris_kick(const KS<T>& k, double qm, double dt, const T D[3], const T B[3], T u[3]) {
    /* half electric kick (q/m)(alpha dt/2) gamma_ij D^j */
    const T Dl[3] = {k.g_rr * D[0] + k.g_rp * D[2], k.g_tt * D[1], k.g_rp * D[0] + k.g_pp * D[2]};
    const T h = qm * k.alpha * dt * 0.5;
    T um[3];
    for (int c = 0; c < 3; ++c) um[c] = u[c] + h * Dl[c];
    /* ubar^0 from u^- (eq. u0bar) */
    const T uu = k.h_rr * um[0] * um[0] + 2.0 * k.h_rp * um[0] * um[2]
               + k.h_tt * um[1] * um[1] + k.h_pp * um[2] * um[2];
    const T u0bar = sqrt(1.0 + uu) / k.alpha;
    T t[3];
    for (int c = 0; c < 3; ++c) t[c] = qm * B[c] * dt / (2.0 * u0bar);
    /* t^k t_k with t_k = gamma_kl t^l */
    const T tt = k.g_rr * t[0] * t[0] + 2.0 * k.g_rp * t[0] * t[2]
               + k.g_tt * t[1] * t[1] + k.g_pp * t[2] * t[2];
    T x[3], ut[3], s[3], up[3];
    cross_lower(k, um, t, x);
    for (int c = 0; c < 3; ++c) ut[c] = um[c] + x[c];
    for (int c = 0; c < 3; ++c) s[c] = 2.0 * t[c] / (1.0 + tt);
    cross_lower(k, ut, s, x);
    for (int c = 0; c < 3; ++c) up[c] = um[c] + x[c];
    for (int c = 0; c < 3; ++c) u[c] = up[c] + h * Dl[c];
}

/* Vay's momentum update (Vay 2008) carried out in the FIDO frame, the
 * alternative the paper mentions in Sec. 2.2.  The FIDO measures D, B and
 * the spatial momentum u_i, and its clock advances alpha dt, so Vay's
 * flat-space step applies with dt -> alpha dt; written with the spatial
 * metric (dot products as gamma contractions, cross products with
 * e_ijk = sqrt(gamma) eps_ijk) it needs no explicit triad.  Vay's steps,
 * with h = (q/m) alpha dt / 2 and gamma = sqrt(1 + u^2):
 *   1. u_half = u + h (D + (u / gamma) x B)       explicit first half
 *   2. u'     = u_half + h D
 *   3. tau    = h B,  sigma = 1 + u'^2 - tau^2,  w = u'.tau,
 *      gamma_new^2 = (sigma + sqrt(sigma^2 + 4 (tau^2 + w^2))) / 2
 *      (the Lorentz factor that solves u_new = u' + (u_new/gamma_new) x tau)
 *   4. t = tau / gamma_new,  s = 1 / (1 + t^2),
 *      u_new = s (u' + (u'.t) t + u' x t).                              */
template <class T>
void vay_kick(const KS<T>& k, double qm, double dt, const T D[3], const T B[3], T u[3]) {
    const T Dl[3] = {k.g_rr * D[0] + k.g_rp * D[2], k.g_tt * D[1], k.g_rp * D[0] + k.g_pp * D[2]};
    const T h = qm * k.alpha * dt * 0.5;
    const T uu = k.h_rr * u[0] * u[0] + 2.0 * k.h_rp * u[0] * u[2]
               + k.h_tt * u[1] * u[1] + k.h_pp * u[2] * u[2];
    const T gam = sqrt(1.0 + uu);
    T v[3], vxB[3], up[3];
    for (int c = 0; c < 3; ++c) v[c] = u[c] / gam;
    cross_lower(k, v, B, vxB);
    for (int c = 0; c < 3; ++c) up[c] = (u[c] + h * (Dl[c] + vxB[c])) + h * Dl[c];
    T tau[3];
    for (int c = 0; c < 3; ++c) tau[c] = h * B[c];
    const T tau2 = k.g_rr * tau[0] * tau[0] + 2.0 * k.g_rp * tau[0] * tau[2]
                 + k.g_tt * tau[1] * tau[1] + k.g_pp * tau[2] * tau[2];
    const T w = up[0] * tau[0] + up[1] * tau[1] + up[2] * tau[2];
    const T upup = k.h_rr * up[0] * up[0] + 2.0 * k.h_rp * up[0] * up[2]
                 + k.h_tt * up[1] * up[1] + k.h_pp * up[2] * up[2];
    const T sigma = 1.0 + upup - tau2;
    const T gnew = sqrt(0.5 * (sigma + sqrt(sigma * sigma + 4.0 * (tau2 + w * w))));
    T t[3];
    for (int c = 0; c < 3; ++c) t[c] = tau[c] / gnew;
    const T s = 1.0 / (1.0 + tau2 / (gnew * gnew));
    const T ut = w / gnew;                                   /* u'_k t^k */
    const T tl[3] = {k.g_rr * t[0] + k.g_rp * t[2], k.g_tt * t[1], k.g_rp * t[0] + k.g_pp * t[2]};
    T x[3];
    cross_lower(k, up, t, x);
    for (int c = 0; c < 3; ++c) u[c] = s * (up[c] + ut * tl[c] + x[c]);
}

enum { KICK_BORIS = 0, KICK_VAY = 1 };

/* ------------------------------------------------------------------ */
/* 3+4. Kick at x^n, then the geodesic predictor-corrector.            */
/* Returns the raw end point y1 = (xi, eta, phi, u_r, u_th, u_ph).     */
/* ------------------------------------------------------------------ */
template <class T>
void push_with_fields(const Geom& g, const Species& sp, double dt, int ncorr,
                      const T& xi, const T& eta, const T u[3], const T D[3], const T B[3], T y1[6],
                      int kick = KICK_BORIS) {
    T uk[3] = {u[0], u[1], u[2]};
    const double eps = sp.massless ? 0.0 : 1.0;
    if (!sp.massless) {                 /* photons skip the Boris step */
        const T r = exp(g.lnr0 + xi * g.dlnr);
        const T th = eta * g.dth;
        KS<T> k;
        ks_metric(g.a, g.M, r, th, k);
        if (kick == KICK_VAY) vay_kick(k, sp.q / sp.m, dt, D, B, uk);
        else boris_kick(k, sp.q / sp.m, dt, D, B, uk);
    }
    const T y0[6] = {xi, eta, T(0.0), uk[0], uk[1], uk[2]};
    T f0[6], f1[6], yt[6];
    geodesic_rhs(g, eps, y0, f0);
    for (int c = 0; c < 6; ++c) yt[c] = y0[c] + dt * f0[c];            /* predictor */
    for (int it = 0; it < ncorr; ++it) {                                 /* corrector */
        geodesic_rhs(g, eps, yt, f1);
        for (int c = 0; c < 6; ++c) yt[c] = y0[c] + 0.5 * dt * (f1[c] + f0[c]);
    }
    for (int c = 0; c < 6; ++c) y1[c] = yt[c];
}

/* ------------------------------------------------------------------ */
/* 6. Esirkepov deposit of one move (xi0,eta0) -> (xi1,eta1).          */
/* ------------------------------------------------------------------ */
template <class T>
T shape1(const T& x) {                  /* CIC: W(x) = max(0, 1 - |x|) */
    const T ax = fabs(x);
    return val(ax) >= 1.0 ? T(0.0) : 1.0 - ax;
}

/* Accumulator with Neumaier compensation, so that the summed J is close
 * to correctly rounded whatever the particle order.                    */
struct Acc {
    double* sum;
    double* comp;
    double* scale;          /* optional: sum of the contributions' magnitude scales */
    void add(long e, double x, double sc) {
        const double s = sum[e], t = s + x;
        if (std::fabs(s) >= std::fabs(x)) comp[e] += (s - t) + x;
        else comp[e] += (x - t) + s;
        sum[e] = t;
        if (scale) scale[e] += sc;
    }
};

struct PlainAcc {
    double* sum;
    void add(long e, double x, double) { sum[e] += x; }
};

template <class T>
struct Move {
    int i0, j0;
    T Fr[2][3];     /* flux through (i0+a+1/2, j0+b) */
    T Ft[3][2];     /* flux through (i0+a, j0+b+1/2) */
    T Gp[3][3];     /* J^ph dV at (i0+a, j0+b)       */
    /* Magnitude scales |q w|/dt and |q w dphi|/dt of the terms that make up
     * each F and G value (shape weights are at most 1): a bound for the
     * rounding error of a value is a few ulps of its scale, whatever
     * cancellation happened inside it. */
    double scale_f, scale_p;
};

template <class T>
void esirkepov(double qw, double dt, const T& xi0, const T& eta0, const T& xi1, const T& eta1,
               const T& dphi, Move<T>& mv) {
    mv.i0 = (int)std::floor(std::min(val(xi0), val(xi1)));
    mv.j0 = (int)std::floor(std::min(val(eta0), val(eta1)));
    T Wr[3][3], Wt[3][3];
    for (int a = 0; a < 3; ++a) {
        const T wx0 = shape1(xi0 - (double)(mv.i0 + a));
        const T wx1 = shape1(xi1 - (double)(mv.i0 + a));
        for (int b = 0; b < 3; ++b) {
            const T wy0 = shape1(eta0 - (double)(mv.j0 + b));
            const T wy1 = shape1(eta1 - (double)(mv.j0 + b));
            /* S_ab = S(xi^a, eta^b), superscripts 0 = step n, 1 = step n+1 */
            const T S00 = wx0 * wy0, S01 = wx0 * wy1, S10 = wx1 * wy0, S11 = wx1 * wy1;
            Wr[a][b] = 0.5 * (S11 - S01 + S10 - S00);       /* Delta rho_r / q */
            Wt[a][b] = 0.5 * (S11 - S10 + S01 - S00);       /* Delta rho_th / q */
            mv.Gp[a][b] = qw * dphi / dt * (S11 / 3.0 + S10 / 6.0 + S01 / 6.0 + S00 / 3.0);
        }
    }
    mv.scale_f = std::fabs(qw) / dt;
    mv.scale_p = std::fabs(qw * val(dphi)) / dt;
    /* local prefix sums, zero flux on the low side of the window */
    for (int b = 0; b < 3; ++b) {
        T run(0.0);
        for (int a = 0; a < 2; ++a) { run = run + Wr[a][b]; mv.Fr[a][b] = -qw / dt * run; }
    }
    for (int a = 0; a < 3; ++a) {
        T run(0.0);
        for (int b = 0; b < 2; ++b) { run = run + Wt[a][b]; mv.Ft[a][b] = -qw / dt * run; }
    }
}

template <class AccT>
void scatter_move(const Geom& g, const Move<double>& mv, AccT& Fr, AccT& Ft, AccT& Gp) {
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) Fr.add(idx(g, mv.i0 + a, mv.j0 + b), mv.Fr[a][b], mv.scale_f);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 2; ++b) Ft.add(idx(g, mv.i0 + a, mv.j0 + b), mv.Ft[a][b], mv.scale_f);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Gp.add(idx(g, mv.i0 + a, mv.j0 + b), mv.Gp[a][b], mv.scale_p);
}

/* ------------------------------------------------------------------ */
/* Third-order spline shape (the option Sec. 2.3 names beside CIC):    */
/* the cubic B-spline, W(d) = (4 - 6 d^2 + 3 |d|^3)/6 for |d| < 1,     */
/* (2 - |d|)^3 / 6 for 1 <= |d| < 2, zero beyond; support 4 vertices.  */
/* ------------------------------------------------------------------ */
template <class T>
T shape3(const T& x) {
    const T ax = fabs(x);
    if (val(ax) >= 2.0) return T(0.0);
    if (val(ax) >= 1.0) {
        const T y = 2.0 - ax;
        return y * y * y / 6.0;
    }
    return (4.0 - 6.0 * ax * ax + 3.0 * ax * ax * ax) / 6.0;
}

/* Gather with the cubic shape: the 4 x 4 vertices of the component's
 * own stagger around the point (rows and columns beyond the grid are the
 * guard rows and the columns beyond the axes).                         */
template <class T, class Arr>
T spline3_gather(const Geom& g, const Arr& arr, double sr, double st, const T& xi, const T& eta) {
    const T f = xi - sr, h = eta - st;
    const int i = (int)std::floor(val(f)), j = (int)std::floor(val(h));
    T sum(0.0);
    for (int a = -1; a <= 2; ++a)
        for (int b = -1; b <= 2; ++b) sum = sum + shape3(f - (double)(i + a)) * shape3(h - (double)(j + b)) * arr[idx(g, i + a, j + b)];
    return sum;
}

/* Esirkepov deposit of one move with the cubic shape: the same
 * decomposition as for CIC on the 5 x 5 vertex window that holds both
 * supports (moves are under one cell), lower corner (floor(min xi) - 1,
 * floor(min eta) - 1).                                                  */
struct Move3 {
    int i0, j0;
    double Fr[4][5];     /* flux through (i0+a+1/2, j0+b) */
    double Ft[5][4];     /* flux through (i0+a, j0+b+1/2) */
    double Gp[5][5];     /* J^ph dV at (i0+a, j0+b)       */
    double scale_f, scale_p;
};

void esirkepov3(double qw, double dt, double xi0, double eta0, double xi1, double eta1, double dphi, Move3& mv) {
    mv.i0 = (int)std::floor(std::min(xi0, xi1)) - 1;
    mv.j0 = (int)std::floor(std::min(eta0, eta1)) - 1;
    double Wr[5][5], Wt[5][5];
    for (int a = 0; a < 5; ++a) {
        const double wx0 = shape3(xi0 - (double)(mv.i0 + a)), wx1 = shape3(xi1 - (double)(mv.i0 + a));
        for (int b = 0; b < 5; ++b) {
            const double wy0 = shape3(eta0 - (double)(mv.j0 + b)), wy1 = shape3(eta1 - (double)(mv.j0 + b));
            const double S00 = wx0 * wy0, S01 = wx0 * wy1, S10 = wx1 * wy0, S11 = wx1 * wy1;
            Wr[a][b] = 0.5 * (S11 - S01 + S10 - S00);
            Wt[a][b] = 0.5 * (S11 - S10 + S01 - S00);
            mv.Gp[a][b] = qw * dphi / dt * (S11 / 3.0 + S10 / 6.0 + S01 / 6.0 + S00 / 3.0);
        }
    }
    mv.scale_f = std::fabs(qw) / dt;
    mv.scale_p = std::fabs(qw * dphi) / dt;
    for (int b = 0; b < 5; ++b) {
        double run = 0.0;
        for (int a = 0; a < 4; ++a) { run += Wr[a][b]; mv.Fr[a][b] = -qw / dt * run; }
    }
    for (int a = 0; a < 5; ++a) {
        double run = 0.0;
        for (int b = 0; b < 4; ++b) { run += Wt[a][b]; mv.Ft[a][b] = -qw / dt * run; }
    }
}

/* Folding across the axes: a deposit at a vertex column beyond an axis
 * belongs to its mirror (axisymmetry maps (r, -theta, phi) to (r, theta,
 * phi + pi)); vertex columns j < 0 -> -j, j > nth -> 2 nth - j, values
 * kept (charge, J^r, J^ph are even); theta-face columns (j + 1/2) < 0 ->
 * -j - 1, > nth -> 2 nth - 1 - j, values negated (J^th is odd).  Each
 * vertex's discrete continuity is kept: the folded faces carry the
 * divergence of the folded vertices.                                    */
inline int fold_vertex(const Geom& g, int j) { return j < 0 ? -j : (j > g.nth ? 2 * g.nth - j : j); }
inline int fold_face(const Geom& g, int j, double& sign) {
    sign = 1.0;
    if (j < 0) { sign = -1.0; return -j - 1; }
    if (j >= g.nth) { sign = -1.0; return 2 * g.nth - 1 - j; }
    return j;
}

template <class AccT>
void scatter_move3(const Geom& g, const Move3& mv, AccT& Fr, AccT& Ft, AccT& Gp) {
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 5; ++b)
            Fr.add(idx(g, mv.i0 + a, fold_vertex(g, mv.j0 + b)), mv.Fr[a][b], mv.scale_f);
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 4; ++b) {
            double sgn;
            const int jf = fold_face(g, mv.j0 + b, sgn);
            Ft.add(idx(g, mv.i0 + a, jf), sgn * mv.Ft[a][b], mv.scale_f);
        }
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 5; ++b)
            Gp.add(idx(g, mv.i0 + a, fold_vertex(g, mv.j0 + b)), mv.Gp[a][b], mv.scale_p);
}

enum { SHAPE_CIC = 1, SHAPE_SPLINE3 = 3 };

/* ------------------------------------------------------------------ */
/* One particle, one step: gather, push, boundaries, deposit, store.   */
/* ------------------------------------------------------------------ */
enum { ST_ALIVE = 0, ST_OUT = 1, ST_BAD = 2, ST_DEAD = 3 };

struct Outcome {
    int status;
    int reflected;
    Move<double> mv;
    Move3 mv3;          /* the cubic shape's move (order 3) */
    int32_t cell;
    double xr, xth, u[3], dphi;
};

Outcome step_one(const Geom& g, const Species& sp, const double* const F[6], double w, double dt, int ncorr,
                 int32_t cell, double xr, double xth, const double u[3], int kick = KICK_BORIS,
                 int order = SHAPE_CIC) {
    Outcome o;
    o.reflected = 0;
    o.status = ST_DEAD;
    if (cell < 0) return o;
    /* inputs that would index outside the grid arrays: removed, no deposit */
    if (cell >= g.nr * g.nth || !(xr >= 0.0 && xr <= 1.0 && xth >= 0.0 && xth <= 1.0)) {
        o.status = ST_BAD;
        o.cell = -1;
        return o;
    }
    const int ci = cell / g.nth, cj = cell % g.nth;
    const double xi0 = ci + xr, eta0 = cj + xth;

    double D[3], B[3];
    for (int c = 0; c < 3; ++c) {
        if (order == SHAPE_SPLINE3) {
            D[c] = spline3_gather(g, F[c], kStagR[c], kStagT[c], xi0, eta0);
            B[c] = spline3_gather(g, F[3 + c], kStagR[3 + c], kStagT[3 + c], xi0, eta0);
        } else {
            D[c] = cic_gather(g, F[c], kStagR[c], kStagT[c], xi0, eta0);
            B[c] = cic_gather(g, F[3 + c], kStagR[3 + c], kStagT[3 + c], xi0, eta0);
        }
    }
    double y1[6];
    push_with_fields(g, sp, dt, ncorr, xi0, eta0, u, D, B, y1, kick);

    double xi1 = y1[0], eta1 = y1[1];
    double u1[3] = {y1[3], y1[4], y1[5]};
    bool finite = std::isfinite(xi1) && std::isfinite(eta1) && std::isfinite(y1[2]);
    for (int c = 0; c < 3; ++c) finite = finite && std::isfinite(u1[c]);
    if (!finite || std::fabs(xi1 - xi0) >= 1.0 || std::fabs(eta1 - eta0) >= 1.0) {
        o.status = ST_BAD;
        o.cell = -1;
        return o;
    }
    /* 5. axis reflection */
    if (eta1 < 0.0) { eta1 = -eta1; u1[1] = -u1[1]; o.reflected = 1; }
    else if (eta1 > (double)g.nth) { eta1 = 2.0 * g.nth - eta1; u1[1] = -u1[1]; o.reflected = 1; }

    if (order == SHAPE_SPLINE3) esirkepov3(sp.q * w, dt, xi0, eta0, xi1, eta1, y1[2], o.mv3);
    else esirkepov(sp.q * w, dt, xi0, eta0, xi1, eta1, y1[2], o.mv);
    o.dphi = y1[2];
    if (xi1 < 0.0 || xi1 >= (double)g.nr) {     /* radial outflow: removed after depositing */
        o.status = ST_OUT;
        o.cell = -1;
        return o;
    }
    /* 7. store as cell + offset */
    const int i1 = (int)std::floor(xi1);
    int j1 = (int)std::floor(eta1);
    if (j1 >= g.nth) j1 = g.nth - 1;
    o.status = ST_ALIVE;
    o.cell = i1 * g.nth + j1;
    o.xr = xi1 - i1;
    o.xth = eta1 - j1;
    for (int c = 0; c < 3; ++c) o.u[c] = u1[c];
    return o;
}

/* ------------------------------------------------------------------ */
/* Loss L = sum over steps of lambda . (F^r, F^th, G^ph) for one        */
/* particle, on any scalar type; with T = Dual its tangent is the exact */
/* directional derivative of L.  Positions are carried as xi, eta (the  */
/* double path's cell + offset is the same number).                     */
/* ------------------------------------------------------------------ */
struct DualArray {                       /* value and tangent arrays as one Dual array */
    const double* v;
    const double* d;
    Dual operator[](long e) const { return Dual(v[e], d ? d[e] : 0.0); }
};

/* The field arrays of step n when each component's states of successive
 * steps lie `stride` elements apart (stride 0: the same fields every step). */
inline const double* at_step(const double* a, long off) { return a + off; }
inline DualArray at_step(const DualArray& a, long off) { return DualArray{a.v + off, a.d ? a.d + off : nullptr}; }

template <class T, class Arr>
int particle_loss(const Geom& g, const Species& sp, const Arr* fld, const double* const* lam,
                  double w, double dt, int nsteps, int ncorr, T xi, T eta, T u[3], T& L,
                  double* traj = nullptr, long fstride = 0) {
    for (int n = 0; n < nsteps; ++n) {
        if (traj) { traj[2 * n] = val(xi); traj[2 * n + 1] = val(eta); }
        T D[3], B[3];
        for (int c = 0; c < 3; ++c) {
            D[c] = cic_gather(g, at_step(fld[c], n * fstride), kStagR[c], kStagT[c], xi, eta);
            B[c] = cic_gather(g, at_step(fld[3 + c], n * fstride), kStagR[3 + c], kStagT[3 + c], xi, eta);
        }
        T y1[6];
        push_with_fields(g, sp, dt, ncorr, xi, eta, u, D, B, y1);
        T xi1 = y1[0], eta1 = y1[1], ut1 = y1[4];
        bool finite = true;
        for (int c = 0; c < 6; ++c) finite = finite && std::isfinite(val(y1[c]));
        if (!finite || std::fabs(val(xi1) - val(xi)) >= 1.0 || std::fabs(val(eta1) - val(eta)) >= 1.0)
            return ST_BAD;
        if (val(eta1) < 0.0) { eta1 = -eta1; ut1 = -ut1; }
        else if (val(eta1) > (double)g.nth) { eta1 = 2.0 * g.nth - eta1; ut1 = -ut1; }
        Move<T> mv;
        esirkepov(sp.q * w, dt, xi, eta, xi1, eta1, y1[2], mv);
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 3; ++b) L = L + lam[0][idx(g, mv.i0 + a, mv.j0 + b)] * mv.Fr[a][b];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 2; ++b) L = L + lam[1][idx(g, mv.i0 + a, mv.j0 + b)] * mv.Ft[a][b];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) L = L + lam[2][idx(g, mv.i0 + a, mv.j0 + b)] * mv.Gp[a][b];
        if (traj) { traj[2 * n + 2] = val(xi1); traj[2 * n + 3] = val(eta1); }
        if (val(xi1) < 0.0 || val(xi1) >= (double)g.nr) return ST_OUT;
        xi = xi1;
        eta = eta1;
        u[0] = y1[3];
        u[1] = ut1;
        u[2] = y1[5];
    }
    return ST_ALIVE;
}

bool valid_input(const Geom& g, int nsp, int32_t cell, double xr, double xth, uint8_t s) {
    return cell >= 0 && cell < g.nr * g.nth && xr >= 0.0 && xr <= 1.0 && xth >= 0.0 && xth <= 1.0 && s < nsp;
}

/* ------------------------------------------------------------------ */
/* Photon emission and pair conversion (Sec. 4, the monopole spark-gap */
/* application; eq. optical-depth).                                    */
/*                                                                     */
/* Readings (also in the design notes):                                */
/*   - an e+- whose FIDO-frame Lorentz factor Gamma = sqrt(1 + u^2)     */
/*     (u^2 = gamma^ij u_i u_j at the end point of its step) exceeds    */
/*     gamma_thr emits one photon of FIDO energy eps_ph along its own   */
/*     momentum, at its end point, with its weight; its momentum        */
/*     magnitude drops by eps_ph (momentum conservation along the       */
/*     common direction);                                              */
/*   - a photon (FIDO energy eps = sqrt(gamma^ij u_i u_j)) converts     */
/*     with probability P = 1 - exp(-tau dt) per step, drawn after its  */
/*     push; the e- and e+ each get FIDO energy eps/2 along the        */
/*     photon's direction, at its end point, with its weight, and the  */
/*     photon is removed; photons below 2 m c^2 do not convert;        */
/*   - particles created in a step are not pushed in that step, and    */
/*     particles that left the grid in it neither emit nor convert;    */
/*   - random numbers: Philox4x64-10 (Salmon et al. 2011) with counter */
/*     (tag, step, 0, 0) and key (seed, 0): the first word gives the   */
/*     uniform U = (x0 >> 11) 2^-53 of a photon's conversion, the      */
/*     second the tag of an emitted photon or of the e-, the third     */
/*     that of the e+.                                                  */
/* ------------------------------------------------------------------ */
struct Philox4x64 {
    uint64_t x[4];
};

/* The high and low 64 bits of a * b. */
inline void mul_hi_lo(uint64_t a, uint64_t b, uint64_t& hi, uint64_t& lo) {
    const unsigned __int128 p = (unsigned __int128)a * b;
    hi = (uint64_t)(p >> 64);
    lo = (uint64_t)p;
}

/* Ten rounds of the Philox 4x64 bijection of the counter under the key,
 * the key advanced by the Weyl constants between rounds.                */
Philox4x64 philox4x64_10(const uint64_t ctr[4], const uint64_t key[2]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    uint64_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint64_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t hi0, lo0, hi1, lo1;
        mul_hi_lo(M0, x0, hi0, lo0);
        mul_hi_lo(M1, x2, hi1, lo1);
        const uint64_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
        x0 = y0; x1 = lo1; x2 = y2; x3 = lo0;
        k0 += W0;
        k1 += W1;
    }
    Philox4x64 r;
    r.x[0] = x0; r.x[1] = x1; r.x[2] = x2; r.x[3] = x3;
    return r;
}

struct Qed {
    double gamma_thr, eps_ph, tau;
    uint64_t seed;
    int32_t electron_sp, positron_sp, photon_sp, pad;
};

/* gamma^ij u_i u_j at the grid point (xi, eta). */
double u_squared(const Geom& g, double xi, double eta, const double u[3]) {
    KS<double> k;
    ks_metric(g.a, g.M, std::exp(g.lnr0 + xi * g.dlnr), eta * g.dth, k);
    return k.h_rr * u[0] * u[0] + 2.0 * k.h_rp * u[0] * u[2] + k.h_tt * u[1] * u[1] + k.h_pp * u[2] * u[2];
}

struct Created {
    int32_t cell;
    double xr, xth, u[3], w;
    uint8_t sp;
    uint64_t tag;
};

}  // namespace

/* ==================================================================== */
/* C entry points used by oracle/oracle.py (ctypes).                    */
/* ==================================================================== */
extern "C" {

/* Metric at (r, theta).  out[23]: alpha, beta^r, g_rr, g_rph, g_thth, g_phph,
 * h_rr, h_rph, h_thth, h_phph, sqrtg, then d/dr and d/dtheta of alpha,
 * beta^r, h_rr, h_rph, h_thth, h_phph (interleaved r, theta).            */
void orc_metric(double a, double M, double r, double th, double* out) {
    KS<double> k;
    ks_metric(a, M, r, th, k);
    const double v[11] = {k.alpha, k.beta, k.g_rr, k.g_rp, k.g_tt, k.g_pp,
                          k.h_rr, k.h_rp, k.h_tt, k.h_pp, k.sqrtg};
    std::memcpy(out, v, sizeof v);
    const double* d[6] = {k.dal, k.dbe, k.dh_rr, k.dh_rp, k.dh_tt, k.dh_pp};
    for (int q = 0; q < 6; ++q) { out[11 + 2 * q] = d[q][0]; out[12 + 2 * q] = d[q][1]; }
}

void orc_rhs(const Geom* g, double eps, const double* y, double* f) { geodesic_rhs(*g, eps, y, f); }

void orc_boris(const Geom* g, double qm, double dt, double xi, double eta,
               const double* u, const double* D, const double* B, double* out) {
    const double r = std::exp(g->lnr0 + xi * g->dlnr), th = eta * g->dth;
    KS<double> k;
    ks_metric(g->a, g->M, r, th, k);
    double uk[3] = {u[0], u[1], u[2]};
    boris_kick(k, qm, dt, D, B, uk);
    for (int c = 0; c < 3; ++c) out[c] = uk[c];
}

void orc_vay(const Geom* g, double qm, double dt, double xi, double eta,
             const double* u, const double* D, const double* B, double* out) {
    const double r = std::exp(g->lnr0 + xi * g->dlnr), th = eta * g->dth;
    KS<double> k;
    ks_metric(g->a, g->M, r, th, k);
    double uk[3] = {u[0], u[1], u[2]};
    vay_kick(k, qm, dt, D, B, uk);
    for (int c = 0; c < 3; ++c) out[c] = uk[c];
}

/* Kick with the given fields at x^n, then the geodesic PC; no boundaries. */
void orc_push_point(const Geom* g, const Species* sp, double dt, int ncorr, double xi, double eta,
                    const double* u, const double* D, const double* B, double* y1, int kick) {
    push_with_fields(*g, *sp, dt, ncorr, xi, eta, u, D, B, y1, kick);
}

void orc_gather(const Geom* g, const double* const* F, double xi, double eta, double* out) {
    for (int c = 0; c < 6; ++c) out[c] = cic_gather(*g, F[c], kStagR[c], kStagT[c], xi, eta);
}

/* Deposit one move into Fr, Fth, Gph (plain +=). */
void orc_deposit_move(const Geom* g, double qw, double dt, double xi0, double eta0,
                      double xi1, double eta1, double dphi, double* Fr, double* Fth, double* Gph) {
    Move<double> mv;
    esirkepov(qw, dt, xi0, eta0, xi1, eta1, dphi, mv);
    PlainAcc a{Fr}, b{Fth}, c{Gph};
    scatter_move(*g, mv, a, b, c);
}

void orc_gather3(const Geom* g, const double* const* F, double xi, double eta, double* out) {
    for (int c = 0; c < 6; ++c) out[c] = spline3_gather(*g, F[c], kStagR[c], kStagT[c], xi, eta);
}

/* Deposit one move with the cubic shape, folded across the axes (+=). */
void orc_deposit_move3(const Geom* g, double qw, double dt, double xi0, double eta0,
                       double xi1, double eta1, double dphi, double* Fr, double* Fth, double* Gph) {
    Move3 mv;
    esirkepov3(qw, dt, xi0, eta0, xi1, eta1, dphi, mv);
    PlainAcc a{Fr}, b{Fth}, c{Gph};
    scatter_move3(*g, mv, a, b, c);
}

/* Charge with the cubic shape, folded across the axes (Q is +=). */
void orc_charge3(const Geom* g, const Species* sp, int nsp, int64_t n, const int32_t* cell,
                 const double* xr, const double* xth, const double* w, const uint8_t* spi, double* Q) {
    (void)nsp;
    for (int64_t p = 0; p < n; ++p) {
        if (cell[p] < 0) continue;
        const int i = cell[p] / g->nth, j = cell[p] % g->nth;
        const double qw = sp[spi[p]].q * w[p];
        const double xi = i + xr[p], eta = j + xth[p];
        for (int a = -1; a <= 2; ++a)
            for (int b = -1; b <= 2; ++b)
                Q[idx(*g, i + a, fold_vertex(*g, j + b))] +=
                    qw * shape3(xi - (double)(i + a)) * shape3(eta - (double)(j + b));
    }
}

/* Charge Q_ij = sum_p q w S_ij(x_p) over live particles (Q is +=). */
void orc_charge(const Geom* g, const Species* sp, int nsp, int64_t n, const int32_t* cell,
                const double* xr, const double* xth, const double* w, const uint8_t* spi, double* Q) {
    (void)nsp;
    for (int64_t p = 0; p < n; ++p) {
        if (cell[p] < 0) continue;
        const int i = cell[p] / g->nth, j = cell[p] % g->nth;
        const double qw = sp[spi[p]].q * w[p];
        const double fx = xr[p], fy = xth[p];
        Q[idx(*g, i, j)] += qw * (1.0 - fx) * (1.0 - fy);
        Q[idx(*g, i + 1, j)] += qw * fx * (1.0 - fy);
        Q[idx(*g, i, j + 1)] += qw * (1.0 - fx) * fy;
        Q[idx(*g, i + 1, j + 1)] += qw * fx * fy;
    }
}

/* nsteps full steps over all particles, updated in place.  J arrays are +=.
 * nthreads == 1: serial, Neumaier-compensated J (parity mode), optional
 * A arrays receive, per element, the sum of the contributions' magnitude
 * scales (|q w|/dt for F^r and F^th, |q w dphi|/dt for G^ph).  nthreads > 1: OpenMP over particles
 * with thread-private J reduced in thread order (timing mode).
 * stats[4] (+=): particles removed at the radial edges, removed as
 * non-finite or moving >= 1 cell, axis reflections, live particle-steps.
 * kick: KICK_BORIS (the generalised Boris kick) or KICK_VAY.  order:
 * SHAPE_CIC or SHAPE_SPLINE3 (the cubic shape for gather and deposit,
 * folded across the axes; needs guard >= 3).                           */
void orc_run(const Geom* gp, const Species* sp, int nsp, int64_t n,
             int32_t* cell, double* xr, double* xth, double* ur, double* uth, double* uph,
             const double* w, const uint8_t* spi, double* phi,
             const double* const* F, double* Fr, double* Fth, double* Gph,
             double* Afr, double* Afth, double* Agph,
             double dt, int nsteps, int ncorr, int nthreads, int64_t* stats, int kick, int order) {
    const Geom& g = *gp;
    const long ncell = (long)(g.nr + 1 + 2 * g.guard) * g.pitch;
    int64_t st_out = 0, st_bad = 0, st_refl = 0, st_live = 0;

    if (nthreads <= 1) {
        std::vector<double> cr(ncell, 0.0), ct(ncell, 0.0), cp(ncell, 0.0);
        Acc A_r{Fr, cr.data(), Afr}, A_t{Fth, ct.data(), Afth}, A_p{Gph, cp.data(), Agph};
        for (int s = 0; s < nsteps; ++s) {
            for (int64_t p = 0; p < n; ++p) {
                const double u[3] = {ur[p], uth[p], uph[p]};
                if (cell[p] >= 0 && spi[p] >= nsp) { ++st_live; ++st_bad; cell[p] = -1; continue; }
                Outcome o = step_one(g, sp[spi[p]], F, w[p], dt, ncorr, cell[p], xr[p], xth[p], u, kick, order);
                if (o.status == ST_DEAD) continue;
                ++st_live;
                if (o.status == ST_BAD) { ++st_bad; cell[p] = -1; continue; }
                st_refl += o.reflected;
                if (order == SHAPE_SPLINE3) scatter_move3(g, o.mv3, A_r, A_t, A_p);
                else scatter_move(g, o.mv, A_r, A_t, A_p);
                if (phi) phi[p] += o.dphi;
                if (o.status == ST_OUT) { ++st_out; cell[p] = -1; continue; }
                cell[p] = o.cell; xr[p] = o.xr; xth[p] = o.xth;
                ur[p] = o.u[0]; uth[p] = o.u[1]; uph[p] = o.u[2];
            }
        }
        for (long e = 0; e < ncell; ++e) { Fr[e] += cr[e]; Fth[e] += ct[e]; Gph[e] += cp[e]; }
    } else {
#ifdef _OPENMP
        const int nt = nthreads;
        std::vector<std::vector<double>> priv(nt, std::vector<double>(3 * ncell, 0.0));
        for (int s = 0; s < nsteps; ++s) {
#pragma omp parallel num_threads(nt) reduction(+ : st_out, st_bad, st_refl, st_live)
            {
                const int tid = omp_get_thread_num();
                PlainAcc A_r{priv[tid].data()}, A_t{priv[tid].data() + ncell}, A_p{priv[tid].data() + 2 * ncell};
#pragma omp for schedule(static)
                for (int64_t p = 0; p < n; ++p) {
                    const double u[3] = {ur[p], uth[p], uph[p]};
                    if (cell[p] >= 0 && spi[p] >= nsp) { ++st_live; ++st_bad; cell[p] = -1; continue; }
                    Outcome o = step_one(g, sp[spi[p]], F, w[p], dt, ncorr, cell[p], xr[p], xth[p], u, kick, order);
                    if (o.status == ST_DEAD) continue;
                    ++st_live;
                    if (o.status == ST_BAD) { ++st_bad; cell[p] = -1; continue; }
                    st_refl += o.reflected;
                    if (order == SHAPE_SPLINE3) scatter_move3(g, o.mv3, A_r, A_t, A_p);
                    else scatter_move(g, o.mv, A_r, A_t, A_p);
                    if (phi) phi[p] += o.dphi;
                    if (o.status == ST_OUT) { ++st_out; cell[p] = -1; continue; }
                    cell[p] = o.cell; xr[p] = o.xr; xth[p] = o.xth;
                    ur[p] = o.u[0]; uth[p] = o.u[1]; uph[p] = o.u[2];
                }
            }
        }
        for (int t = 0; t < nt; ++t)
            for (long e = 0; e < ncell; ++e) {
                Fr[e] += priv[t][e]; Fth[e] += priv[t][ncell + e]; Gph[e] += priv[t][2 * ncell + e];
            }
#endif
    }
    if (stats) { stats[0] += st_out; stats[1] += st_bad; stats[2] += st_refl; stats[3] += st_live; }
}

/* L and its derivative along a direction: tangents tur, tuth, tuph per
 * particle (NULL = 0) and tF per field array (NULL array or entry = 0).
 * out[0] = L, out[1] = dL/deps, Neumaier-summed over particles.
 * status (optional, per particle): 0 alive after nsteps, 1 left radially,
 * 2 removed as bad, -1 not taken (removed or invalid input).            */
void orc_loss_dual_steps(const Geom* gp, const Species* sp, int nsp, int64_t n, const int32_t* cell,
                         const double* xr, const double* xth, const double* ur, const double* uth,
                         const double* uph, const double* w, const uint8_t* spi, const double* tur,
                         const double* tuth, const double* tuph, const double* const* F, const double* const* tF,
                         long fstride, const double* const* lam, double dt, int nsteps, int ncorr, double* out,
                         int32_t* status);

void orc_loss_dual(const Geom* gp, const Species* sp, int nsp, int64_t n, const int32_t* cell,
                   const double* xr, const double* xth, const double* ur, const double* uth, const double* uph,
                   const double* w, const uint8_t* spi, const double* tur, const double* tuth, const double* tuph,
                   const double* const* F, const double* const* tF, const double* const* lam,
                   double dt, int nsteps, int ncorr, double* out, int32_t* status) {
    orc_loss_dual_steps(gp, sp, nsp, n, cell, xr, xth, ur, uth, uph, w, spi, tur, tuth, tuph, F, tF, 0, lam, dt,
                        nsteps, ncorr, out, status);
}

/* orc_loss_dual with fields that change from step to step: component c of
 * step k at F[c] + k * fstride (tangents likewise), as a field solver
 * between the pushes would leave them; the derivative does not pass through
 * the field states (they are inputs). */
void orc_loss_dual_steps(const Geom* gp, const Species* sp, int nsp, int64_t n, const int32_t* cell,
                         const double* xr, const double* xth, const double* ur, const double* uth,
                         const double* uph, const double* w, const uint8_t* spi, const double* tur,
                         const double* tuth, const double* tuph, const double* const* F, const double* const* tF,
                         long fstride, const double* const* lam, double dt, int nsteps, int ncorr, double* out,
                         int32_t* status) {
    const Geom& g = *gp;
    DualArray fd[6];
    for (int c = 0; c < 6; ++c) fd[c] = DualArray{F[c], tF ? tF[c] : nullptr};
    double s0 = 0.0, c0 = 0.0, s1 = 0.0, c1 = 0.0;
    auto nadd = [](double& sum, double& comp, double x) {
        const double t = sum + x;
        if (std::fabs(sum) >= std::fabs(x)) comp += (sum - t) + x; else comp += (x - t) + sum;
        sum = t;
    };
    for (int64_t p = 0; p < n; ++p) {
        if (!valid_input(g, nsp, cell[p], xr[p], xth[p], spi[p])) {
            if (status) status[p] = -1;
            continue;
        }
        const int ci = cell[p] / g.nth, cj = cell[p] % g.nth;
        Dual u[3] = {Dual(ur[p], tur ? tur[p] : 0.0), Dual(uth[p], tuth ? tuth[p] : 0.0),
                     Dual(uph[p], tuph ? tuph[p] : 0.0)};
        Dual L(0.0, 0.0);
        const int st = particle_loss(g, sp[spi[p]], fd, lam, w[p], dt, nsteps, ncorr, Dual(ci + xr[p]),
                                     Dual(cj + xth[p]), u, L, nullptr, fstride);
        nadd(s0, c0, L.v);
        nadd(s1, c1, L.d);
        if (status) status[p] = st;
    }
    out[0] = s0 + c0;
    out[1] = s1 + c1;
}

/* L on plain doubles for one particle (finite differences); returns status.
 * traj (optional, 2 * (nsteps + 1)): positions (xi, eta) after each step. */
int orc_loss_particle(const Geom* gp, const Species* sp, double xi, double eta, const double* u0,
                      double w, const double* const* F, const double* const* lam, double dt, int nsteps,
                      int ncorr, double* L, double* traj) {
    double u[3] = {u0[0], u0[1], u0[2]};
    double l = 0.0;
    const int st = particle_loss(*gp, *sp, F, lam, w, dt, nsteps, ncorr, xi, eta, u, l, traj);
    *L = l;
    return st;
}

/* Operation counts of one particle-step (gather of the six components,
 * push, deposit) through the counting scalar.  out[7] (+=): add/sub, mul,
 * div, sqrt, exp, sin, cos. */
void orc_count_ops(const Geom* g, const Species* sp, const double* const* F, double w, double dt, int ncorr,
                   double xi, double eta, const double* u, long* out) {
    g_ops = OpCount{0, 0, 0, 0, 0, 0, 0};
    const Cnt cxi(xi), ceta(eta);
    Cnt D[3], B[3];
    for (int c = 0; c < 3; ++c) {
        D[c] = cic_gather(*g, F[c], kStagR[c], kStagT[c], cxi, ceta);
        B[c] = cic_gather(*g, F[3 + c], kStagR[3 + c], kStagT[3 + c], cxi, ceta);
    }
    const Cnt cu[3] = {Cnt(u[0]), Cnt(u[1]), Cnt(u[2])};
    Cnt y1[6];
    push_with_fields(*g, *sp, dt, ncorr, cxi, ceta, cu, D, B, y1);
    Move<Cnt> mv;
    esirkepov(sp->q * w, dt, cxi, ceta, y1[0], y1[1], y1[2], mv);
    const long v[7] = {g_ops.add, g_ops.mul, g_ops.div, g_ops.sqrt_, g_ops.exp_, g_ops.sin_, g_ops.cos_};
    for (int k = 0; k < 7; ++k) out[k] += v[k];
}

/* Philox4x64-10 of one counter under one key (for the pins). */
void orc_philox(const uint64_t* ctr, const uint64_t* key, uint64_t* out) {
    const Philox4x64 r = philox4x64_10(ctr, key);
    for (int k = 0; k < 4; ++k) out[k] = r.x[k];
}

/* One step of the monopole-workload particles: the push and deposit of
 * orc_run (Boris kick for massive species, none for photons; serial,
 * Neumaier-compensated J, optional scale arrays A), then photon emission
 * by e+- above gamma_thr and pair conversion of photons (the readings
 * above).  Particles are updated in place; created particles are appended
 * to the c_* arrays (capacity cap, in particle order: an emitter's photon,
 * a photon's e- then e+); *n_created receives their number (those beyond
 * cap are dropped).  stats[4] (+=) as in orc_run; qstats[3] (+=): photons
 * emitted, photons converted, created particles dropped.                */
void orc_run_qed(const Geom* gp, const Species* sp, int nsp, int64_t n,
                 int32_t* cell, double* xr, double* xth, double* ur, double* uth, double* uph,
                 const double* w, uint8_t* spi, const uint64_t* tag,
                 const double* const* F, double* Fr, double* Fth, double* Gph,
                 double* Afr, double* Afth, double* Agph, double dt, int ncorr, int64_t step, const Qed* qed,
                 int64_t cap, int32_t* c_cell, double* c_xr, double* c_xth, double* c_ur, double* c_uth,
                 double* c_uph, double* c_w, uint8_t* c_sp, uint64_t* c_tag, int64_t* n_created,
                 int64_t* stats, int64_t* qstats) {
    const Geom& g = *gp;
    const long ncell = (long)(g.nr + 1 + 2 * g.guard) * g.pitch;
    std::vector<double> cr(ncell, 0.0), ct(ncell, 0.0), cp(ncell, 0.0);
    Acc A_r{Fr, cr.data(), Afr}, A_t{Fth, ct.data(), Afth}, A_p{Gph, cp.data(), Agph};
    const double P = 1.0 - std::exp(-qed->tau * dt);          /* eq. optical-depth */
    int64_t st_out = 0, st_bad = 0, st_refl = 0, st_live = 0, emitted = 0, converted = 0, lost = 0, nc = 0;
    auto append = [&](const Created& c) {
        if (nc < cap) {
            c_cell[nc] = c.cell; c_xr[nc] = c.xr; c_xth[nc] = c.xth;
            c_ur[nc] = c.u[0]; c_uth[nc] = c.u[1]; c_uph[nc] = c.u[2];
            c_w[nc] = c.w; c_sp[nc] = c.sp; c_tag[nc] = c.tag;
            ++nc;
        } else {
            ++lost;
        }
    };
    for (int64_t p = 0; p < n; ++p) {
        const double u0[3] = {ur[p], uth[p], uph[p]};
        if (cell[p] >= 0 && spi[p] >= nsp) { ++st_live; ++st_bad; cell[p] = -1; continue; }
        const Outcome o = step_one(g, sp[spi[p]], F, w[p], dt, ncorr, cell[p], xr[p], xth[p], u0);
        if (o.status == ST_DEAD) continue;
        ++st_live;
        if (o.status == ST_BAD) { ++st_bad; cell[p] = -1; continue; }
        st_refl += o.reflected;
        scatter_move(g, o.mv, A_r, A_t, A_p);
        if (o.status == ST_OUT) { ++st_out; cell[p] = -1; continue; }
        cell[p] = o.cell; xr[p] = o.xr; xth[p] = o.xth;
        double u[3] = {o.u[0], o.u[1], o.u[2]};
        const int s = spi[p];
        const bool lepton = s == qed->electron_sp || s == qed->positron_sp;
        const bool photon = s == qed->photon_sp;
        if (lepton || photon) {
            const double xi1 = (o.cell / g.nth) + o.xr, eta1 = (o.cell % g.nth) + o.xth;
            const double uu = u_squared(g, xi1, eta1, u);
            const uint64_t ctr[4] = {tag[p], (uint64_t)step, 0, 0}, key[2] = {qed->seed, 0};
            if (lepton && std::sqrt(1.0 + uu) > qed->gamma_thr) {
                const Philox4x64 rn = philox4x64_10(ctr, key);
                const double umag = std::sqrt(uu);
                Created ph;
                ph.cell = o.cell; ph.xr = o.xr; ph.xth = o.xth; ph.w = w[p];
                ph.sp = (uint8_t)qed->photon_sp; ph.tag = rn.x[1];
                for (int c = 0; c < 3; ++c) ph.u[c] = u[c] * (qed->eps_ph / umag);
                append(ph);
                for (int c = 0; c < 3; ++c) u[c] = u[c] * ((umag - qed->eps_ph) / umag);
                ++emitted;
            } else if (photon) {
                const Philox4x64 rn = philox4x64_10(ctr, key);
                const double U = (double)(rn.x[0] >> 11) * (1.0 / 9007199254740992.0);
                const double eps = std::sqrt(uu);
                if (U < P && eps >= 2.0) {
                    const double scale = std::sqrt(0.25 * eps * eps - 1.0) / eps;
                    Created e[2];
                    for (int k = 0; k < 2; ++k) {
                        e[k].cell = o.cell; e[k].xr = o.xr; e[k].xth = o.xth; e[k].w = w[p];
                        for (int c = 0; c < 3; ++c) e[k].u[c] = u[c] * scale;
                    }
                    e[0].sp = (uint8_t)qed->electron_sp; e[0].tag = rn.x[1];
                    e[1].sp = (uint8_t)qed->positron_sp; e[1].tag = rn.x[2];
                    append(e[0]);
                    append(e[1]);
                    cell[p] = -1;
                    ++converted;
                    continue;
                }
            }
        }
        ur[p] = u[0]; uth[p] = u[1]; uph[p] = u[2];
    }
    for (long e = 0; e < ncell; ++e) { Fr[e] += cr[e]; Fth[e] += ct[e]; Gph[e] += cp[e]; }
    *n_created = nc;
    if (stats) { stats[0] += st_out; stats[1] += st_bad; stats[2] += st_refl; stats[3] += st_live; }
    if (qstats) { qstats[0] += emitted; qstats[1] += converted; qstats[2] += lost; }
}

int orc_has_openmp(void) {
#ifdef _OPENMP
    return 1;
#else
    return 0;
#endif
}

}  /* extern "C" */

/* ================================================================== */
/* Field solver (Sec. 2.1, eqs. integral-form, fld-predictor,          */
/* fld-corrector, Dr-axis; App. B, eqs. D-update, auxH, B-update,      */
/* auxE), plain and slow.                                              */
/*                                                                     */
/* Locations (Fig. Yee), array element (i, j) of each component:       */
/*   D^r, B^th, E_r, H_th at (i+1/2, j)    D^th, B^r, E_th, H_r at     */
/*   (i, j+1/2)    D^ph, E_ph at (i, j)    B^ph, H_ph at (i+1/2, j+1/2) */
/* with r_x = exp(lnr0 + x dlnr), theta_y = y dth.  Areas and volumes  */
/* are per unit phi, so the flux-form currents of the deposit are       */
/* J^r A^D_r, J^th A^D_th, J^ph A^D_ph.                                */
/*                                                                     */
/* Readings (also in the design notes):                                */
/*   - corrector: X^{n+1} = X^n + dt (w0 C(X^n) + w1 C(X~)) - dt J with */
/*     w0 + w1 = 1 (the printed dt/2 in front would not give Heun's    */
/*     method at w0 = w1 = 1/2, as the text says it does);             */
/*   - auxE: the sqrt(gamma) beta^r B^th term of E_ph is averaged with  */
/*     a factor 1/2 like every other interpolated term;                */
/*   - Dr-axis: D^r on an axis gains dt (+-H_ph / A^D_r - J^r); H_ph    */
/*     beyond the axis is zero (the phi loop there has no length);     */
/*   - inner and outer guard rows copy the nearest physical row (zero   */
/*     gradient; the outer one under the damping layer);               */
/*   - damping layer: after each step every component at radial grid    */
/*     position x >= nr - L is multiplied by 1 - d ((x - nr + L)/L)^2;  */
/*   - columns beyond the axes (read by the particle gather) are set     */
/*     after each step from the mirrored columns by axisymmetry, the    */
/*     theta components negated.                                        */
/* ================================================================== */
namespace {

/* 10-point Gauss-Legendre nodes and weights on [-1, 1]: roots of P_10
 * by Newton's method from the Chebyshev guesses, w = 2/((1-x^2) P'^2). */
struct Gauss10 {
    double x[10], w[10];
    Gauss10() {
        const int n = 10;
        for (int k = 0; k < n; ++k) {
            double z = std::cos(M_PI * (k + 0.75) / (n + 0.5));
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = z;
                for (int m = 2; m <= n; ++m) {
                    const double p2 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p0) / m;
                    p0 = p1;
                    p1 = p2;
                }
                const double dp = n * (z * p1 - p0) / (z * z - 1.0);
                const double dz = p1 / dp;
                z -= dz;
                if (std::fabs(dz) < 1e-16) break;
            }
            double p0 = 1.0, p1 = z;
            for (int m = 2; m <= n; ++m) {
                const double p2 = ((2.0 * m - 1.0) * z * p1 - (m - 1.0) * p0) / m;
                p0 = p1;
                p1 = p2;
            }
            const double dp = n * (z * p1 - p0) / (z * z - 1.0);
            x[k] = z;
            w[k] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
    }
};

struct FieldGeo {
    Geom g;
    double r(double x) const { return std::exp(g.lnr0 + x * g.dlnr); }
    double th(double y) const { return y * g.dth; }
    KS<double> at(double x, double y) const {
        KS<double> k;
        ks_metric<double>(g.a, g.M, r(x), th(y), k);
        return k;
    }
    double sqrtg(double rr, double t) const {
        KS<double> k;
        ks_metric<double>(g.a, g.M, rr, t, k);
        return k.sqrtg;
    }
    /* int_{t0}^{t1} sqrt(gamma)(r, theta) dtheta */
    double int_th(double rr, double t0, double t1) const {
        static const Gauss10 G;
        double s = 0.0;
        for (int k = 0; k < 10; ++k) {
            const double t = 0.5 * (t0 + t1) + 0.5 * (t1 - t0) * G.x[k];
            s += G.w[k] * sqrtg(rr, t);
        }
        return 0.5 * (t1 - t0) * s;
    }
    /* int_{r0}^{r1} sqrt(gamma)(r, theta) dr */
    double int_r(double t, double r0, double r1) const {
        static const Gauss10 G;
        double s = 0.0;
        for (int k = 0; k < 10; ++k) {
            const double rr = 0.5 * (r0 + r1) + 0.5 * (r1 - r0) * G.x[k];
            s += G.w[k] * sqrtg(rr, t);
        }
        return 0.5 * (r1 - r0) * s;
    }
    /* int int sqrt(gamma) dr dtheta over [r0, r1] x [t0, t1] */
    double int_rth(double r0, double r1, double t0, double t1) const {
        static const Gauss10 G;
        double s = 0.0;
        for (int k = 0; k < 10; ++k) {
            const double rr = 0.5 * (r0 + r1) + 0.5 * (r1 - r0) * G.x[k];
            s += G.w[k] * int_th(rr, t0, t1);
        }
        return 0.5 * (r1 - r0) * s;
    }
    double clamp_th(double y) const { return std::min(std::max(y, 0.0), (double)g.nth) * g.dth; }

    /* Area elements per unit phi, at the locations of the six components. */
    double AD_r(int i, int j) const {      /* r = r_{i+1/2}, theta over [j-1/2, j+1/2] within [0, pi] */
        return int_th(r(i + 0.5), clamp_th(j - 0.5), clamp_th(j + 0.5));
    }
    double AD_th(int i, int j) const {     /* theta_{j+1/2}, r over [i-1/2, i+1/2] */
        return int_r(th(j + 0.5), r(i - 0.5), r(i + 0.5));
    }
    double AD_ph(int i, int j) const {
        return int_rth(r(i - 0.5), r(i + 0.5), clamp_th(j - 0.5), clamp_th(j + 0.5));
    }
    double AB_r(int i, int j) const { return int_th(r(i), th(j), th(j + 1)); }
    double AB_th(int i, int j) const { return int_r(th(j), r(i), r(i + 1)); }
    double AB_ph(int i, int j) const { return int_rth(r(i), r(i + 1), th(j), th(j + 1)); }
};

/* Grid arrays of the solver: three D, three B components. */
struct FieldState {
    std::vector<double> c[6];   /* D^r, D^th, D^ph, B^r, B^th, B^ph */
};

/* Rows of a component that are updated; half: located at i + 1/2.      */
inline bool half_r(int comp) { return comp == 0 || comp == 4 || comp == 5; }

/* Zero-gradient guard rows; D^ph and B^th are zero on the axes. */
void fill_guards(const Geom& g, std::vector<double>* c) {
    for (int comp = 0; comp < 6; ++comp) {
        const int last = half_r(comp) ? g.nr - 1 : g.nr;
        for (int j = -g.guard; j < g.pitch - g.guard; ++j) {
            for (int i = -g.guard; i < 0; ++i) c[comp][idx(g, i, j)] = c[comp][idx(g, 0, j)];
            for (int i = last + 1; i <= g.nr + g.guard; ++i) c[comp][idx(g, i, j)] = c[comp][idx(g, last, j)];
        }
    }
    for (int i = -g.guard; i <= g.nr + g.guard; ++i) {
        c[2][idx(g, i, 0)] = c[2][idx(g, i, g.nth)] = 0.0;
        c[4][idx(g, i, 0)] = c[4][idx(g, i, g.nth)] = 0.0;
    }
}

/* Columns beyond the axes, which the particles' CIC gather reads within
 * half a cell of an axis.  The extended chart's point (r, -theta, phi) is
 * (r, theta, phi + pi): the theta basis vector is reversed there and the r
 * and phi ones are not, so by axisymmetry a component beyond the axis is
 * its value at the mirrored location, negated for D^th and B^th.  Mirror
 * pairs: integer columns -m <-> m and nth + m <-> nth - m; columns at
 * j + 1/2 (D^th, B^r, B^ph) -m <-> m - 1 and nth - 1 + m <-> nth - m.   */
void fill_axis_ghosts(const Geom& g, std::vector<double>* c) {
    for (int comp = 0; comp < 6; ++comp) {
        const double p = (comp == 1 || comp == 4) ? -1.0 : 1.0;
        const bool half_th = comp == 1 || comp == 3 || comp == 5;
        for (int i = -g.guard; i <= g.nr + g.guard; ++i)
            for (int m = 1; m <= g.guard; ++m) {
                auto& v = c[comp];
                if (half_th) {
                    v[idx(g, i, -m)] = p * v[idx(g, i, m - 1)];
                    v[idx(g, i, g.nth - 1 + m)] = p * v[idx(g, i, g.nth - m)];
                } else {
                    v[idx(g, i, -m)] = p * v[idx(g, i, m)];
                    v[idx(g, i, g.nth + m)] = p * v[idx(g, i, g.nth - m)];
                }
            }
    }
}

/* Auxiliary fields (eqs. auxE, auxH), metric coefficients formed first,
 * then averaged to the auxiliary field's location.  E[0..2] = E_r, E_th,
 * E_ph; H[0..2] = H_r, H_th, H_ph; each over the rows its circulations
 * use (-1 .. nr).                                                      */
void aux_fields(const FieldGeo& fg, const std::vector<double>* c, std::vector<double>* E, std::vector<double>* H) {
    const Geom& g = fg.g;
    const std::vector<double>&Dr = c[0], &Dt = c[1], &Dp = c[2], &Br = c[3], &Bt = c[4], &Bp = c[5];
    auto aG_rr = [&](double x, double y) { const KS<double> k = fg.at(x, y); return k.alpha * k.g_rr; };
    auto aG_rp = [&](double x, double y) { const KS<double> k = fg.at(x, y); return k.alpha * k.g_rp; };
    auto aG_tt = [&](double x, double y) { const KS<double> k = fg.at(x, y); return k.alpha * k.g_tt; };
    auto aG_pp = [&](double x, double y) { const KS<double> k = fg.at(x, y); return k.alpha * k.g_pp; };
    auto sgB = [&](double x, double y) { const KS<double> k = fg.at(x, y); return k.sqrtg * k.beta; };
    for (int i = -1; i <= g.nr; ++i) {
        for (int j = 0; j <= g.nth; ++j) {
            const long e = idx(g, i, j);
            const long em = idx(g, i - 1, j), ep = idx(g, i + 1, j);
            /* E_r at (i+1/2, j) */
            E[0][e] = aG_rr(i + 0.5, j) * Dr[e] + 0.5 * (aG_rp(i, j) * Dp[e] + aG_rp(i + 1, j) * Dp[ep]);
            /* E_th at (i, j+1/2) */
            if (j < g.nth)
                E[1][e] = aG_tt(i, j + 0.5) * Dt[e] -
                          0.5 * (sgB(i + 0.5, j + 0.5) * Bp[e] + sgB(i - 0.5, j + 0.5) * Bp[em]);
            /* E_ph at (i, j) */
            E[2][e] = aG_pp(i, j) * Dp[e] + 0.5 * (aG_rp(i + 0.5, j) * Dr[e] + aG_rp(i - 0.5, j) * Dr[em]) +
                      0.5 * (sgB(i + 0.5, j) * Bt[e] + sgB(i - 0.5, j) * Bt[em]);
            /* H_r at (i, j+1/2) */
            if (j < g.nth)
                H[0][e] = aG_rr(i, j + 0.5) * Br[e] +
                          0.5 * (aG_rp(i + 0.5, j + 0.5) * Bp[e] + aG_rp(i - 0.5, j + 0.5) * Bp[em]);
            /* H_th at (i+1/2, j) */
            H[1][e] = aG_tt(i + 0.5, j) * Bt[e] + 0.5 * (sgB(i, j) * Dp[e] + sgB(i + 1, j) * Dp[ep]);
            /* H_ph at (i+1/2, j+1/2) */
            if (j < g.nth)
                H[2][e] = aG_pp(i + 0.5, j + 0.5) * Bp[e] +
                          0.5 * (aG_rp(i, j + 0.5) * Br[e] + aG_rp(i + 1, j + 0.5) * Br[ep]) -
                          0.5 * (sgB(i, j + 0.5) * Dt[e] + sgB(i + 1, j + 0.5) * Dt[ep]);
        }
    }
}

/* Circulations C (eqs. D-update, B-update, Dr-axis) of the state c:
 * C[0..2] for D^r, D^th, D^ph (C_H, current not included), C[3..5] for
 * B^r, B^th, B^ph (C_E); zero outside the updated ranges.              */
void circulations(const FieldGeo& fg, const std::vector<double>* c, std::vector<double>* C) {
    const Geom& g = fg.g;
    const long n = (long)(g.nr + 1 + 2 * g.guard) * g.pitch;
    std::vector<double> E[3], H[3];
    for (int k = 0; k < 3; ++k) { E[k].assign(n, 0.0); H[k].assign(n, 0.0); }
    aux_fields(fg, c, E, H);
    for (int k = 0; k < 6; ++k) C[k].assign(n, 0.0);
    const double dth = g.dth;
    for (int i = 0; i <= g.nr; ++i) {
        const double dr_dual = fg.r(i + 0.5) - fg.r(i - 0.5), dr = fg.r(i + 1) - fg.r(i);
        for (int j = 0; j <= g.nth; ++j) {
            const long e = idx(g, i, j), em = idx(g, i - 1, j), ep = idx(g, i + 1, j);
            const long ejm = idx(g, i, j - 1), ejp = idx(g, i, j + 1);
            if (i < g.nr) {        /* D^r at (i+1/2, j), the axes included */
                const double hp = j < g.nth ? H[2][e] : 0.0, hm = j > 0 ? H[2][ejm] : 0.0;
                C[0][e] = (hp - hm) / fg.AD_r(i, j);
            }
            if (j < g.nth)         /* D^th at (i, j+1/2) */
                C[1][e] = (H[2][em] - H[2][e]) / fg.AD_th(i, j);
            if (j > 0 && j < g.nth)   /* D^ph at (i, j) */
                C[2][e] = ((H[1][e] - H[1][em]) * dth + (H[0][ejm] - H[0][e]) * dr_dual) / fg.AD_ph(i, j);
            if (j < g.nth)         /* B^r at (i, j+1/2) */
                C[3][e] = -(E[2][ejp] - E[2][e]) / fg.AB_r(i, j);
            if (i < g.nr && j > 0 && j < g.nth)   /* B^th at (i+1/2, j) */
                C[4][e] = -(E[2][e] - E[2][ep]) / fg.AB_th(i, j);
            if (i < g.nr && j < g.nth)            /* B^ph at (i+1/2, j+1/2) */
                C[5][e] = -((E[1][ep] - E[1][e]) * dth + (E[0][e] - E[0][ejp]) * dr) / fg.AB_ph(i, j);
        }
    }
}

/* Current per unit area (flux form / area) at the D locations. */
void current_density(const FieldGeo& fg, const double* const* F, std::vector<double>* J) {
    const Geom& g = fg.g;
    const long n = (long)(g.nr + 1 + 2 * g.guard) * g.pitch;
    for (int k = 0; k < 3; ++k) J[k].assign(n, 0.0);
    if (!F) return;
    for (int i = 0; i <= g.nr; ++i)
        for (int j = 0; j <= g.nth; ++j) {
            const long e = idx(g, i, j);
            if (i < g.nr && F[0]) J[0][e] = F[0][e] / fg.AD_r(i, j);
            if (j < g.nth && F[1]) J[1][e] = F[1][e] / fg.AD_th(i, j);
            if (j > 0 && j < g.nth && F[2]) J[2][e] = F[2][e] / fg.AD_ph(i, j);
        }
}

}  /* namespace */

extern "C" {

/* Area elements per unit phi at the six component locations (arrays of
 * the grid's shape, zero where the component does not live).          */
void orc_field_areas(const Geom* gp, double* const* A) {
    const FieldGeo fg{*gp};
    const Geom& g = *gp;
    for (int i = 0; i <= g.nr; ++i)
        for (int j = 0; j <= g.nth; ++j) {
            const long e = idx(g, i, j);
            if (i < g.nr) A[0][e] = fg.AD_r(i, j);
            if (j < g.nth) A[1][e] = fg.AD_th(i, j);
            A[2][e] = fg.AD_ph(i, j);
            if (j < g.nth) A[3][e] = fg.AB_r(i, j);
            if (i < g.nr) A[4][e] = fg.AB_th(i, j);
            if (i < g.nr && j < g.nth) A[5][e] = fg.AB_ph(i, j);
        }
}

/* Circulations of the state (arrays D^r..B^ph) into C[6] (guard rows of
 * the state are filled first; D^ph, B^th are zeroed on the axes).      */
void orc_field_circulations(const Geom* gp, double* const* X, double* const* C) {
    const FieldGeo fg{*gp};
    const long n = (long)(gp->nr + 1 + 2 * gp->guard) * gp->pitch;
    std::vector<double> c[6], out[6];
    for (int k = 0; k < 6; ++k) c[k].assign(X[k], X[k] + n);
    fill_guards(*gp, c);
    circulations(fg, c, out);
    for (int k = 0; k < 6; ++k) std::copy(out[k].begin(), out[k].end(), C[k]);
}

/* One field step in place: X[6] = D^r, D^th, D^ph, B^r, B^th, B^ph (grid
 * arrays); F[3] = flux-form currents of the step (NULL = none); predictor
 * and ncorr corrector passes with weights w0 = 1 - w1, w1; then the
 * damping layer over the last damp_cells rows (0 = none) and the columns
 * beyond the axes.                                                     */
void orc_field_step(const Geom* gp, double* const* X, const double* const* F, double dt, double w1,
                    int ncorr, int damp_cells, double damp_max) {
    const Geom& g = *gp;
    const FieldGeo fg{g};
    const long n = (long)(g.nr + 1 + 2 * g.guard) * g.pitch;
    std::vector<double> x0[6], xt[6], C0[6], C1[6], J[3];
    for (int k = 0; k < 6; ++k) x0[k].assign(X[k], X[k] + n);
    fill_guards(g, x0);
    circulations(fg, x0, C0);
    current_density(fg, F, J);
    const double w0 = 1.0 - w1;
    /* updated ranges: the circulations are zero elsewhere, so x0 + dt C
     * leaves guard rows and the axis zeros of D^ph, B^th unchanged, and
     * the guards are refilled after every pass                          */
    for (int k = 0; k < 6; ++k) {
        xt[k] = x0[k];
        for (long e = 0; e < n; ++e) xt[k][e] = x0[k][e] + dt * (C0[k][e] - (k < 3 ? J[k][e] : 0.0));
    }
    fill_guards(g, xt);
    for (int it = 0; it < ncorr; ++it) {
        circulations(fg, xt, C1);
        for (int k = 0; k < 6; ++k)
            for (long e = 0; e < n; ++e)
                xt[k][e] = x0[k][e] + dt * (w0 * C0[k][e] + w1 * C1[k][e]) - dt * (k < 3 ? J[k][e] : 0.0);
        fill_guards(g, xt);
    }
    if (damp_cells > 0) {
        const double x_in = (double)(g.nr - damp_cells);
        for (int k = 0; k < 6; ++k)
            for (int i = 0; i <= g.nr; ++i) {
                const double x = i + (half_r(k) ? 0.5 : 0.0);
                if (x < x_in) continue;
                const double s = (x - x_in) / damp_cells;
                const double f = 1.0 - damp_max * s * s;
                for (int j = 0; j <= g.nth; ++j) xt[k][idx(g, i, j)] *= f;
            }
        fill_guards(g, xt);
    }
    fill_axis_ghosts(g, xt);
    for (int k = 0; k < 6; ++k) std::copy(xt[k].begin(), xt[k].end(), X[k]);
}

}  /* extern "C" */
