// grpic_device.hpp -- device-side building blocks of the GRPIC particle step
// (arXiv:2503.04558, Sec. 2.2-2.3, App. A), written once over the real type R
// so that the FP64 kernel and the split-precision kernel share them.
//
// Positions are handled in grid units: xi = (ln r - lnr0)/dlnr and
// eta = theta/dth, so a cell is the unit square.  Momenta are the covariant
// Kerr-Schild components u_r, u_th, u_ph.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace grpic {

constexpr int kMaxSpecies = 8;

// Everything a push+deposit launch needs, passed by value.
struct StepArgs {
    double a, M;
    int nr, nth, guard, pitch;
    double lnr0, dlnr, dth;
    double idlnr, idth;                     // 1/dlnr, 1/dth
    double inv_nth, inv_tpr;                // 1/nth, 1/tiles per row (integer quotients)
    int small_steps;                        // Taylor offsets: 2 with 2 dlnr, 2 dth <= kTinyArg, 1 <= kSmallArg, else 0
    int fp64_rows;                          // split precision: rows i < fp64_rows run in FP64
    int pole_cols;                          // split precision: columns this close to the axis run in FP64
    double dt, idt;                         // step, 1/step
    int ncorr, nsp;
    double q[kMaxSpecies], m[kMaxSpecies];
    double qm[kMaxSpecies];                 // q/m (0 for massless species)
    int massless[kMaxSpecies];
    int64_t n;
    int32_t* cell;
    void *xr, *xth, *ur, *uth, *uph, *w;
    const uint8_t* sp;
    void* phi;
    const void* F[6];                       // D^r, D^th, D^ph, B^r, B^th, B^ph
    double *Fr, *Fth, *Gph;
    unsigned long long* counters;           // optional, GRPIC_NCOUNTERS entries
};

template <class R>
struct Metric {
    R alpha, beta;                          // lapse, radial shift beta^r
    R g_rr, g_rp, g_tt, g_pp;               // gamma_ij
    R h_rr, h_rp, h_tt, h_pp;               // gamma^ij
    R sqrtg;                                // sqrt(det gamma_ij) = rho^2 sin sqrt(1+z)
    R ialpha;                               // 1/alpha = sqrt(1+z)
};

// 1/x from the hardware reciprocal estimate, refined by two Newton steps for
// double (a few ulp, no division sequence); float takes the estimate (1 ulp).
__device__ __forceinline__ double rcp(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }   // 1 ulp

// sqrt(x) and 1/sqrt(x) together, for x >= 1 (or a positive normal x):
// double refines the hardware reciprocal-square-root estimate y by two
// coupled Newton steps on g ~ sqrt(x) = x y and h ~ 1/(2 sqrt(x)) = y/2
// (residual r = 1/2 - g h; each step squares the relative error, so a few
// ulp remain); float takes the estimate (1 ulp) and one product.
__device__ __forceinline__ void sqrt_rsqrt(double x, double& sq, double& rsq) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    r = fma(-g, h, 0.5);
    sq = fma(g, r, g);
    rsq = 2.0 * fma(h, r, h);
}
__device__ __forceinline__ void sqrt_rsqrt(float x, float& sq, float& rsq) {
    rsq = __builtin_amdgcn_rsqf(x);
    sq = x * rsq;
}

// Kerr-Schild 3+1 quantities of App. A (mass M reinstated) at radius r and
// polar angle with sine s, cosine c, as the kick needs them.  1/rho^2 and
// 1/sin^2 come from one reciprocal of their product.
template <class R>
__device__ __forceinline__ void ks_metric(R a, R M, R r, R s, R c, Metric<R>& k) {
    const R a2 = a * a, r2 = r * r, s2 = s * s;
    const R rho2 = r2 + a2 * (c * c);
    const R iP = rcp(s2 * rho2);
    const R irho2 = s2 * iP;
    const R z = R(2) * M * r * irho2;
    const R opz = R(1) + z;
    R sq, rsq;                                    // sqrt(1+z) = 1/alpha, 1/sqrt(1+z) = alpha
    sqrt_rsqrt(opz, sq, rsq);
    const R iopz = rsq * rsq;
    const R is2 = rho2 * iP;
    const R ra2 = r2 + a2;
    const R Delta = ra2 - R(2) * M * r;
    const R Sigma = ra2 * ra2 - a2 * Delta * s2;
    k.ialpha = sq;
    k.alpha = rsq;
    k.beta = z * iopz;
    k.g_rr = opz;
    k.g_rp = -a * s2 * opz;
    k.g_tt = rho2;
    k.g_pp = Sigma * s2 * irho2;
    k.h_rr = ra2 * irho2 - k.beta;
    k.h_rp = a * irho2;
    k.h_tt = irho2;
    k.h_pp = irho2 * is2;
    k.sqrtg = rho2 * s * sq;
}

// exp(x), sin(y), cos(y) for the small offsets of the predictor-corrector
// points from a particle's start cell: Taylor polynomials, within an ulp or
// two for |x|, |y| <= kSmallArg.  A point of a step is less than two cells
// from its start cell's corner (a move is below one cell), so grids with
// 2 dlnr and 2 dth <= kSmallArg use them; coarser grids use the library
// functions (a grid-uniform choice).  Grids with 2 dlnr and 2 dth <=
// kTinyArg take shorter series (exp to x^5, sin to y^5, cos to y^4; the
// first omitted term is below a quarter ulp there).
constexpr double kSmallArg = 0.07;
constexpr double kTinyArg = 0.005;
// Within ~5.7 degrees of a pole (anchor sin(theta) < kPoleSin) sin and cos
// are taken from theta = eta * dth directly: there the centrifugal terms
// (gamma^phph ~ 1/sin^2) amplify how sin(theta) is rounded, and this keeps
// the rounding the same as in the plain formula.
constexpr double kPoleSin = 0.1;

// SHORT selects the short series (a launch-uniform choice made once per
// particle step, so that each variant is straight-line code).
template <bool SHORT, class R>
__device__ __forceinline__ R exp_small(R x) {
    if constexpr (std::is_same<R, float>::value) {
        // float: the series cut where the next term is below 1e-9 (|x| <= kSmallArg)
        float p = 1.0f / 120.0f;
        p = fmaf(p, x, 1.0f / 24.0f);
        p = fmaf(p, x, 1.0f / 6.0f);
        p = fmaf(p, x, 0.5f);
        p = fmaf(p, x, 1.0f);
        return fmaf(p, x, 1.0f);
    } else {
        R p = R(1.0 / 120.0);
        if constexpr (!SHORT) {
            p = R(1.0 / 3628800.0);
            p = fma(p, x, R(1.0 / 362880.0));
            p = fma(p, x, R(1.0 / 40320.0));
            p = fma(p, x, R(1.0 / 5040.0));
            p = fma(p, x, R(1.0 / 720.0));
            p = fma(p, x, R(1.0 / 120.0));
        }
        p = fma(p, x, R(1.0 / 24.0));
        p = fma(p, x, R(1.0 / 6.0));
        p = fma(p, x, R(0.5));
        p = fma(p, x, R(1.0));
        return fma(p, x, R(1.0));
    }
}

template <bool SHORT, class R>
__device__ __forceinline__ void sincos_small(R y, R& sn, R& cs) {
    const R y2 = y * y;
    if constexpr (std::is_same<R, float>::value) {
        const float ps = fmaf(1.0f / 120.0f, y2, -1.0f / 6.0f);
        sn = fmaf(ps * y2, y, y);
        const float pc = fmaf(1.0f / 24.0f, y2, -0.5f);
        cs = fmaf(pc, y2, 1.0f);
    } else {
        R ps = R(1.0 / 120.0), pc = R(1.0 / 24.0);
        if constexpr (!SHORT) {
            ps = R(1.0 / 362880.0);
            ps = fma(ps, y2, R(-1.0 / 5040.0));
            ps = fma(ps, y2, R(1.0 / 120.0));
            pc = R(-1.0 / 3628800.0);
            pc = fma(pc, y2, R(1.0 / 40320.0));
            pc = fma(pc, y2, R(-1.0 / 720.0));
            pc = fma(pc, y2, R(1.0 / 24.0));
        }
        ps = fma(ps, y2, R(-1.0 / 6.0));
        sn = fma(ps * y2, y, y);
        pc = fma(pc, y2, R(-0.5));
        cs = fma(pc, y2, R(1.0));
    }
}

// r, sin(theta), cos(theta) at the corner (ci, cj) of a particle's start
// cell; points of the step are reached from it by small offsets.
template <class R>
struct Anchor {
    R r, s, c;
    int ci, cj;
};

// Computed in double for either R, so an anchor does not depend on where it
// was evaluated (per particle, or once per tile and shared through LDS).
__device__ __forceinline__ double anchor_r(const StepArgs& A, int ci) { return exp(A.lnr0 + (double)ci * A.dlnr); }
__device__ __forceinline__ void anchor_sc(const StepArgs& A, int cj, double& s, double& c) {
    sincos((double)cj * A.dth, &s, &c);
}
__device__ __forceinline__ void anchor_values(const StepArgs& A, int ci, int cj, double& r, double& s, double& c) {
    r = anchor_r(A, ci);
    anchor_sc(A, cj, s, c);
}

template <class R>
__device__ __forceinline__ Anchor<R> make_anchor(const StepArgs& A, int ci, int cj) {
    Anchor<R> an;
    an.ci = ci;
    an.cj = cj;
    if (A.small_steps) {
        double r, s, c;
        anchor_values(A, ci, cj, r, s, c);
        an.r = R(r);
        an.s = R(s);
        an.c = R(c);
    } else {
        an.r = an.s = an.c = R(0);
    }
    return an;
}

// r, sin(theta), cos(theta) of the point (xi, eta) in grid units.
template <bool SHORT, class R>
__device__ __forceinline__ void point_at(const StepArgs& A, const Anchor<R>& an, R xi, R eta, R& r, R& s, R& c) {
    if (A.small_steps) {
        r = an.r * exp_small<SHORT>((xi - R(an.ci)) * R(A.dlnr));
        if (an.s >= R(kPoleSin)) {
            R sy, cy;
            sincos_small<SHORT>((eta - R(an.cj)) * R(A.dth), sy, cy);
            s = fma(an.s, cy, an.c * sy);
            c = fma(an.c, cy, -(an.s * sy));
        } else {
            const R th = eta * R(A.dth);
            s = sin(th);
            c = cos(th);
        }
    } else {
        r = exp(R(A.lnr0) + xi * R(A.dlnr));
        const R th = eta * R(A.dth);
        s = sin(th);
        c = cos(th);
    }
}

// Same from offsets (dxi, deta) relative to the anchor cell's corner (the
// split-precision path integrates positions this way: in float an absolute
// xi near 2000 would carry an ulp of 1e-4 cells).
template <bool SHORT, class R>
__device__ __forceinline__ void point_rel(const StepArgs& A, const Anchor<R>& an, R dxi, R deta, R& r, R& s, R& c) {
    if (A.small_steps) {
        r = an.r * exp_small<SHORT>(dxi * R(A.dlnr));
        if (an.s >= R(kPoleSin)) {
            R sy, cy;
            sincos_small<SHORT>(deta * R(A.dth), sy, cy);
            s = fma(an.s, cy, an.c * sy);
            c = fma(an.c, cy, -(an.s * sy));
            return;
        }
    } else {
        r = exp(R(A.lnr0) + (R(an.ci) + dxi) * R(A.dlnr));
    }
    const R th = (R(an.cj) + deta) * R(A.dth);
    s = sin(th);
    c = cos(th);
}

// Geodesic right-hand side of eq. particle-eom (no Lorentz force) in grid
// units at the point with radius r and polar angle of sine s, cosine c:
// f = (dxi/dt, deta/dt, dphi/dt, du_r/dt, du_th/dt), du_ph/dt = 0.  App. A's
// lapse, shift and gamma^ij and their r and theta derivatives are
// substituted into it, so that it takes two hardware estimates:
//  - with Q = rho^2 + 2Mr = rho^2 (1 + z), the reciprocals of r, sin^2,
//    rho^2 and Q come from one reciprocal of r sin^2 rho^2 Q (double; float
//    takes two, of r sin^2 and of rho^2 Q, to stay in range);
//  - u^0 = sqrt(eps + u^2)/alpha = sqrt((eps + u^2) Q / rho^2) and 1/u^0 come
//    from one square root;
//  - alpha = (1+z)^(-1/2) and beta^r = z/(1+z) = 2Mr/Q give -alpha u^0
//    d alpha = u^0 d beta^r / 2, with d beta^r = 2M (rho^2 - 2r^2)/Q^2 in r
//    and 4 M a^2 r sin cos / Q^2 in theta;
//  - the gamma^ij derivatives share their factor 1/rho^4, so the quadratic
//    form u_i u_j d gamma^ij is summed inside it.
template <class R>
__device__ __forceinline__ void geodesic_rhs_point(const StepArgs& A, R eps, R r, R s, R c,
                                                   R ur, R ut, R up, R f[5]) {
    const R a = R(A.a), M = R(A.M);
    const R a2 = a * a, r2 = r * r, s2 = s * s;
    const R rho2 = r2 + a2 * (c * c);
    const R tMr = R(2) * M * r;
    const R Q = rho2 + tMr;
    const R rs2 = r * s2, rQ = rho2 * Q;
    R x1, x2;                                           // 1/(r sin^2), 1/(rho^2 Q)
    if constexpr (std::is_same<R, float>::value) {
        x1 = rcp(rs2);
        x2 = rcp(rQ);
    } else {
        const R iP = rcp(rs2 * rQ);
        x1 = rQ * iP;
        x2 = rs2 * iP;
    }
    const R ir = s2 * x1, is2 = r * x1;
    const R irho2 = Q * x2, iQ = rho2 * x2;
    const R beta = tMr * iQ;
    const R ra2 = r2 + a2;
    const R aur = a * ur;
    const R uu = irho2 * (ra2 * ur * ur + R(2) * aur * up + ut * ut + is2 * up * up) - beta * ur * ur;
    R u0, iu0;
    sqrt_rsqrt((eps + uu) * (Q * irho2), u0, iu0);
    f[0] = (irho2 * (ra2 * ur + a * up) * iu0 - beta * fma(ur, iu0, R(1))) * ir * R(A.idlnr);
    f[1] = irho2 * ut * iu0 * R(A.idth);
    f[2] = irho2 * (aur + is2 * up) * iu0;
    const R iQ2 = iQ * iQ, irho4 = irho2 * irho2;
    const R sc = s * c;
    const R dbe0 = R(2) * M * (rho2 - R(2) * r2) * iQ2;
    const R dbe1 = R(4) * M * a2 * r * sc * iQ2;
    const R ur2 = ur * ur, up2 = up * up, ut2 = ut * ut;
    const R quad0 = R(-2) * r * irho4 * (a2 * s2 * ur2 + R(2) * aur * up + ut2 + is2 * up2) - ur2 * dbe0;
    const R quad1 = R(2) * sc * irho4 * (a2 * (ra2 * ur2 + R(2) * aur * up + ut2) - (rho2 - a2 * s2) * is2 * is2 * up2)
                  - ur2 * dbe1;
    const R hu0 = R(0.5) * u0 + ur, hiu0 = R(0.5) * iu0;
    f[3] = dbe0 * hu0 - quad0 * hiu0;
    f[4] = dbe1 * hu0 - quad1 * hiu0;
}

// Same, evaluating the metric at (xi, eta) from the anchor.
template <bool SHORT, class R>
__device__ __forceinline__ void geodesic_rhs(const StepArgs& A, const Anchor<R>& an, R eps, R xi, R eta,
                                             R ur, R ut, R up, R f[5]) {
    R r, s, c;
    point_at<SHORT>(A, an, xi, eta, r, s, c);
    geodesic_rhs_point(A, eps, r, s, c, ur, ut, up, f);
}

// (v x w)_i = sqrt(gamma) eps_ijk v^j w^k; v covariant (raised here), w contravariant.
template <class R>
__device__ __forceinline__ void cross_lower(const Metric<R>& k, const R v[3], const R w[3], R o[3]) {
    const R vr = k.h_rr * v[0] + k.h_rp * v[2];
    const R vt = k.h_tt * v[1];
    const R vp = k.h_rp * v[0] + k.h_pp * v[2];
    o[0] = k.sqrtg * (vt * w[2] - vp * w[1]);
    o[1] = k.sqrtg * (vp * w[0] - vr * w[2]);
    o[2] = k.sqrtg * (vr * w[1] - vt * w[0]);
}

// Full-step generalised Boris kick (eqs. boris-plus-minus, u0bar, boris-scheme).
template <class R>
__device__ __forceinline__ void boris_kick(const Metric<R>& k, R qm, R dt, const R D[3], const R B[3], R u[3]) {
    const R Dl[3] = {k.g_rr * D[0] + k.g_rp * D[2], k.g_tt * D[1], k.g_rp * D[0] + k.g_pp * D[2]};
    const R h = qm * k.alpha * dt * R(0.5);
    R um[3];
    for (int i = 0; i < 3; ++i) um[i] = u[i] + h * Dl[i];
    const R uu = k.h_rr * um[0] * um[0] + R(2) * k.h_rp * um[0] * um[2]
               + k.h_tt * um[1] * um[1] + k.h_pp * um[2] * um[2];
    R su, rsu;
    sqrt_rsqrt(R(1) + uu, su, rsu);
    const R tf = qm * dt * R(0.5) * rsu * k.alpha;            // q/m dt / (2 u0bar), u0bar = sqrt(1 + u^2)/alpha
    const R t[3] = {tf * B[0], tf * B[1], tf * B[2]};
    const R tt = k.g_rr * t[0] * t[0] + R(2) * k.g_rp * t[0] * t[2]
               + k.g_tt * t[1] * t[1] + k.g_pp * t[2] * t[2];
    R x[3], ut[3], sv[3];
    cross_lower(k, um, t, x);
    for (int i = 0; i < 3; ++i) ut[i] = um[i] + x[i];
    const R sf = R(2) * rcp(R(1) + tt);
    for (int i = 0; i < 3; ++i) sv[i] = sf * t[i];
    cross_lower(k, ut, sv, x);
    for (int i = 0; i < 3; ++i) u[i] = um[i] + x[i] + h * Dl[i];
}

// Momentum kick variants of the particle step.
enum Kick { kBoris = 0, kVay = 1 };

// Vay's momentum update (Vay 2008) in the FIDO frame, the alternative
// kick of Sec. 2.2: the FIDO measures D, B and u_i and its clock advances
// alpha dt, so with h = (q/m) alpha dt / 2, dot products as gamma
// contractions and cross products with e_ijk:
//   u' = u + h (D + (u / gamma) x B) + h D;  tau = h B;
//   gamma_new^2 = (sigma + sqrt(sigma^2 + 4 (tau^2 + (u'.tau)^2))) / 2,
//   sigma = 1 + u'^2 - tau^2 (the Lorentz factor that makes
//   u_new = u' + (u_new / gamma_new) x tau solvable);
//   t = tau / gamma_new, u_new = (u' + (u'.t) t + u' x t) / (1 + t^2).
template <class R>
__device__ __forceinline__ void vay_kick(const Metric<R>& k, R qm, R dt, const R D[3], const R B[3], R u[3]) {
    const R Dl[3] = {k.g_rr * D[0] + k.g_rp * D[2], k.g_tt * D[1], k.g_rp * D[0] + k.g_pp * D[2]};
    const R h = qm * k.alpha * dt * R(0.5);
    const R uu = k.h_rr * u[0] * u[0] + R(2) * k.h_rp * u[0] * u[2]
               + k.h_tt * u[1] * u[1] + k.h_pp * u[2] * u[2];
    R gam, rgam;
    sqrt_rsqrt(R(1) + uu, gam, rgam);
    const R v[3] = {u[0] * rgam, u[1] * rgam, u[2] * rgam};
    R x[3], up[3];
    cross_lower(k, v, B, x);
    for (int i = 0; i < 3; ++i) up[i] = (u[i] + h * (Dl[i] + x[i])) + h * Dl[i];
    const R tau[3] = {h * B[0], h * B[1], h * B[2]};
    const R tau2 = k.g_rr * tau[0] * tau[0] + R(2) * k.g_rp * tau[0] * tau[2]
                 + k.g_tt * tau[1] * tau[1] + k.g_pp * tau[2] * tau[2];
    const R w = up[0] * tau[0] + up[1] * tau[1] + up[2] * tau[2];
    const R upup = k.h_rr * up[0] * up[0] + R(2) * k.h_rp * up[0] * up[2]
                 + k.h_tt * up[1] * up[1] + k.h_pp * up[2] * up[2];
    const R sigma = R(1) + upup - tau2;
    R sd, rsd;
    sqrt_rsqrt(sigma * sigma + R(4) * (tau2 + w * w), sd, rsd);   // > 0: sigma >= 1 when tau = 0
    R gn, rgn;
    sqrt_rsqrt(R(0.5) * (sigma + sd), gn, rgn);                     // gamma_new >= 1
    const R t[3] = {tau[0] * rgn, tau[1] * rgn, tau[2] * rgn};
    const R s = rcp(R(1) + tau2 * rgn * rgn);
    const R ut = w * rgn;                                          // u'_k t^k
    const R tl[3] = {k.g_rr * t[0] + k.g_rp * t[2], k.g_tt * t[1], k.g_rp * t[0] + k.g_pp * t[2]};
    cross_lower(k, up, t, x);
    for (int i = 0; i < 3; ++i) u[i] = s * (up[i] + ut * tl[i] + x[i]);
}

template <int KICK, class R>
__device__ __forceinline__ void kick(const Metric<R>& k, R qm, R dt, const R D[3], const R B[3], R u[3]) {
    if constexpr (KICK == kVay) vay_kick(k, qm, dt, D, B, u);
    else boris_kick(k, qm, dt, D, B, u);
}

// CIC weights W(d - a) = max(0, 1 - |d - a|) of the vertices a = 0, 1, 2 of
// a move's window, for an end point at d = x - i0 in [0, 2) from the
// window's first vertex: with e = d - 1 they are max(0, -e), 1 - |e| and
// max(0, e).  d - 1 and d - 2 are exact (d is a multiple of x's ulp, below
// 2), so these are the values of the plain formula, bit for bit.
__device__ __forceinline__ void cic_window_weights(double d, double w[3]) {
    const double e = d - 1.0;
    w[0] = fmax(0.0, -e);
    w[1] = 1.0 - fabs(e);
    w[2] = fmax(0.0, e);
}

// One particle move to deposit: charge q w, start and end point in grid
// units, phi advance, and the lower corner (i0, j0) = (floor(min xi),
// floor(min eta)) of its 3x3 vertex window.
struct Move {
    double qw, xi0, eta0, xi1, eta1, dphi;
    int i0, j0;
};

__device__ __forceinline__ Move make_move(double qw, double xi0, double eta0, double xi1, double eta1, double dphi) {
    Move m;
    m.qw = qw;
    m.xi0 = xi0;
    m.eta0 = eta0;
    m.xi1 = xi1;
    m.eta1 = eta1;
    m.dphi = dphi;
    m.i0 = (int)floor(fmin(xi0, xi1));
    m.j0 = (int)floor(fmin(eta0, eta1));
    return m;
}

// Esirkepov fluxes of a move on its 3x3 vertex window (eqs. esirkepov-decomp,
// j-phi-deposit, with the local prefix sum), handed to add(component, i, j,
// value) as they are formed: 6 F^r through (i0+a+1/2, j0+b), 6 F^th through
// (i0+a, j0+b+1/2), 9 G^ph = J^ph dV at (i0+a, j0+b).
// With CIC shapes S_ab = wx_a wy_b the decomposition factorises:
//   W^r_ab = (wx1_a - wx0_a)(wy0_b + wy1_b)/2,  W^th_ab = (wx0_a + wx1_a)(wy1_b - wy0_b)/2,
// so the prefix sums over a (resp. b) act on one factor only, and
//   S11/3 + S10/6 + S01/6 + S00/3 = (wx1_a (2 wy1_b + wy0_b) + wx0_a (wy1_b + 2 wy0_b))/6.
// The same values as the term-by-term form, up to rounding.
template <class Add>
__device__ __forceinline__ void esirkepov(const Move& m, double idt, Add&& add) {
    double wx0[3], wx1[3], wy0[3], wy1[3];
    const double fi0 = (double)m.i0, fj0 = (double)m.j0;
    cic_window_weights(m.xi0 - fi0, wx0);
    cic_window_weights(m.xi1 - fi0, wx1);
    cic_window_weights(m.eta0 - fj0, wy0);
    cic_window_weights(m.eta1 - fj0, wy1);
    const double hf = -0.5 * m.qw * idt;                // -(q w / dt) / 2
    const double cp6 = m.qw * m.dphi * idt * (1.0 / 6.0);   // (q w dphi / dt) / 6
    // A move that stays in one cell row (column) touches vertex rows i0, i0+1
    // only, and its r-flux prefix sum is zero from the second row on (the
    // shape weights of both end points sum to 1 over those rows): those
    // values are exactly zero and are not added.  The 21 entries fall into
    // four groups by which of the two conditions they need (8 always, 5 with
    // two_r, 5 with two_t, 3 with both), so a wave branches three times.
    const bool two_r = floor(m.xi0) != floor(m.xi1), two_t = floor(m.eta0) != floor(m.eta1);
    const double fx[2] = {hf * (wx1[0] - wx0[0]), hf * ((wx1[0] - wx0[0]) + (wx1[1] - wx0[1]))};
    const double fy[2] = {hf * (wy1[0] - wy0[0]), hf * ((wy1[0] - wy0[0]) + (wy1[1] - wy0[1]))};
    double p1[3], p0[3];
    for (int b = 0; b < 3; ++b) {
        p1[b] = cp6 * fma(2.0, wy1[b], wy0[b]);
        p0[b] = cp6 * fma(2.0, wy0[b], wy1[b]);
    }
    // F^r through (i0+a+1/2, j0+b), F^th through (i0+b, j0+a+1/2), G^ph at (i0+a, j0+b)
    auto fr = [&](int a, int b) { add(0, m.i0 + a, m.j0 + b, fx[a] * (wy0[b] + wy1[b])); };
    auto ft = [&](int a, int b) { add(1, m.i0 + b, m.j0 + a, fy[a] * (wx0[b] + wx1[b])); };
    auto gp = [&](int a, int b) { add(2, m.i0 + a, m.j0 + b, fma(wx1[a], p1[b], wx0[a] * p0[b])); };
    fr(0, 0); fr(0, 1); ft(0, 0); ft(0, 1);
    gp(0, 0); gp(1, 0); gp(0, 1); gp(1, 1);
    if (two_r) {
        fr(1, 0); fr(1, 1); ft(0, 2);
        gp(2, 0); gp(2, 1);
    }
    if (two_t) {
        fr(0, 2); ft(1, 0); ft(1, 1);
        gp(0, 2); gp(1, 2);
    }
    if (two_r && two_t) {
        fr(1, 2); ft(1, 2);
        gp(2, 2);
    }
}

// Third-order shape (the spline option of Sec. 2.3): the cubic B-spline,
// W(d) = 2/3 - d^2 + |d|^3 / 2 for |d| < 1, (2 - |d|)^3 / 6 for 1 <= |d| < 2,
// zero beyond; four vertices carry a particle.
__device__ __forceinline__ double shape3(double x) {
    const double a = fabs(x);
    const double y = 2.0 - a;
    const double outer = y * y * y * (1.0 / 6.0);
    const double inner = fma(a * a, fma(0.5, a, -1.0), 2.0 / 3.0);
    return a >= 2.0 ? 0.0 : (a >= 1.0 ? outer : inner);
}

// Columns beyond an axis fold onto their mirror (axisymmetry: (r, -theta,
// phi) is (r, theta, phi + pi)).  Vertex columns keep the value (charge,
// J^r, J^ph are even); theta-face columns (j + 1/2) change sign (J^th is
// odd).  Every vertex keeps its discrete continuity.
__device__ __forceinline__ int fold_vertex(int j, int nth) { return j < 0 ? -j : (j > nth ? 2 * nth - j : j); }
__device__ __forceinline__ int fold_face(int j, int nth, double& sign) {
    sign = (j < 0 || j >= nth) ? -1.0 : 1.0;
    return j < 0 ? -j - 1 : (j >= nth ? 2 * nth - 1 - j : j);
}

// Esirkepov fluxes of a move with the cubic shape on the 5 x 5 vertex window
// (lower corner floor(min xi) - 1, floor(min eta) - 1) that holds both
// supports, in the factorised form of the CIC version, folded across the
// axes and handed to add(component, i, j, value): 20 F^r, 20 F^th, 25 G^ph.
// The theta-direction weights are formed one window column at a time (the
// F^th prefix sum runs along with them), so only the five r-direction
// weights of each end point and their prefix sums stay live.
template <class Add>
__device__ __forceinline__ void esirkepov3(const Move& m, double idt, int nth, Add&& add) {
    const int i0 = (int)floor(fmin(m.xi0, m.xi1)) - 1, j0 = (int)floor(fmin(m.eta0, m.eta1)) - 1;
    double wx0[5], wx1[5];
    for (int a = 0; a < 5; ++a) {
        wx0[a] = shape3(m.xi0 - (double)(i0 + a));
        wx1[a] = shape3(m.xi1 - (double)(i0 + a));
    }
    const double hf = -0.5 * m.qw * idt;
    const double cp6 = m.qw * m.dphi * idt * (1.0 / 6.0);
    double fx[4], runx = 0.0, runy = 0.0;
    for (int a = 0; a < 4; ++a) {
        runx += wx1[a] - wx0[a];
        fx[a] = hf * runx;
    }
    for (int b = 0; b < 5; ++b) {
        const double wy0 = shape3(m.eta0 - (double)(j0 + b)), wy1 = shape3(m.eta1 - (double)(j0 + b));
        const int jv = fold_vertex(j0 + b, nth);
        const double sy = wy0 + wy1;
        const double p1 = cp6 * fma(2.0, wy1, wy0), p0 = cp6 * fma(2.0, wy0, wy1);
        for (int a = 0; a < 4; ++a) add(0, i0 + a, jv, fx[a] * sy);
        for (int a = 0; a < 5; ++a) add(2, i0 + a, jv, fma(wx1[a], p1, wx0[a] * p0));
        if (b < 4) {
            runy += wy1 - wy0;
            const double fy = hf * runy;
            double sg;
            const int jf = fold_face(j0 + b, nth, sg);
            for (int a = 0; a < 5; ++a) add(1, i0 + a, jf, sg * fy * (wx0[a] + wx1[a]));
        }
    }
}

// n / d for 0 <= n < 2^31 and d > 0, from the double product n * (1/d)
// (within 2^-21 of the quotient, so truncation is off by at most one) and
// one correction on the remainder; cheaper than the integer division
// sequence, for a divisor known only at run time.
__device__ __forceinline__ int div_by(int n, int d, double inv_d) {
    int q = (int)((double)n * inv_d);
    const int64_t r = (int64_t)n - (int64_t)q * d;
    q += (r >= d) - (r < 0);
    return q;
}

// Element index of vertex (i, j) in a grid array; every grid array is below
// 4 GiB (checked at the boundary), so indices and byte offsets fit in 32 bits.
__device__ __forceinline__ uint32_t grid_index(const StepArgs& A, int i, int j) {
    return (uint32_t)((i + A.guard) * A.pitch + (j + A.guard));
}

// Element idx of an array from a workgroup-uniform base by a 32-bit byte
// offset, which the loads and stores take as a scalar base register plus a
// vector offset (no 64-bit address arithmetic per lane).
template <class T>
__device__ __forceinline__ T* elem(T* base, uint32_t idx) {
    return reinterpret_cast<T*>(reinterpret_cast<typename std::conditional<std::is_const<T>::value, const char, char>::type*>(base) +
                                idx * (uint32_t)sizeof(T));
}

}  // namespace grpic
