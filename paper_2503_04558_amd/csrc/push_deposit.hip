// push_deposit.hip -- FP64 push + deposit kernel and the charge kernel.
//
// One thread per particle.  Per step (Sec. 2.2-2.3 of arXiv:2503.04558):
// CIC gather of the six staggered field components at x^n, a full-step
// generalised Boris kick at x^n, the geodesic predictor and `ncorr`
// trapezoid corrector passes, axis reflection, Esirkepov deposit of the move
// on a 3x3 vertex window, and removal at the radial edges.
#include "grpic_device.hpp"
#include "grpic_launch.hpp"

namespace grpic {

// Bilinear interpolation in index space of the grid array F at (f, h),
// where (f, h) are grid coordinates already shifted by the stagger.
__device__ __forceinline__ double cic_f64(const double* __restrict__ F, const StepArgs& A, double f, double h) {
    const int i = (int)floor(f), j = (int)floor(h);
    const double wf = f - (double)i, wh = h - (double)j;
    const double* p = F + grid_index(A, i, j);
    return (1.0 - wf) * (1.0 - wh) * p[0] + wf * (1.0 - wh) * p[A.pitch]
         + (1.0 - wf) * wh * p[1] + wf * wh * p[A.pitch + 1];
}

__device__ __forceinline__ void scatter_global(const StepArgs& A, const MoveFlux& mv) {
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) atomicAdd(A.Fr + grid_index(A, mv.i0 + a, mv.j0 + b), mv.Fr[a][b]);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 2; ++b) atomicAdd(A.Fth + grid_index(A, mv.i0 + a, mv.j0 + b), mv.Ft[a][b]);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) atomicAdd(A.Gph + grid_index(A, mv.i0 + a, mv.j0 + b), mv.Gp[a][b]);
}

__device__ __forceinline__ void count_events(const StepArgs& A, int live, int out, int bad, int refl) {
    if (!A.counters) return;
    const unsigned long long bl = __ballot(live), bo = __ballot(out), bb = __ballot(bad), br = __ballot(refl);
    if ((threadIdx.x & 63) == 0) {
        if (bo) atomicAdd(A.counters + 0, (unsigned long long)__popcll(bo));
        if (bb) atomicAdd(A.counters + 1, (unsigned long long)__popcll(bb));
        if (br) atomicAdd(A.counters + 2, (unsigned long long)__popcll(br));
        if (bl) atomicAdd(A.counters + 3, (unsigned long long)__popcll(bl));
    }
}

__global__ __launch_bounds__(256) void push_deposit_f64(const StepArgs A) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int live = 0, out = 0, bad = 0, refl = 0;
    if (p < A.n && A.cell[p] >= 0) {
        live = 1;
        const int cell = A.cell[p];
        double* xr = static_cast<double*>(A.xr);
        double* xth = static_cast<double*>(A.xth);
        double* ur = static_cast<double*>(A.ur);
        double* uth = static_cast<double*>(A.uth);
        double* uph = static_cast<double*>(A.uph);
        const double* w = static_cast<const double*>(A.w);
        const double dxr = xr[p], dxt = xth[p];
        const int s = A.sp[p];
        // Inputs that would index outside the grid arrays are removed as bad.
        if (cell >= A.nr * A.nth || s >= A.nsp || !(dxr >= 0.0 && dxr <= 1.0 && dxt >= 0.0 && dxt <= 1.0)) {
            bad = 1;
            A.cell[p] = -1;
        } else {
            const int ci = cell / A.nth, cj = cell - ci * A.nth;
            const double xi0 = (double)ci + dxr, eta0 = (double)cj + dxt;
            double u[3] = {ur[p], uth[p], uph[p]};
            const double* const* F = reinterpret_cast<const double* const*>(A.F);
            const double D[3] = {cic_f64(F[0], A, xi0 - 0.5, eta0), cic_f64(F[1], A, xi0, eta0 - 0.5),
                                 cic_f64(F[2], A, xi0, eta0)};
            const double B[3] = {cic_f64(F[3], A, xi0, eta0 - 0.5), cic_f64(F[4], A, xi0 - 0.5, eta0),
                                 cic_f64(F[5], A, xi0 - 0.5, eta0 - 0.5)};
            const bool massless = A.massless[s] != 0;
            const double dt = A.dt;
            if (!massless) {
                double r, sn, cs;
                grid_point(A, xi0, eta0, r, sn, cs);
                Metric<double> k;
                ks_metric<double, false>(A.a, A.M, r, sn, cs, k, nullptr);
                boris_kick(k, A.q[s] / A.m[s], dt, D, B, u);
            }
            const double eps = massless ? 0.0 : 1.0;
            // geodesic predictor-corrector on y = (xi, eta, phi, u_r, u_th); u_ph is constant
            const double y0[5] = {xi0, eta0, 0.0, u[0], u[1]};
            double f0[5], f1[5], yt[5];
            geodesic_rhs(A, eps, xi0, eta0, u[0], u[1], u[2], f0);
            for (int c = 0; c < 5; ++c) yt[c] = y0[c] + dt * f0[c];
            for (int it = 0; it < A.ncorr; ++it) {
                geodesic_rhs(A, eps, yt[0], yt[1], yt[3], yt[4], u[2], f1);
                for (int c = 0; c < 5; ++c) yt[c] = y0[c] + 0.5 * dt * (f1[c] + f0[c]);
            }
            double xi1 = yt[0], eta1 = yt[1];
            double u1t = yt[4];
            const bool finite = isfinite(xi1) && isfinite(eta1) && isfinite(yt[2]) && isfinite(yt[3])
                              && isfinite(yt[4]) && isfinite(u[2]);
            if (!finite || fabs(xi1 - xi0) >= 1.0 || fabs(eta1 - eta0) >= 1.0) {
                bad = 1;
                A.cell[p] = -1;
            } else {
                if (eta1 < 0.0) { eta1 = -eta1; u1t = -u1t; refl = 1; }
                else if (eta1 > (double)A.nth) { eta1 = 2.0 * A.nth - eta1; u1t = -u1t; refl = 1; }
                MoveFlux mv;
                esirkepov(A.q[s] * w[p], dt, xi0, eta0, xi1, eta1, yt[2], mv);
                scatter_global(A, mv);
                if (A.phi) static_cast<double*>(A.phi)[p] += yt[2];
                if (xi1 < 0.0 || xi1 >= (double)A.nr) {
                    out = 1;
                    A.cell[p] = -1;
                } else {
                    const int i1 = (int)floor(xi1);
                    int j1 = (int)floor(eta1);
                    if (j1 >= A.nth) j1 = A.nth - 1;
                    A.cell[p] = i1 * A.nth + j1;
                    xr[p] = xi1 - (double)i1;
                    xth[p] = eta1 - (double)j1;
                    ur[p] = yt[3];
                    uth[p] = u1t;
                    uph[p] = u[2];
                }
            }
        }
    }
    count_events(A, live, out, bad, refl);
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

static inline dim3 blocks_for(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

hipError_t launch_push_deposit_f64(const StepArgs& A, hipStream_t stream) {
    if (A.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(push_deposit_f64, blocks_for(A.n), dim3(256), 0, stream, A);
    return hipGetLastError();
}

hipError_t launch_charge(const StepArgs& A, bool split, double* Q, hipStream_t stream) {
    if (A.n <= 0) return hipSuccess;
    if (split) hipLaunchKernelGGL(charge_kernel<float>, blocks_for(A.n), dim3(256), 0, stream, A, Q);
    else hipLaunchKernelGGL(charge_kernel<double>, blocks_for(A.n), dim3(256), 0, stream, A, Q);
    return hipGetLastError();
}

}  // namespace grpic
