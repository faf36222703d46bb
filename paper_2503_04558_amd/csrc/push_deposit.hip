// push_deposit.hip -- FP64 push + deposit kernels and the charge kernel.
//
// Per particle and step (Sec. 2.2-2.3 of arXiv:2503.04558): CIC gather of the
// six staggered field components at x^n, a full-step generalised Boris kick
// at x^n, the geodesic predictor and `ncorr` trapezoid corrector passes, axis
// reflection, Esirkepov deposit of the move on a 3x3 vertex window, and
// removal at the radial edges.
//
// Two kernels share that body:
//   push_deposit_f64        one thread per particle, any particle order,
//                           deposit with global FP64 atomics;
//   push_deposit_f64_tiled  one workgroup per slice of a cell-sorted tile
//                           (see grpic_launch.hpp), deposit into an LDS
//                           window with LDS FP64 atomics, one flush of the
//                           window's non-zero entries to global memory.
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

struct Events {
    int live, out, bad, refl, spill;
};

// Advances live particle p by one step in place.  Returns true when the move
// is to be deposited (mv filled), false when the particle was or became
// removed without a deposit.
__device__ __forceinline__ bool advance_f64(const StepArgs& A, int64_t p, MoveFlux& mv, Events& ev) {
    const int cell = A.cell[p];
    if (cell < 0) return false;
    ev.live = 1;
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
        ev.bad = 1;
        A.cell[p] = -1;
        return false;
    }
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
        ev.bad = 1;
        A.cell[p] = -1;
        return false;
    }
    if (eta1 < 0.0) { eta1 = -eta1; u1t = -u1t; ev.refl = 1; }
    else if (eta1 > (double)A.nth) { eta1 = 2.0 * A.nth - eta1; u1t = -u1t; ev.refl = 1; }
    esirkepov(A.q[s] * w[p], dt, xi0, eta0, xi1, eta1, yt[2], mv);
    if (A.phi) static_cast<double*>(A.phi)[p] += yt[2];
    if (xi1 < 0.0 || xi1 >= (double)A.nr) {
        ev.out = 1;
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
    return true;
}

__device__ __forceinline__ void scatter_global(const StepArgs& A, const MoveFlux& mv) {
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) atomicAdd(A.Fr + grid_index(A, mv.i0 + a, mv.j0 + b), mv.Fr[a][b]);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 2; ++b) atomicAdd(A.Fth + grid_index(A, mv.i0 + a, mv.j0 + b), mv.Ft[a][b]);
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) atomicAdd(A.Gph + grid_index(A, mv.i0 + a, mv.j0 + b), mv.Gp[a][b]);
}

// Adds the wave's event counts to the global counters (all lanes of the wave
// must call it).
__device__ __forceinline__ void count_events(const StepArgs& A, const Events& ev) {
    if (!A.counters) return;
    const unsigned long long bl = __ballot(ev.live), bo = __ballot(ev.out);
    const unsigned long long bb = __ballot(ev.bad), br = __ballot(ev.refl);
    if ((threadIdx.x & 63) == 0) {
        if (bo) atomicAdd(A.counters + 0, (unsigned long long)__popcll(bo));
        if (bb) atomicAdd(A.counters + 1, (unsigned long long)__popcll(bb));
        if (br) atomicAdd(A.counters + 2, (unsigned long long)__popcll(br));
        if (bl) atomicAdd(A.counters + 3, (unsigned long long)__popcll(bl));
    }
}

__global__ __launch_bounds__(256) void push_deposit_f64(const StepArgs A) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    Events ev = {0, 0, 0, 0, 0};
    if (p < A.n) {
        MoveFlux mv;
        if (advance_f64(A, p, mv, ev)) scatter_global(A, mv);
    }
    count_events(A, ev);
}

// Sum over the 64 lanes of a wave.
__device__ __forceinline__ int wave_sum(int v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

__global__ __launch_bounds__(kPushThreads) void push_deposit_f64_tiled(const StepArgs A, const TilingHeader* hdr,
                                                                       const Slice* __restrict__ slices,
                                                                       int64_t slice_cap) {
    __shared__ double win[3][kWinRows][kWinCols];
    // XCD-aware order: workgroup b runs on XCD b % 8; give each XCD a
    // contiguous band of slices so neighbouring tiles share its L2.
    const int64_t nslices = hdr->nslices;
    const int64_t per_xcd = (nslices + 7) / 8;
    // (workgroups past 8 * per_xcd would alias the next XCD's band: they exit)
    if ((int64_t)(blockIdx.x / 8) >= per_xcd) return;          // uniform across the workgroup
    const int64_t logical = (int64_t)(blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
    if (logical >= nslices || logical >= slice_cap) return;
    const Slice sl = slices[logical];
    if (sl.start < 0 || sl.len <= 0) return;
    const int tpr = (A.nth + kTileCells - 1) / kTileCells;
    const int ti = sl.tile / tpr;
    const int j_lo = (sl.tile - ti * tpr) * kTileCells;
    const int wi0 = ti - kMarginRows - 1;                // window origin (vertex indices)
    const int wj0 = j_lo - kMarginCols - 1;

    double* wflat = &win[0][0][0];
    for (int e = threadIdx.x; e < 3 * kWinRows * kWinCols; e += kPushThreads) wflat[e] = 0.0;
    __syncthreads();

    Events tot = {0, 0, 0, 0, 0};
    const int64_t end = sl.start + sl.len < A.n ? sl.start + sl.len : A.n;
    for (int k = 0; k < kPushIter; ++k) {
        // lanes of a wave take particles kPushIter apart, so that they fall
        // in different cells and their LDS atomics rarely hit one address
        const int64_t p = sl.start + k + (int64_t)kPushIter * threadIdx.x;
        if (p >= end) continue;
        MoveFlux mv;
        Events ev = {0, 0, 0, 0, 0};
        if (advance_f64(A, p, mv, ev)) {
            const int li = mv.i0 - wi0, lj = mv.j0 - wj0;
            if (li >= 0 && li + 2 < kWinRows && lj >= 0 && lj + 2 < kWinCols) {
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 3; ++b) atomicAdd(&win[0][li + a][lj + b], mv.Fr[a][b]);
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 2; ++b) atomicAdd(&win[1][li + a][lj + b], mv.Ft[a][b]);
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) atomicAdd(&win[2][li + a][lj + b], mv.Gp[a][b]);
            } else {
                scatter_global(A, mv);                   // drifted out of the window
                ev.spill = 1;
            }
        }
        tot.live += ev.live; tot.out += ev.out; tot.bad += ev.bad; tot.refl += ev.refl; tot.spill += ev.spill;
    }
    __syncthreads();
    // flush the window's non-zero entries that lie inside the grid arrays
    double* const J[3] = {A.Fr, A.Fth, A.Gph};
    const int rows_lo = -A.guard, rows_hi = A.nr + A.guard;             // inclusive vertex rows
    const int cols_lo = -A.guard, cols_hi = A.pitch - A.guard - 1;      // inclusive vertex columns
    for (int e = threadIdx.x; e < kWinRows * kWinCols; e += kPushThreads) {
        const int r = e / kWinCols, c = e - r * kWinCols;
        const int gi = wi0 + r, gj = wj0 + c;
        if (gi < rows_lo || gi > rows_hi || gj < cols_lo || gj > cols_hi) continue;
        const long g = grid_index(A, gi, gj);
        for (int a = 0; a < 3; ++a) {
            const double v = win[a][r][c];
            if (v != 0.0) atomicAdd(J[a] + g, v);
        }
    }
    if (A.counters) {
        const int l = wave_sum(tot.live), o = wave_sum(tot.out), b = wave_sum(tot.bad), f = wave_sum(tot.refl);
        const int x = wave_sum(tot.spill);
        if ((threadIdx.x & 63) == 0) {
            if (o) atomicAdd(A.counters + 0, (unsigned long long)o);
            if (b) atomicAdd(A.counters + 1, (unsigned long long)b);
            if (f) atomicAdd(A.counters + 2, (unsigned long long)f);
            if (l) atomicAdd(A.counters + 3, (unsigned long long)l);
            if (x) atomicAdd(A.counters + 4, (unsigned long long)x);
        }
    }
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

hipError_t launch_push_deposit_f64_tiled(const StepArgs& A, const void* tiling, int64_t slice_cap,
                                         hipStream_t stream) {
    if (A.n <= 0) return hipSuccess;
    const TilingHeader* hdr = static_cast<const TilingHeader*>(tiling);
    const Slice* slices = reinterpret_cast<const Slice*>(hdr + 1);
    const int64_t grid = (slice_cap + 7) / 8 * 8;
    hipLaunchKernelGGL(push_deposit_f64_tiled, dim3((unsigned)grid), dim3(kPushThreads), 0, stream, A, hdr, slices,
                       slice_cap);
    return hipGetLastError();
}

hipError_t launch_charge(const StepArgs& A, bool split, double* Q, hipStream_t stream) {
    if (A.n <= 0) return hipSuccess;
    if (split) hipLaunchKernelGGL(charge_kernel<float>, blocks_for(A.n), dim3(256), 0, stream, A, Q);
    else hipLaunchKernelGGL(charge_kernel<double>, blocks_for(A.n), dim3(256), 0, stream, A, Q);
    return hipGetLastError();
}

}  // namespace grpic
