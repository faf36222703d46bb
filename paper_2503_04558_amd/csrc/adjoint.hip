// adjoint.hip -- checkpoints of the forward push and the reverse sweep of K
// push + deposit steps (FP64).
//
// The loss is L = sum over steps n and particles of
// lambda . (F^r, F^th, G^ph)_n, lambda being given per grid element (the
// cotangent of the accumulated current).  Particles are independent given the
// fields, so the reverse sweep runs one thread per particle:
//   for each checkpoint segment, last first:
//     recompute the segment's start-of-step states from its checkpoint
//     (stored in the workspace), then for each step of the segment, last
//     first: replay the step into a tape and run its reverse
//     (grpic_adjoint.hpp), carrying the state cotangent in registers and
//     adding field cotangents to the gradient arrays with FP64 atomics.
// d L / d u_i(0) is the state cotangent left after the first step.
#include "grpic_adjoint.hpp"
#include "grpic_launch.hpp"

namespace grpic {

// Checkpoint slot layout: cell (int32, padded to 8 bytes) then xr, xth, ur,
// uth, uph (double), each n long.
static inline __host__ __device__ size_t slot_cell_bytes(int64_t n) { return ((size_t)n * 4 + 7) / 8 * 8; }
size_t checkpoint_slot_bytes(int64_t n) { return slot_cell_bytes(n) + (size_t)n * 5 * 8; }
int adj_max_corr() { return adj::kMaxCorr; }

__global__ __launch_bounds__(256) void save_state(const StepArgs A, char* slot) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.n) return;
    int32_t* cell = reinterpret_cast<int32_t*>(slot);
    double* d = reinterpret_cast<double*>(slot + slot_cell_bytes(A.n));
    cell[p] = A.cell[p];
    const double* src[5] = {static_cast<const double*>(A.xr), static_cast<const double*>(A.xth),
                            static_cast<const double*>(A.ur), static_cast<const double*>(A.uth),
                            static_cast<const double*>(A.uph)};
    for (int k = 0; k < 5; ++k) d[(int64_t)k * A.n + p] = src[k][p];
}

hipError_t launch_save_state(const StepArgs& A, void* slot, hipStream_t stream) {
    if (A.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(save_state, dim3((unsigned)((A.n + 255) / 256)), dim3(256), 0, stream, A,
                       static_cast<char*>(slot));
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void push_deposit_backward_f64(const BackArgs B) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= B.n) return;
    const int64_t n = B.n;
    const adj::Geo G{B.a, B.M, B.lnr0, B.dlnr, B.dth, B.nr, B.nth, B.guard, B.pitch};
    const int s = B.sp[p];
    double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (s < B.nsp) {
        const bool massless = B.massless[s] != 0;
        const double qm = massless ? 0.0 : B.q[s] / B.m[s];
        const double qw = B.q[s] * B.w[p];
        const int C = B.ckpt_every;
        const int nseg = B.nsteps / C;
        double* ws = B.ws;                                       // [m][component][particle]
        for (int seg = nseg - 1; seg >= 0; --seg) {
            const char* slot = static_cast<const char*>(B.ckpt) + (size_t)seg * B.slot_bytes;
            const int32_t cell = reinterpret_cast<const int32_t*>(slot)[p];
            const double* sd = reinterpret_cast<const double*>(slot + slot_cell_bytes(n));
            bool alive = cell >= 0 && cell < B.nr * B.nth;
            double xi = 0.0, eta = 0.0, u[3] = {0.0, 0.0, 0.0};
            if (alive) {
                const double xr = sd[p], xth = sd[n + p];
                alive = xr >= 0.0 && xr <= 1.0 && xth >= 0.0 && xth <= 1.0;
                xi = (double)(cell / B.nth) + xr;
                eta = (double)(cell % B.nth) + xth;
                u[0] = sd[2 * n + p];
                u[1] = sd[3 * n + p];
                u[2] = sd[4 * n + p];
            }
            // start-of-step states of the segment (xi = NaN marks a removed particle)
            for (int m = 0; m < C; ++m) {
                double* w = ws + (size_t)m * 5 * n;
                w[p] = alive ? xi : NAN;
                w[n + p] = eta;
                w[2 * n + p] = u[0];
                w[3 * n + p] = u[1];
                w[4 * n + p] = u[2];
                if (!alive) continue;
                adj::StepTape T;
                const int st = adj::replay_step(G, B.F, qm, massless, B.dt, B.ncorr, xi, eta, u, T);
                if (st != adj::ST_ALIVE) { alive = false; continue; }
                xi = T.xi1;
                eta = T.eta1;
                u[0] = T.y[3];
                u[1] = T.refl ? -T.y[4] : T.y[4];
                u[2] = T.up[2];
            }
            for (int m = C - 1; m >= 0; --m) {
                const double* w = ws + (size_t)m * 5 * n;
                const double x0 = w[p];
                if (isnan(x0)) continue;
                const double u0[3] = {w[2 * n + p], w[3 * n + p], w[4 * n + p]};
                adj::StepTape T;
                adj::replay_step(G, B.F, qm, massless, B.dt, B.ncorr, x0, w[n + p], u0, T);
                adj::reverse_step(G, B.F, B.lam, qm, massless, qw, B.dt, B.ncorr, T, a,
                                  [&](int c, long e, double v) { atomicAdd(B.gradF[c] + e, v); });
            }
        }
    }
    B.grad_u[0][p] = a[2];
    B.grad_u[1][p] = a[3];
    B.grad_u[2][p] = a[4];
}

hipError_t launch_push_deposit_backward(const BackArgs& B, hipStream_t stream) {
    if (B.n <= 0) return hipSuccess;
    hipLaunchKernelGGL(push_deposit_backward_f64, dim3((unsigned)((B.n + 255) / 256)), dim3(256), 0, stream, B);
    return hipGetLastError();
}

}  // namespace grpic
