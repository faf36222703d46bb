// grpic_backward.hpp -- the per-particle reverse sweep of K push + deposit
// steps (FP64), host/device so that it can also be run on the CPU.
#pragma once

#include "grpic_adjoint.hpp"
#include "grpic_launch.hpp"

namespace grpic {

// Checkpoint slot layout: cell (int32, padded to 8 bytes) then xr, xth, ur,
// uth, uph (double), each n long.
__host__ __device__ inline size_t slot_cell_bytes(int64_t n) { return ((size_t)n * 4 + 7) / 8 * 8; }
constexpr int kFastCorr = 3;           // the paper's corrector count gets a kernel with a tape of its size

// Could lambda be non-zero on vertices i in [i_lo, i_hi], j in [j_lo, j_hi]
// (grid vertex indices, guards not included)?
__host__ __device__ inline bool lam_in_box(const BackArgs& B, int i_lo, int i_hi, int j_lo, int j_hi) {
    i_lo = max(i_lo + B.guard, 0);
    i_hi = min(i_hi + B.guard, B.rows - 1);
    j_lo = max(j_lo + B.guard, 0);
    j_hi = min(j_hi + B.guard, B.pitch - 1);
    if (i_lo > i_hi || j_lo > j_hi) return false;
    return B.row_pre[i_hi + 1] > B.row_pre[i_lo] && B.col_pre[j_hi + 1] > B.col_pre[j_lo];
}

__host__ __device__ inline bool all_zero(const double a[5]) {
    return a[0] == 0.0 && a[1] == 0.0 && a[2] == 0.0 && a[3] == 0.0 && a[4] == 0.0;
}

// The reverse sweep of particle p (one thread per particle on the GPU), the
// q-th of the batch [first, first + count).
// With a zero cotangent a step (or a whole segment)
// whose deposit window(s) cannot touch a non-zero lambda contributes nothing
// and is skipped: a move is below one cell per step, so a segment of C steps
// from a checkpoint in cell (i, j) deposits only on vertices within C + 2 of it.
// Step k gathers from the field arrays B.F[c] + k fstride and its field
// cotangents go to element e + k gstride of the gradient arrays.  T is the
// storage of the step's tape (the caller's choice: registers, or the
// thread's slot of an LDS array).
template <int NC, class AddF>
__host__ __device__ inline void backward_particle(const BackArgs& B, int64_t q, AddF addF, adj::StepTape<NC>& T) {
    const int64_t n = B.n, nb = B.count;
    const int64_t p = B.first + q;
    const int ncorr = NC == kFastCorr ? kFastCorr : B.ncorr;
    const adj::Geo G{B.a, B.M, B.lnr0, B.dlnr, B.dth, B.nr, B.nth, B.guard, B.pitch, 1.0 / B.dlnr, 1.0 / B.dth};
    const int s = B.sp[p];
    double a[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (s < B.nsp) {
        const bool massless = B.massless[s] != 0;
        const double qm = massless ? 0.0 : B.q[s] / B.m[s];
        const double qw = B.q[s] * B.w[p];
        const int C = B.ckpt_every;
        const int nseg = B.nsteps / C;
        double* ws = B.ws;                                       // [m][component][batch particle]
        for (int seg = nseg - 1; seg >= 0; --seg) {
            const char* slot = static_cast<const char*>(B.ckpt) + (size_t)seg * B.slot_bytes;
            const int32_t cell = reinterpret_cast<const int32_t*>(slot)[p];
            if (cell < 0 || cell >= B.nr * B.nth) continue;       // removed before the segment
            const double* sd = reinterpret_cast<const double*>(slot + slot_cell_bytes(n));
            const double xr = sd[p], xth = sd[n + p];
            if (!(xr >= 0.0 && xr <= 1.0 && xth >= 0.0 && xth <= 1.0)) continue;
            const int ci = cell / B.nth, cj = cell - (cell / B.nth) * B.nth;
            if (all_zero(a) && !lam_in_box(B, ci - C - 1, ci + C + 2, cj - C - 1, cj + C + 2)) continue;
            double xi = (double)ci + xr, eta = (double)cj + xth;
            double u[3] = {sd[2 * n + p], sd[3 * n + p], sd[4 * n + p]};
            // start-of-step states of the segment (xi = NaN marks a removed particle)
            bool alive = true;
            for (int m = 0; m < C; ++m) {
                double* w = ws + (size_t)m * 5 * nb;
                w[q] = alive ? xi : NAN;
                w[nb + q] = eta;
                w[2 * nb + q] = u[0];
                w[3 * nb + q] = u[1];
                w[4 * nb + q] = u[2];
                if (!alive) continue;
                const size_t fo = (size_t)(seg * C + m) * B.fstride;
                const double* const Fk[6] = {B.F[0] + fo, B.F[1] + fo, B.F[2] + fo,
                                             B.F[3] + fo, B.F[4] + fo, B.F[5] + fo};
                const int st = adj::replay_step(G, Fk, qm, massless, B.dt, ncorr, xi, eta, u, T);
                if (st != adj::ST_ALIVE) { alive = false; continue; }
                xi = T.xi1;
                eta = T.eta1;
                u[0] = T.y[3];
                u[1] = T.refl ? -T.y[4] : T.y[4];
                u[2] = T.up[2];
            }
            for (int m = C - 1; m >= 0; --m) {
                const double* w = ws + (size_t)m * 5 * nb;
                const double x0 = w[q];
                if (isnan(x0)) continue;
                const double e0 = w[nb + q];
                const int fi = (int)floor(x0), fj = (int)floor(e0);
                if (all_zero(a) && !lam_in_box(B, fi - 1, fi + 2, fj - 1, fj + 2)) continue;
                const double u0[3] = {w[2 * nb + q], w[3 * nb + q], w[4 * nb + q]};
                const size_t k = (size_t)(seg * C + m);
                const size_t fo = k * B.fstride;
                const long go = (long)(k * B.gstride);
                const double* const Fk[6] = {B.F[0] + fo, B.F[1] + fo, B.F[2] + fo,
                                             B.F[3] + fo, B.F[4] + fo, B.F[5] + fo};
                adj::replay_step(G, Fk, qm, massless, B.dt, ncorr, x0, e0, u0, T);
                adj::reverse_step(G, Fk, B.lam, qm, massless, qw, B.dt, ncorr, T, a,
                                  [&](int c, long e, double g00, double g10, double g01, double g11) {
                                      addF(c, e + go, g00, g10, g01, g11);
                                  });
            }
        }
    }
    B.grad_u[0][q] = a[2];
    B.grad_u[1][q] = a[3];
    B.grad_u[2][q] = a[4];
}

}  // namespace grpic
