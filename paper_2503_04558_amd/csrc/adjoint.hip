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
// d L / d u_i(0) is the state cotangent left after the first step.  A
// prepass marks the rows and columns where lambda is non-zero; particles and
// steps whose deposits cannot reach them while their cotangent is zero are
// skipped (exactly: their contribution is zero).
#include "grpic_backward.hpp"

namespace grpic {

size_t checkpoint_slot_bytes(int64_t n) { return slot_cell_bytes(n) + (size_t)n * 5 * 8; }
int adj_max_corr() { return adj::kMaxCorr; }

// The state before a step, in double whatever the particles' precision (a
// float state is promoted exactly).
template <class T>
__global__ __launch_bounds__(256) void save_state(const StepArgs A, char* slot) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= A.n) return;
    int32_t* cell = reinterpret_cast<int32_t*>(slot);
    double* d = reinterpret_cast<double*>(slot + slot_cell_bytes(A.n));
    cell[p] = A.cell[p];
    const T* src[5] = {static_cast<const T*>(A.xr), static_cast<const T*>(A.xth), static_cast<const T*>(A.ur),
                       static_cast<const T*>(A.uth), static_cast<const T*>(A.uph)};
    for (int k = 0; k < 5; ++k) d[(int64_t)k * A.n + p] = (double)src[k][p];
}

hipError_t launch_save_state(const StepArgs& A, bool split, void* slot, hipStream_t stream) {
    if (A.n <= 0) return hipSuccess;
    const dim3 g((unsigned)((A.n + 255) / 256));
    if (split) hipLaunchKernelGGL(save_state<float>, g, dim3(256), 0, stream, A, static_cast<char*>(slot));
    else hipLaunchKernelGGL(save_state<double>, g, dim3(256), 0, stream, A, static_cast<char*>(slot));
    return hipGetLastError();
}

// ---------------------------------------------------------------- lambda support
// Rows and columns (storage indices, guards included) holding a non-zero
// lambda entry, as exclusive prefix counts, so that "is lambda zero on this
// box" is two subtractions.  A conservative test: a box is reported non-zero
// when some row and some column in its ranges hold non-zeros.
__global__ __launch_bounds__(256) void lam_row_any(const BackArgs B, int* __restrict__ row_flag) {
    const int i = blockIdx.x;
    int any = 0;
    const int64_t base = (int64_t)i * B.pitch;
    for (int j = threadIdx.x; j < B.pitch; j += blockDim.x)
        any |= (B.lam[0][base + j] != 0.0) | (B.lam[1][base + j] != 0.0) | (B.lam[2][base + j] != 0.0);
    any = __syncthreads_or(any);
    if (threadIdx.x == 0) row_flag[i] = any;
}

// (only the rows that lam_row_any found non-zero are read)
__global__ __launch_bounds__(256) void lam_col_any(const BackArgs B, const int* __restrict__ row_flag,
                                                   int* __restrict__ col_flag) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= B.pitch) return;
    int any = 0;
    for (int i = 0; i < B.rows; ++i) {
        if (!row_flag[i]) continue;
        const int64_t e = (int64_t)i * B.pitch + j;
        any |= (B.lam[0][e] != 0.0) | (B.lam[1][e] != 0.0) | (B.lam[2][e] != 0.0);
    }
    col_flag[j] = any;
}

// flag[0..len) -> pre[0..len]; one thread per array (rows: thread 0, columns: thread 64).
__global__ __launch_bounds__(128) void lam_prefix(const BackArgs B, const int* __restrict__ row_flag,
                                                  const int* __restrict__ col_flag, int* __restrict__ row_pre,
                                                  int* __restrict__ col_pre) {
    if (threadIdx.x == 0) {
        int acc = 0;
        for (int i = 0; i < B.rows; ++i) { row_pre[i] = acc; acc += row_flag[i]; }
        row_pre[B.rows] = acc;
    } else if (threadIdx.x == 64) {
        int acc = 0;
        for (int j = 0; j < B.pitch; ++j) { col_pre[j] = acc; acc += col_flag[j]; }
        col_pre[B.pitch] = acc;
    }
}

// Field cotangents of one particle are summed in LDS (one slot per thread)
// while successive steps gather from the same 2 x 2 block of a component,
// and added to the gradient arrays with atomics when the block changes and
// at the end: a particle stays in a cell for a few steps, so this takes a
// few times fewer global atomics than adding every step.
constexpr int kBackThreads = 256;

// The three-corrector kernel keeps each thread's step tape in LDS (the
// register file is this sweep's limit; at one wave per SIMD a workgroup has
// the CU's LDS to itself).  A tape of 43 doubles (an odd count) puts the
// 64-bit accesses of 16 consecutive lanes on distinct banks.
template <int NC>
constexpr bool kTapeInLds = NC == kFastCorr;
static_assert(sizeof(adj::StepTape<kFastCorr>) == 43 * 8, "an odd number of doubles per tape");

template <int NC>
__global__ __launch_bounds__(kBackThreads) void push_deposit_backward_f64(const BackArgs B) {
    __shared__ double acc[6][4][kBackThreads];
    __shared__ long base[6][kBackThreads];
    __shared__ adj::StepTape<NC> tapes[kTapeInLds<NC> ? kBackThreads : 1];
    const int t = threadIdx.x;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + t;
    if (q >= B.count) return;                   // (no barrier below: the slots are per thread)
    for (int c = 0; c < 6; ++c) base[c][t] = -1;
    auto flush = [&](int c) {
        const long e = base[c][t];
        if (e < 0 || !B.gradF[c]) return;
        double* g = B.gradF[c];
        const long off[4] = {0, B.pitch, 1, B.pitch + 1};
        for (int k = 0; k < 4; ++k)
            if (acc[c][k][t] != 0.0) atomicAdd(g + e + off[k], acc[c][k][t]);
    };
    adj::StepTape<NC> reg_tape;
    adj::StepTape<NC>& T = kTapeInLds<NC> ? tapes[t] : reg_tape;
    backward_particle<NC>(B, q, [&](int c, long e, double g00, double g10, double g01, double g11) {
        if (base[c][t] != e) {
            flush(c);
            base[c][t] = e;
            acc[c][0][t] = g00;
            acc[c][1][t] = g10;
            acc[c][2][t] = g01;
            acc[c][3][t] = g11;
        } else {
            acc[c][0][t] += g00;
            acc[c][1][t] += g10;
            acc[c][2][t] += g01;
            acc[c][3][t] += g11;
        }
    }, T);
    for (int c = 0; c < 6; ++c) flush(c);
}

size_t backward_aux_bytes(int rows, int pitch) {
    return (size_t)(2 * rows + 2 * pitch + 2) * sizeof(int);
}

hipError_t launch_push_deposit_backward(BackArgs B, void* aux, hipStream_t stream) {
    if (B.count <= 0) return hipSuccess;
    int* row_flag = static_cast<int*>(aux);
    int* col_flag = row_flag + B.rows;
    int* row_pre = col_flag + B.pitch;
    int* col_pre = row_pre + B.rows + 1;
    B.row_pre = row_pre;
    B.col_pre = col_pre;
    hipLaunchKernelGGL(lam_row_any, dim3((unsigned)B.rows), dim3(256), 0, stream, B, row_flag);
    hipLaunchKernelGGL(lam_col_any, dim3((unsigned)((B.pitch + 255) / 256)), dim3(256), 0, stream, B, row_flag,
                       col_flag);
    hipLaunchKernelGGL(lam_prefix, dim3(1), dim3(128), 0, stream, B, row_flag, col_flag, row_pre, col_pre);
    const dim3 grid((unsigned)((B.count + kBackThreads - 1) / kBackThreads));
    if (B.ncorr == kFastCorr)
        hipLaunchKernelGGL(push_deposit_backward_f64<kFastCorr>, grid, dim3(kBackThreads), 0, stream, B);
    else
        hipLaunchKernelGGL(push_deposit_backward_f64<adj::kMaxCorr>, grid, dim3(kBackThreads), 0, stream, B);
    return hipGetLastError();
}

}  // namespace grpic
