// sort.hip -- counting sort of particles by cell.
//
// histogram of live cells -> exclusive scan (two-level, 4096 entries per
// block) -> scatter with one atomic cursor per cell.  Removed particles
// (cell < 0) are dropped; the order inside a cell is not specified.
#include "grpic_launch.hpp"

namespace grpic {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

int64_t sort_scan_blocks(int64_t len) { return (len + kScanTile - 1) / kScanTile; }

__global__ __launch_bounds__(256) void fill_u64(unsigned long long* __restrict__ a, int64_t n, unsigned long long v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

__global__ __launch_bounds__(256) void sort_hist(const int32_t* __restrict__ cell, int64_t n, int ncell,
                                                 unsigned long long* __restrict__ counts) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int c = cell[p];
    if (c >= 0 && c < ncell) atomicAdd(counts + c, 1ull);
}

// Inclusive scan of one value per thread across a 256-thread block.
__device__ __forceinline__ unsigned long long block_inclusive_scan(unsigned long long v, unsigned long long* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const unsigned long long add = threadIdx.x >= (unsigned)off ? sh[threadIdx.x - off] : 0ull;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    return sh[threadIdx.x];
}

// In-place exclusive scan of each 4096-entry tile; the tile total goes to blocksums.
__global__ __launch_bounds__(256) void scan_tiles(unsigned long long* __restrict__ a, int64_t len,
                                                  unsigned long long* __restrict__ blocksums) {
    __shared__ unsigned long long sh[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    unsigned long long v[kScanItems];
    unsigned long long tot = 0;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + k;
        v[k] = i < len ? a[i] : 0ull;
        tot += v[k];
    }
    const unsigned long long incl = block_inclusive_scan(tot, sh);
    unsigned long long run = incl - tot;
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t i = base + k;
        if (i < len) a[i] = run;
        run += v[k];
    }
    if (threadIdx.x == kScanThreads - 1) blocksums[blockIdx.x] = incl;
}

// Exclusive scan of the tile totals by one block, in chunks of 256.
__global__ __launch_bounds__(256) void scan_top(unsigned long long* __restrict__ bs, int64_t nb) {
    __shared__ unsigned long long sh[kScanThreads];
    unsigned long long carry = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += kScanThreads) {
        const int64_t i = c0 + threadIdx.x;
        const unsigned long long v = i < nb ? bs[i] : 0ull;
        const unsigned long long incl = block_inclusive_scan(v, sh);
        if (i < nb) bs[i] = carry + incl - v;
        const unsigned long long total = sh[kScanThreads - 1];
        __syncthreads();
        carry += total;
    }
    if (threadIdx.x == 0) bs[nb] = carry;
}

__global__ __launch_bounds__(256) void scan_add(unsigned long long* __restrict__ a, int64_t len,
                                                const unsigned long long* __restrict__ bs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < len) a[i] += bs[i / kScanTile];
}

__global__ __launch_bounds__(256) void sort_offsets_out(const unsigned long long* __restrict__ counts, int ncell,
                                                        int64_t* __restrict__ offsets, int64_t* __restrict__ n_alive) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (offsets && i <= ncell) offsets[i] = (int64_t)counts[i];
    if (i == ncell) *n_alive = (int64_t)counts[ncell];
}

// Elements of the output beyond the live count are marked removed.
__global__ __launch_bounds__(256) void sort_mark_tail(int32_t* __restrict__ cell_out, int64_t n,
                                                      const unsigned long long* __restrict__ total) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n && p >= (int64_t)*total) cell_out[p] = -1;
}

template <class T>
__global__ __launch_bounds__(256) void sort_scatter(const SortArgs S) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= S.n) return;
    const int c = S.cell_in[p];
    if (c < 0 || c >= S.ncell) return;
    const int64_t q = (int64_t)atomicAdd(S.counts + c, 1ull);
    S.cell_out[q] = c;
    for (int k = 0; k < 6; ++k) static_cast<T*>(S.out[k])[q] = static_cast<const T*>(S.in[k])[p];
    S.sp_out[q] = S.sp_in[p];
    if (S.phi_in) static_cast<T*>(S.phi_out)[q] = static_cast<const T*>(S.phi_in)[p];
}

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_sort(const SortArgs& S, hipStream_t stream) {
    const int64_t len = (int64_t)S.ncell + 1;
    const int64_t nb = sort_scan_blocks(len);
    hipLaunchKernelGGL(fill_u64, dim3(nblk(len)), dim3(256), 0, stream, S.counts, len, 0ull);
    if (S.n > 0)
        hipLaunchKernelGGL(sort_hist, dim3(nblk(S.n)), dim3(256), 0, stream, S.cell_in, S.n, S.ncell, S.counts);
    hipLaunchKernelGGL(scan_tiles, dim3((unsigned)nb), dim3(kScanThreads), 0, stream, S.counts, len, S.blocksums);
    hipLaunchKernelGGL(scan_top, dim3(1), dim3(kScanThreads), 0, stream, S.blocksums, nb);
    hipLaunchKernelGGL(scan_add, dim3(nblk(len)), dim3(256), 0, stream, S.counts, len, S.blocksums);
    hipLaunchKernelGGL(sort_offsets_out, dim3(nblk(len)), dim3(256), 0, stream, S.counts, S.ncell,
                       S.cell_offsets, S.n_alive);
    if (S.n > 0) {
        hipLaunchKernelGGL(sort_mark_tail, dim3(nblk(S.n)), dim3(256), 0, stream, S.cell_out, S.n,
                           S.counts + S.ncell);
        if (S.elem == 8) hipLaunchKernelGGL(sort_scatter<double>, dim3(nblk(S.n)), dim3(256), 0, stream, S);
        else hipLaunchKernelGGL(sort_scatter<float>, dim3(nblk(S.n)), dim3(256), 0, stream, S);
    }
    return hipGetLastError();
}

}  // namespace grpic
