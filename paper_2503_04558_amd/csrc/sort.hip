// sort.hip -- counting sort of particles by cell, and the tiling the tiled
// push kernel runs on.
//
// histogram of live cells -> exclusive scan (two-level, 4096 entries per
// block) -> [tiling: per-tile slice counts -> scan -> slice table] ->
// scatter.  Histogram and scatter take a chunk of consecutive particles per
// workgroup and count its cells in an LDS hash table first, so each distinct
// cell of the chunk costs one global atomic: on the almost sorted input of a
// re-sort a chunk holds a few dozen cells, and per-particle (or per-run)
// atomics would queue on the same few counters.  Removed particles
// (cell < 0) are dropped and the tail of the output is marked removed; the
// order inside a cell is not specified.
#include "grpic_launch.hpp"

#include <mutex>

namespace grpic {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;

int64_t sort_scan_blocks(int64_t len) { return (len + kScanTile - 1) / kScanTile; }

size_t sort_workspace_bytes(int nr, int nth) {
    const int64_t len = (int64_t)nr * nth + 1;
    const int64_t ntiles = (int64_t)nr * tiles_per_row(nth);
    return (size_t)(len + sort_scan_blocks(len) + 1 + ntiles + 1) * sizeof(unsigned long long);
}

__global__ __launch_bounds__(256) void fill_u64(unsigned long long* __restrict__ a, int64_t n, unsigned long long v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// Chunk of consecutive particles per histogram / scatter workgroup, and the
// LDS hash table that counts its cells: at most half full, so an empty slot
// is always found.  A scatter workgroup waits once for its cells' atomics
// (with return, at the memory side); 2048-particle chunks halve those waits
// per particle and beat 1024 (7.6 against 8.3 ms per re-sort of 2e8, two
// workgroups per CU instead of five) and 512 (9.2 ms).
constexpr int kChunkThreads = 256;
constexpr int kChunkItems = 8;
constexpr int kChunk = kChunkThreads * kChunkItems;
constexpr int kHashSlots = 2 * kChunk;
static_assert((kHashSlots & (kHashSlots - 1)) == 0, "power-of-two table");
constexpr int kEmpty = -1;

struct CellTable {
    int key[kHashSlots];               // cell, or kEmpty
    int count[kHashSlots];             // particles of the chunk in that cell
};

__device__ __forceinline__ void table_clear(CellTable& T) {
    for (int e = threadIdx.x; e < kHashSlots; e += kChunkThreads) {
        T.key[e] = kEmpty;
        T.count[e] = 0;
    }
}

// Slot of cell c (inserted if new); adds inc to its count and returns the
// count before the add in old.  Multiplicative hashing spreads the cells of
// neighbouring rows (c and c + nth) that a plain mask would collide.
__device__ __forceinline__ int table_insert(CellTable& T, int c, int inc, int& old) {
    int slot = (int)(((unsigned)c * 2654435761u) >> 21) & (kHashSlots - 1);
    for (int probe = 0; probe < kHashSlots; ++probe) {
        const int k = atomicCAS(&T.key[slot], kEmpty, c);
        if (k == kEmpty || k == c) {
            old = atomicAdd(&T.count[slot], inc);
            return slot;
        }
        slot = (slot + 1) & (kHashSlots - 1);
    }
    old = 0;                           // not reached: at most kChunk keys in 2 * kChunk slots
    return -1;
}

// Runs of equal valid cells among adjacent lanes of a wave: the first lane
// of each run (head) and the run's last lane (tail).  Every lane of the
// wave must call it.
__device__ __forceinline__ void wave_runs(int c, bool valid, int& head, int& tail) {
    const int lane = threadIdx.x & 63;
    const int prev = __shfl_up(c, 1);
    const int next = __shfl_down(c, 1);
    const unsigned long long heads = __ballot(valid && (lane == 0 || prev != c));
    const unsigned long long tails = __ballot(valid && (lane == 63 || next != c));
    head = 0;
    tail = 0;
    if (valid) {
        const unsigned long long upto = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
        head = 63 - __clzll(heads & upto);
        const unsigned long long from = ~((1ull << head) - 1ull);
        tail = __ffsll((long long)(tails & from)) - 1;
    }
}

// Inserts the valid cells of one item per lane, one table access per run of
// equal cells; returns the lane's slot (-1 if not valid) and its rank among
// the chunk's particles of that cell.  Every lane of the wave must call it.
__device__ __forceinline__ int wave_insert(CellTable& T, int c, bool valid, int& rank) {
    const int lane = threadIdx.x & 63;
    int head, tail;
    wave_runs(c, valid, head, tail);
    int slot = -1, old = 0;
    if (valid && lane == head) slot = table_insert(T, c, tail - head + 1, old);
    slot = __shfl(slot, head);
    old = __shfl(old, head);
    rank = old + (lane - head);
    return valid ? slot : -1;
}

__device__ __forceinline__ int64_t chunk_index(int k) {
    return (int64_t)blockIdx.x * kChunk + (int64_t)k * kChunkThreads + threadIdx.x;
}

// Histogram of live cells: counts[c] += number of particles in cell c.
__global__ __launch_bounds__(kChunkThreads) void sort_hist(const int32_t* __restrict__ cell, int64_t n, int ncell,
                                                           unsigned long long* __restrict__ counts) {
    __shared__ CellTable T;
    int c[kChunkItems];
    for (int k = 0; k < kChunkItems; ++k) {
        const int64_t p = chunk_index(k);
        c[k] = p < n ? cell[p] : -1;
    }
    table_clear(T);
    __syncthreads();
    for (int k = 0; k < kChunkItems; ++k) {
        int rank;
        wave_insert(T, c[k], c[k] >= 0 && c[k] < ncell, rank);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kHashSlots; e += kChunkThreads)
        if (T.key[e] != kEmpty) atomicAdd(counts + T.key[e], (unsigned long long)T.count[e]);
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

static inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

// Exclusive scan of a[0..len) in place (a[len-1] should be a zero sentinel
// so that it receives the total).
void scan_exclusive(unsigned long long* a, int64_t len, unsigned long long* blocksums, hipStream_t stream) {
    const int64_t nb = sort_scan_blocks(len);
    hipLaunchKernelGGL(scan_tiles, dim3((unsigned)nb), dim3(kScanThreads), 0, stream, a, len, blocksums);
    hipLaunchKernelGGL(scan_top, dim3(1), dim3(kScanThreads), 0, stream, blocksums, nb);
    hipLaunchKernelGGL(scan_add, dim3(nblk(len)), dim3(256), 0, stream, a, len, blocksums);
}

// Number of slices of each tile, from the scanned cell offsets.
__global__ __launch_bounds__(256) void tile_slice_counts(const unsigned long long* __restrict__ offs, int nr, int nth,
                                                         int tpr, int smax, unsigned long long* __restrict__ ns) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ntiles = (int64_t)nr * tpr;
    if (t > ntiles) return;
    if (t == ntiles) { ns[t] = 0ull; return; }
    const int i = (int)(t / tpr), jb = (int)(t - (int64_t)i * tpr);
    const int64_t c0 = (int64_t)i * nth + (int64_t)jb * kTileCells;
    const int64_t c1 = c0 + min(kTileCells, nth - jb * kTileCells);
    const unsigned long long cnt = offs[c1] - offs[c0];
    ns[t] = (cnt + smax - 1) / smax;
}

__global__ __launch_bounds__(256) void slices_empty(Slice* __restrict__ out, int64_t cap) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < cap) out[i] = Slice{-1, 0, 0};
}

// Slice table: tile t's particles cut into ns balanced slices; slice L (in
// tile order) goes to entry (L % per_xcd) * 8 + L / per_xcd, the workgroup
// that runs the L % per_xcd-th slice of XCD L / per_xcd's band.
__global__ __launch_bounds__(256) void tile_slices(const unsigned long long* __restrict__ offs,
                                                   const unsigned long long* __restrict__ base, int nr, int nth,
                                                   int tpr, int64_t n, int64_t cap, TilingHeader* hdr,
                                                   Slice* __restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ntiles = (int64_t)nr * tpr;
    if (t == 0 && hdr) {                                // the header: written with the CIC cut
        hdr->nslices = (int64_t)base[ntiles];
        hdr->n = n;
        hdr->n_sorted = (int64_t)offs[(int64_t)nr * nth];
        hdr->nr = nr;
        hdr->nth = nth;
        hdr->tiles_per_row = tpr;
        hdr->tile_cells = kTileCells;
    }
    if (t >= ntiles) return;
    const int i = (int)(t / tpr), jb = (int)(t - (int64_t)i * tpr);
    const int64_t c0 = (int64_t)i * nth + (int64_t)jb * kTileCells;
    const int64_t c1 = c0 + min(kTileCells, nth - jb * kTileCells);
    const int64_t start = (int64_t)offs[c0];
    const int64_t cnt = (int64_t)offs[c1] - start;
    const int64_t b = (int64_t)base[t];
    const int64_t ns = (int64_t)base[t + 1] - b;
    if (ns <= 0) return;
    const int64_t per_xcd = ((int64_t)base[ntiles] + 7) / 8;
    const int64_t each = (cnt + ns - 1) / ns;
    for (int64_t s = 0; s < ns; ++s) {
        const int64_t s0 = s * each;
        Slice sl;
        sl.start = start + s0;
        sl.len = (int32_t)(cnt - s0 < each ? cnt - s0 : each);
        sl.tile = (int32_t)t;
        const int64_t L = b + s;
        const int64_t e = (L % per_xcd) * 8 + L / per_xcd;
        if (e < cap) out[e] = sl;                        // always: cap >= nslices + 8
    }
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

// Scatter: counts[] holds each cell's next free output index; a chunk
// reserves its particles' range of every cell with one atomic and places
// them by their rank inside the chunk.
template <class T>
__global__ __launch_bounds__(kChunkThreads) void sort_scatter(const SortArgs S) {
    __shared__ CellTable Tb;
    __shared__ unsigned long long base[kHashSlots];
    int c[kChunkItems];
    for (int k = 0; k < kChunkItems; ++k) {
        const int64_t p = chunk_index(k);
        c[k] = p < S.n ? S.cell_in[p] : -1;
    }
    // the particles' data is read first, so its latency overlaps the counting
    T v[kChunkItems][6], ph[kChunkItems];
    uint8_t spv[kChunkItems];
    uint64_t tg[kChunkItems];
    for (int k = 0; k < kChunkItems; ++k) {
        const int64_t p = chunk_index(k);
        const bool valid = c[k] >= 0 && c[k] < S.ncell;
        for (int a = 0; a < 6; ++a) v[k][a] = valid ? static_cast<const T*>(S.in[a])[p] : T(0);
        spv[k] = valid ? S.sp_in[p] : 0;
        ph[k] = valid && S.phi_in ? static_cast<const T*>(S.phi_in)[p] : T(0);
        tg[k] = valid && S.tag_in ? S.tag_in[p] : 0ull;
    }
    table_clear(Tb);
    __syncthreads();
    int slot[kChunkItems], rank[kChunkItems];
    for (int k = 0; k < kChunkItems; ++k) slot[k] = wave_insert(Tb, c[k], c[k] >= 0 && c[k] < S.ncell, rank[k]);
    __syncthreads();
    for (int e = threadIdx.x; e < kHashSlots; e += kChunkThreads)
        if (Tb.key[e] != kEmpty) base[e] = atomicAdd(S.counts + Tb.key[e], (unsigned long long)Tb.count[e]);
    __syncthreads();
    for (int k = 0; k < kChunkItems; ++k) {
        if (slot[k] < 0) continue;
        const int64_t q = (int64_t)base[slot[k]] + rank[k];
        S.cell_out[q] = c[k];
        for (int a = 0; a < 6; ++a) static_cast<T*>(S.out[a])[q] = v[k][a];
        S.sp_out[q] = spv[k];
        if (S.phi_in) static_cast<T*>(S.phi_out)[q] = ph[k];
        if (S.tag_in) S.tag_out[q] = tg[k];
    }
}

static inline unsigned nchunk(int64_t n) { return (unsigned)((n + kChunk - 1) / kChunk); }

hipError_t launch_sort(const SortArgs& S, hipStream_t stream) {
    const int64_t len = (int64_t)S.ncell + 1;
    hipLaunchKernelGGL(fill_u64, dim3(nblk(len)), dim3(256), 0, stream, S.counts, len, 0ull);
    if (S.n > 0)
        hipLaunchKernelGGL(sort_hist, dim3(nchunk(S.n)), dim3(kChunkThreads), 0, stream, S.cell_in, S.n, S.ncell, S.counts);
    scan_exclusive(S.counts, len, S.blocksums, stream);
    if (S.tiling) {
        const int tpr = tiles_per_row(S.nth);
        const int64_t ntiles = (int64_t)S.nr * tpr;
        const TilingLayout L = tiling_layout(S.n, S.nr, S.nth);
        TilingHeader* hdr = static_cast<TilingHeader*>(S.tiling);
        // the two cuts, one after the other (they share the tile_slices workspace)
        for (int cut = 0; cut < 2; ++cut) {
            const int smax = cut == 0 ? kSliceThreads : kSliceThreads3;
            const int64_t cap = cut == 0 ? L.cap : L.cap3;
            Slice* slices = tiling_at<Slice>(S.tiling, cut == 0 ? L.slices : L.slices3);
            hipLaunchKernelGGL(tile_slice_counts, dim3(nblk(ntiles + 1)), dim3(256), 0, stream, S.counts, S.nr, S.nth,
                               tpr, smax, S.tile_slices);
            scan_exclusive(S.tile_slices, ntiles + 1, S.blocksums, stream);
            hipLaunchKernelGGL(slices_empty, dim3(nblk(cap)), dim3(256), 0, stream, slices, cap);
            hipLaunchKernelGGL(tile_slices, dim3(nblk(ntiles + 1)), dim3(256), 0, stream, S.counts, S.tile_slices,
                               S.nr, S.nth, tpr, S.n, cap, cut == 0 ? hdr : nullptr, slices);
        }
        const hipError_t e = launch_anchor_table(S.lnr0, S.dlnr, S.dth, S.nr, S.nth,
                                                 tiling_at<double>(S.tiling, L.anchors), stream);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(sort_offsets_out, dim3(nblk(len)), dim3(256), 0, stream, S.counts, S.ncell,
                       S.cell_offsets, S.n_alive);
    if (S.n > 0) {
        hipLaunchKernelGGL(sort_mark_tail, dim3(nblk(S.n)), dim3(256), 0, stream, S.cell_out, S.n,
                           S.counts + S.ncell);
        if (S.elem == 8) hipLaunchKernelGGL(sort_scatter<double>, dim3(nchunk(S.n)), dim3(kChunkThreads), 0, stream, S);
        else hipLaunchKernelGGL(sort_scatter<float>, dim3(nchunk(S.n)), dim3(kChunkThreads), 0, stream, S);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------- no-allocation sort
// The workspace of grpic_sort_noalloc: a file-scope device array that every
// GPU the library runs on holds until the process ends.  Host code never
// passes its name to a kernel (on the host the name is only a stand-in):
// its device address is looked up once per device, with that device
// current, and kept.
static __device__ __align__(256) unsigned char scratch[kSortScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t sort_scratch(void** ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace grpic
