// grpic_launch.hpp -- host-side launchers of the device kernels, called by
// the C ABI in api.hip, and the layout of the tiling buffer shared by the
// sort (which writes it) and the tiled push kernels (which read it).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "grpic_device.hpp"

namespace grpic {

// ---------------------------------------------------------------- tiling
// A tile is a segment of kTileCells consecutive cells of one grid row
// (theta is the contiguous direction, so a tile's particles are contiguous
// in a cell-sorted particle array).  Each tile's particles are cut into
// balanced slices; one workgroup pushes one slice, one particle per thread,
// and accumulates its current in an LDS window that covers the tile plus
// kMarginRows rows and kMarginCols columns of drift on each side.  The
// tiling holds two cuts of the same tiles, one per kind of tiled kernel.
constexpr int kTileCells = 64;
// Slice size (= workgroup size) of the CIC kernels: four waves.  Their
// FP64 push needs at most 128 VGPRs, and the window (14 x 75 vertices x 3
// arrays, 25.2 KB) with the staged states takes 38.1 KB of LDS, so four
// workgroups share a CU: four waves per SIMD.
constexpr int kSliceThreads = 256;
// Slice size of the cubic-shape kernel: three waves.  Its 65 LDS adds and
// 96 gather loads per particle run markedly slower in four-wave slices
// (measured: 5.0 against 2.8 ms for 2e7 particles on 2048^2).
constexpr int kSliceThreads3 = 192;
constexpr int kLaneGroups = 8;                             // lane permutation inside a slice
constexpr int kMarginRows = 5;
constexpr int kMarginCols = 4;
constexpr int kWinRows = 2 * kMarginRows + 4;              // vertex rows of the LDS window
constexpr int kWinCols = kTileCells + 2 * kMarginCols + 3; // vertex columns of the LDS window

struct TilingHeader {
    int64_t nslices;          // written by the sort on the device
    int64_t n;                // particle count the tiling was built for
    int64_t n_sorted;         // live particles at the sort (the slices cover [0, n_sorted))
    int32_t nr, nth, tiles_per_row, tile_cells;
};

// The slice table is in dispatch order: entry b holds the slice that
// workgroup b of a tiled push runs (b runs on XCD b % 8, so each XCD gets a
// contiguous band of slices in tile order, and neighbouring tiles share its
// L2); entries without a slice have len = 0.
struct Slice {
    int64_t start;            // first particle
    int32_t len;              // particles in the slice (<= the tiling's slice size)
    int32_t tile;             // row * tiles_per_row + column block
};

inline int tiles_per_row(int nth) { return (nth + kTileCells - 1) / kTileCells; }
// At most n / smax + ntiles slices of at most smax particles; 8 more entries
// because the table is kept in dispatch order (below), which rounds each
// XCD's band up.
inline int64_t slice_capacity(int64_t n, int nr, int nth, int smax = kSliceThreads) {
    return n / smax + (int64_t)nr * tiles_per_row(nth) + 8;
}
// Layout (byte offsets, each 8-byte aligned): the header; the CIC slice
// table (cap entries) and one int32 per slice that a push with counters
// fills with the slice's live particle count (so that the count needs no
// same-address atomics; a small kernel sums it); the same two for the cubic
// cut (cap3 entries); then the anchor table, which depends on the grid only
// and is written by the sort: r at the corners of rows -kMarginRows .. nr +
// kMarginRows - 1, then sin and cos at columns -kMarginCols ..
// tiles_per_row * kTileCells + kMarginCols, i.e. every anchor a tile's
// window can ask for.
inline int anchor_table_rows(int nr) { return nr + 2 * kMarginRows; }
inline int anchor_table_cols(int nth) { return tiles_per_row(nth) * kTileCells + 2 * kMarginCols + 1; }
struct TilingLayout {
    int64_t cap, cap3;                    // entries of the CIC and the cubic slice tables
    size_t slices, live, slices3, live3, anchors, bytes;
};
inline size_t align8(size_t b) { return (b + 7) / 8 * 8; }
inline TilingLayout tiling_layout(int64_t n, int nr, int nth) {
    TilingLayout L;
    L.cap = slice_capacity(n, nr, nth, kSliceThreads);
    L.cap3 = slice_capacity(n, nr, nth, kSliceThreads3);
    L.slices = sizeof(TilingHeader);
    L.live = L.slices + (size_t)L.cap * sizeof(Slice);
    L.slices3 = align8(L.live + (size_t)L.cap * sizeof(int32_t));
    L.live3 = L.slices3 + (size_t)L.cap3 * sizeof(Slice);
    L.anchors = align8(L.live3 + (size_t)L.cap3 * sizeof(int32_t));
    L.bytes = L.anchors + sizeof(double) * ((size_t)anchor_table_rows(nr) + 2 * (size_t)anchor_table_cols(nth));
    return L;
}
inline size_t tiling_bytes(int64_t n, int nr, int nth) { return tiling_layout(n, nr, nth).bytes; }
template <class T>
inline T* tiling_at(void* tiling, size_t off) { return reinterpret_cast<T*>(static_cast<char*>(tiling) + off); }

// ---------------------------------------------------------------- launchers
// kick: kBoris (the generalised Boris kick) or kVay (FP64 only).  order:
// the shape, 1 (CIC) or 3 (cubic spline: FP64, Boris kick).
hipError_t launch_push_deposit(const StepArgs& A, bool split, hipStream_t stream, int kick = kBoris, int order = 1);
hipError_t launch_push_deposit_tiled(const StepArgs& A, bool split, void* tiling, hipStream_t stream,
                                     int kick = kBoris, int order = 1);
hipError_t launch_charge(const StepArgs& A, bool split, double* Q, hipStream_t stream, int order = 1);
struct QedArgs;
// One QED step (FP64, Boris, CIC): the tiled slices if a tiling is given,
// then the particles no slice covers; n_used updated on the device.  With
// a workspace (tiled only), each slice stages the particles it creates and
// a scan places them after the others, so the step takes no same-address
// atomics for them.
hipError_t launch_push_deposit_qed(const StepArgs& A, QedArgs Q, void* tiling, int64_t slice_cap, void* ws,
                                   hipStream_t stream);
size_t qed_workspace_bytes(int64_t slice_cap);

struct SortArgs {
    int64_t n;
    int nr, nth, ncell;
    size_t elem;                      // bytes of one xr/xth/ur/uth/uph/w element (8 or 4)
    const int32_t* cell_in;
    const void* in[6];                // xr, xth, ur, uth, uph, w
    const uint8_t* sp_in;
    const void* phi_in;               // optional, same element size
    const uint64_t* tag_in;           // optional
    int32_t* cell_out;
    void* out[6];
    uint8_t* sp_out;
    void* phi_out;
    uint64_t* tag_out;
    unsigned long long* counts;       // ncell + 1 entries of workspace
    unsigned long long* blocksums;    // sort_scan_blocks(ncell + 1) + 1 entries of workspace
    unsigned long long* tile_slices;  // ntiles + 1 entries of workspace (tiling only)
    int64_t* cell_offsets;            // optional output, ncell + 1
    int64_t* n_alive;                 // device output
    void* tiling;                     // optional output, tiling_bytes()
    double lnr0, dlnr, dth;           // the grid's geometry (the tiling's anchor table)
};

// Reverse sweep of K push + deposit steps (adjoint.hip).
struct BackArgs {
    double a, M, lnr0, dlnr, dth;
    int nr, nth, guard, pitch;
    double dt;
    int ncorr, nsteps, ckpt_every, nsp;
    double q[kMaxSpecies], m[kMaxSpecies];
    int massless[kMaxSpecies];
    int64_t n;
    const double* w;
    const uint8_t* sp;
    const double* F[6];               // D^r, D^th, D^ph, B^r, B^th, B^ph
    const double* lam[3];             // dL/dF^r, dL/dF^th, dL/dG^ph
    const void* ckpt;
    size_t slot_bytes;
    int64_t first, count;             // the particles [first, first + count) of the checkpointed n
    size_t fstride, gstride;          // elements between steps' field (gradient) arrays; 0: one set for all steps
    double* ws;                       // ckpt_every * 5 * count doubles
    double* grad_u[3];                // out: dL/du_r, dL/du_th, dL/du_ph at step 0 (count entries)
    double* gradF[6];                 // += dL/dD^i, dL/dB^i (NULL: not wanted)
    int rows;                         // storage rows of the grid arrays (nr + 1 + 2 guard)
    const int* row_pre;               // lambda support, set by the launcher
    const int* col_pre;
};

size_t checkpoint_slot_bytes(int64_t n);
int adj_max_corr();
hipError_t launch_save_state(const StepArgs& A, bool split, void* slot, hipStream_t stream);
size_t backward_aux_bytes(int rows, int pitch);
hipError_t launch_push_deposit_backward(BackArgs B, void* aux, hipStream_t stream);

int64_t sort_scan_blocks(int64_t len);
void scan_exclusive(unsigned long long* a, int64_t len, unsigned long long* blocksums, hipStream_t stream);
size_t sort_workspace_bytes(int nr, int nth);
hipError_t launch_sort(const SortArgs& S, hipStream_t stream);
// The anchor table of a tiling (r at the rows' corners, sin and cos at the
// columns'), which depends on the grid only: written by the sort.
hipError_t launch_anchor_table(double lnr0, double dlnr, double dth, int nr, int nth, double* anchors,
                               hipStream_t stream);

// The sort workspace that grpic_sort_noalloc uses: a static device array of
// kSortScratchBytes per GPU; sort_scratch returns its address on the current
// device (looked up on the first call there).
constexpr size_t kSortScratchBytes = size_t(40) << 20;
hipError_t sort_scratch(void** ptr);

}  // namespace grpic
