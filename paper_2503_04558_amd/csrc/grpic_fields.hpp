// grpic_fields.hpp -- arguments and table layout of the field-solver kernels
// (fields.hip), shared with the C ABI in api.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace grpic {

// Planes of the table: inverse area elements per unit phi of the six
// components at their locations (zero where a component is not updated).
enum FieldTable { kT_iADr, kT_iADt, kT_iADp, kT_iABr, kT_iABt, kT_iABp, kTablePlanes };
// Radial edge lengths per row i = -2 .. nr + 1 (index i + 2): primal
// r_{i+1} - r_i and dual r_{i+1/2} - r_{i-1/2}.
enum { kDrPrimal, kDrDual, kDrRows };
constexpr int kTableRowLo = -2;                  // tables cover rows -2 .. nr + 1
// Radii r(x) at half-integer steps x = -2, -1.5, .. nr + 2 (2 nr + 9
// values) and sin, cos of theta at y = 0, 0.5, .. nth (2 nth + 1 values each).
__host__ __device__ inline int field_nrad(int nr) { return 2 * nr + 9; }
__host__ __device__ inline int field_nang(int nth) { return 2 * nth + 1; }

struct FieldArgs {
    double a, M, lnr0, dlnr, dth;
    int nr, nth, guard, pitch;
    size_t plane;                                 // elements of one grid array
    int nrow;                                     // rows of the radial-length table (nr + 4)
    double* tab;                                  // kTablePlanes planes
    double* drow;                                 // kDrRows x nrow
    double* rad;                                  // field_nrad(nr) radii
    double* sn;                                   // field_nang(nth) sines, then as many cosines
    const double* J[3];                           // flux-form currents (or NULL)
    double dt, w0, w1;
    __host__ __device__ uint32_t at(int i, int j) const { return (uint32_t)((i + guard) * pitch + (j + guard)); }
};

struct FieldPtrs {
    double* c[6];                                 // D^r, D^th, D^ph, B^r, B^th, B^ph (or E, H)
};

inline size_t field_plane(int nr, int pitch, int guard) { return (size_t)(nr + 1 + 2 * guard) * pitch; }
inline size_t field_tables_bytes(int nr, int nth, int pitch, int guard) {
    return sizeof(double) * (kTablePlanes * field_plane(nr, pitch, guard) + (size_t)kDrRows * (nr + 4) +
                             field_nrad(nr) + 2 * (size_t)field_nang(nth));
}
// Workspace: the corrector's constant part X^n + dt (w0 C(X^n) - J) and two
// buffers of corrector iterates: 18 grid arrays.
inline size_t field_workspace_bytes(int nr, int pitch, int guard) {
    return sizeof(double) * 18 * field_plane(nr, pitch, guard);
}

hipError_t launch_field_tables(const FieldArgs& F, const double* gx, const double* gw, hipStream_t stream);
hipError_t launch_field_step(const FieldArgs& F, FieldPtrs X, FieldPtrs R, FieldPtrs W1, FieldPtrs W2, int ncorr,
                             int damp_cells, double damp_max, hipStream_t stream);

}  // namespace grpic
