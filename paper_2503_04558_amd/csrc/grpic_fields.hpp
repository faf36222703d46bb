// grpic_fields.hpp -- arguments and table layout of the field-solver kernels
// (fields.hip), shared with the C ABI in api.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace grpic {

// Planes of the coefficient / inverse-area table, one grid array each.
// Coefficients alpha gamma_ij and sqrt(gamma) beta^r at the location named:
// Dr = (i+1/2, j) (also B^th), Dt = (i, j+1/2) (also B^r), Dp = (i, j),
// Bp = (i+1/2, j+1/2); inverse areas per unit phi of the six components.
enum FieldTable {
    kT_Dr_aGrr, kT_Dr_aGrp, kT_Dr_sgB, kT_Dr_aGtt,
    kT_Dt_aGtt, kT_Dt_sgB, kT_Dt_aGrr, kT_Dt_aGrp,
    kT_Dp_aGpp, kT_Dp_aGrp, kT_Dp_sgB,
    kT_Bp_aGpp, kT_Bp_aGrp, kT_Bp_sgB,
    kT_iADr, kT_iADt, kT_iADp, kT_iABr, kT_iABt, kT_iABp,
    kTablePlanes
};
// Radial edge lengths per row i = -2 .. nr + 1 (index i + 2): primal
// r_{i+1} - r_i and dual r_{i+1/2} - r_{i-1/2}.
enum { kDrPrimal, kDrDual, kDrRows };
constexpr int kTableRowLo = -2;                  // tables cover rows -2 .. nr + 1

struct FieldArgs {
    double a, M, lnr0, dlnr, dth;
    int nr, nth, guard, pitch;
    size_t plane;                                 // elements of one grid array
    int nrow;                                     // rows of the radial-length table (nr + 4)
    double* tab;                                  // kTablePlanes planes
    double* drow;                                 // kDrRows x nrow
    const double* J[3];                           // flux-form currents (or NULL)
    double dt, w0, w1;
    __host__ __device__ uint32_t at(int i, int j) const { return (uint32_t)((i + guard) * pitch + (j + guard)); }
};

struct FieldPtrs {
    double* c[6];                                 // D^r, D^th, D^ph, B^r, B^th, B^ph (or E, H)
};

inline size_t field_plane(int nr, int pitch, int guard) { return (size_t)(nr + 1 + 2 * guard) * pitch; }
inline size_t field_tables_bytes(int nr, int pitch, int guard) {
    return sizeof(double) * (kTablePlanes * field_plane(nr, pitch, guard) + (size_t)kDrRows * (nr + 4));
}
// Workspace: the state at the start of the step, its circulations, the
// auxiliary fields: 18 grid arrays.
inline size_t field_workspace_bytes(int nr, int pitch, int guard) {
    return sizeof(double) * 18 * field_plane(nr, pitch, guard);
}

hipError_t launch_field_tables(const FieldArgs& F, const double* gx, const double* gw, hipStream_t stream);
hipError_t launch_field_step(const FieldArgs& F, FieldPtrs X, FieldPtrs x0, FieldPtrs C0, FieldPtrs aux, int ncorr,
                             int damp_cells, double damp_max, hipStream_t stream);

}  // namespace grpic
