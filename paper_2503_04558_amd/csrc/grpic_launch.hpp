// grpic_launch.hpp -- host-side launchers of the device kernels, called by
// the C ABI in api.hip.  Every launcher enqueues on `stream` and returns the
// launch status.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "grpic_device.hpp"

namespace grpic {

hipError_t launch_push_deposit_f64(const StepArgs& A, hipStream_t stream);
hipError_t launch_charge(const StepArgs& A, bool split, double* Q, hipStream_t stream);

struct SortArgs {
    int64_t n;
    int ncell;
    size_t elem;                      // bytes of one xr/xth/ur/uth/uph/w element (8 or 4)
    const int32_t* cell_in;
    const void* in[6];                // xr, xth, ur, uth, uph, w
    const uint8_t* sp_in;
    const void* phi_in;               // optional, same element size
    int32_t* cell_out;
    void* out[6];
    uint8_t* sp_out;
    void* phi_out;
    unsigned long long* counts;       // ncell + 1 entries of workspace
    unsigned long long* blocksums;    // sort_scan_blocks(ncell + 1) + 1 entries of workspace
    int64_t* cell_offsets;            // optional output, ncell + 1
    int64_t* n_alive;                 // device output
};

int64_t sort_scan_blocks(int64_t len);
hipError_t launch_sort(const SortArgs& S, hipStream_t stream);

}  // namespace grpic
