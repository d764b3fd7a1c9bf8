// pimpc_row.hpp -- host interface of the row-per-lane (long horizon) kernel.
#pragma once
#include <hip/hip_runtime.h>

#include "pimpc_dev.hpp"

namespace pimpc {

struct RowArgs {
    const InstDev* inst;
    int32_t inst_idx;
    int32_t pad;
    const void* mats;
    void* state;
    void* iters_out;
    const void* x0;
    const void* uprev;
    void* u0;
    InfoDev* info;
    void* scratch;  // halo mailboxes and residual partials of this context
    double rho;
    double eps;
    int32_t K;
    int32_t check_every;
    int32_t warm;
    int32_t write_iters;
};

// True if the row family handles an instance of this shape; sets the padded sizes.
bool row_supported(int nx, int nu, int N, int tv, int fp64, int* nxp, int* nup);
// Device scratch bytes the instance needs (halo mailboxes, partials).
size_t row_scratch_bytes(const InstDev& I, int fp64);
// Pick the stage blocking (stored in I.row_s) so the grid stays co-resident;
// I.row_s > 0 on entry is the preferred blocking.
hipError_t row_prepare(int fp64, InstDev& I);
// Form the fused stage data of a row-family instance in its scratch (after
// every factorisation; reads the T block written by the factor kernel).
hipError_t launch_row_fuse(const InstDev* d_inst, int inst_idx, const InstDev& I, const void* mats,
                           void* scratch_base, hipStream_t s);
// Enqueue the solve of one row-family instance (clears the cleared part of its
// scratch first).
hipError_t launch_row(int fp64, const RowArgs* a_dev, const InstDev& I, void* scratch_base, hipStream_t s);

}  // namespace pimpc
