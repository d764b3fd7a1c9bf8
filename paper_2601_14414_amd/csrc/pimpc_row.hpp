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
    void* scratch;        // halo mailboxes, abort flag and residual partials of this instance
    const void* fused;    // fused stage data of this instance (written at factorisation time)
    const int32_t* fbad;  // per instance: non-zero when its stage factorisation failed (not SPD)
    double rho;
    double eps;
    int32_t K;
    int32_t check_every;
    int32_t warm;
    int32_t write_iters;
    double eta;           // restart threshold of Algorithm 1 step 6
    int32_t accel;        // restart acceleration (Algorithm 1 steps 6-7) on
    int32_t pad2;
};

// True if the row family handles an instance of this shape; sets the padded sizes.
bool row_supported(int nx, int nu, int N, int tv, int fp64, int* nxp, int* nup);
// Bytes of the per-solve scratch of an instance (abort flag, reduction words,
// halo mailboxes), cleared before every solve, and of its fused stage data.
size_t row_clear_bytes(const InstDev& I);
size_t row_fused_bytes(const InstDev& I);
// Pick the stage blocking (stored in I.row_s) so the grid stays co-resident;
// I.row_s > 0 on entry is the preferred blocking.
hipError_t row_prepare(int fp64, InstDev& I);
// Form the fused stage data of a row-family instance at `fused` (after every
// factorisation; reads the T block written by the factor kernel).
hipError_t launch_row_fuse(const InstDev* d_inst, int inst_idx, const InstDev& I, const void* mats, void* fused,
                           hipStream_t s);
// Enqueue the solve of one row-family instance: clear its per-solve scratch
// (`scratch`, row_clear_bytes(I)) with a fill kernel, then launch the solve.
hipError_t launch_row(int fp64, const RowArgs* a_dev, const InstDev& I, void* scratch, hipStream_t s);

}  // namespace pimpc
