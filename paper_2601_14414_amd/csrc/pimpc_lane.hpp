// pimpc_lane.hpp -- host/device interface of the lane-per-stage kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "pimpc_dev.hpp"

#ifndef PIMPC_LANE_NPARTS
#define PIMPC_LANE_NPARTS 6
#endif

namespace pimpc {

struct LaneArgs {
    const InstDev* inst;
    const Bin* bins;
    int32_t nbins;
    int32_t* bin_counter;  // nullptr: static bin = blockIdx.x + j * gridDim.x
    const void* mats;
    void* state;
    void* iters_out;
    const void* x0;
    const void* uprev;
    void* u0;
    InfoDev* info;
    double rho;
    double eps;
    int32_t K;
    int32_t check_every;
    int32_t warm;
    int32_t nbmax;
    int32_t write_iters;
    int32_t ckpt_every;  // > 0: store the iterate entering every ckpt_every-th iteration
    void* ckpt;          // checkpoint buffer (T), per instance at InstDev::ck_off
    int32_t accel;       // 1: restart acceleration (Algorithm 1 steps 6-7)
    int32_t pad_;
    double eta;          // restart threshold
    void* prev;          // accel: previous actual iterate (T, state layout)
    const int32_t* fbad; // per instance: non-zero when its stage factorisation failed (not SPD)
    void* tape;          // non-null (FP32, time-invariant boxes): record every iteration's step for the
                         // reverse sweep, per instance at InstDev::tape_off (no checkpoints then)
};

// gs != 0 selects the kernel variant that projects onto non-box sets.
// rec != 0 selects the variant that records every step for the backward.
template <int P>
hipError_t lane_dispatch(int fp64, int cls, int gs, bool rec, const LaneArgs* a_dev, int bw, int grid,
                         hipStream_t s, int* occ, bool* handled);

// Whether a class of padded stage size nb fits the lane kernel in this
// precision: the iterate, the step-1 outputs and the temporaries of one
// stage live in the registers of one lane, which bounds FP64 classes.
constexpr bool lane_fp64_class(int nb) { return nb <= 13; }
inline bool lane_class_fits(int nb, size_t tsize) { return tsize == 4 || lane_fp64_class(nb); }
// Classes with a backward kernel (padded nx + nu <= 16), and so with a
// forward variant that records every step.
constexpr bool lane_rec_class(int nb) { return nb <= 16; }

}  // namespace pimpc
