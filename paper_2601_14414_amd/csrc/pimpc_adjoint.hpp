// pimpc_adjoint.hpp -- host interface of the backward (adjoint) kernels.
#pragma once
#include <hip/hip_runtime.h>

#include "pimpc_dev.hpp"

namespace pimpc {

// Words per stage and step of the backward's segment tape: d = v - beta (nb),
// h (nb), the top rows of w = z - v - ebar + lambda (nx) and the box mask of
// the projection (one word).
__host__ __device__ constexpr int tape_rec_floats(int nb, int nx) { return 2 * nb + nx + 1; }

struct BwdArgs {
    const InstDev* inst;
    const Bin* bins;
    int32_t nbins;
    int32_t* bin_counter;
    const float* mats;
    const float* ckpt;
    float* tape;
    float* grads;
    const float* x0;
    const float* uprev;
    const float* dLdu0;
    double rho;
    int32_t K;
    int32_t ckpt_every;
    int32_t full_tape;  // 1: the forward recorded all K steps (tape of K records, no checkpoints)
    int32_t pad_;
};

// Backward of one lane class (time-invariant, FP32, padded nx + nu <= 16).
hipError_t launch_backward_class(int cls, const BwdArgs& a, int grid, hipStream_t s, bool* handled);
bool backward_class_supported(int cls);
// FP64 chain from the raw adjoints to dL/d(x0, diag Q, diag R, A, B).
hipError_t launch_chain(const InstDev* inst, int count, const double* mats64, const float* grads, double rho,
                        float* dx0, float* dQd, float* dRd, float* dA, float* dB, hipStream_t s);

}  // namespace pimpc
