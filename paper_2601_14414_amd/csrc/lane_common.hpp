// lane_common.hpp -- device helpers shared by the lane-per-stage kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pimpc {

// Explicit address spaces: constant (4) for read-only data with uniform
// addresses (scalar loads), global (1) for per-lane data.  Needed because the
// per-class bodies are separate functions whose pointer arguments would
// otherwise be generic (flat) pointers.
#if defined(__HIP_DEVICE_COMPILE__)
template <typename T>
using cptr = const T __attribute__((address_space(4)))*;
template <typename T>
using gptr = T __attribute__((address_space(1)))*;
#else  // the host pass only parses device code; plain pointers suffice there
template <typename T>
using cptr = const T*;
template <typename T>
using gptr = T*;
#endif


// Mark a pointer as wave-uniform (kept in SGPRs; loads through it become
// scalar loads).  Only valid for pointers that are equal across the wave.
template <typename P>
__device__ inline P* uniform_ptr(P* p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (P*)(((uint64_t)hi << 32) | lo);
}

}  // namespace pimpc
