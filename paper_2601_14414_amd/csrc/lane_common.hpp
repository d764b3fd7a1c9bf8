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

// ---- streaming of uniform rows through SGPRs
template <typename T, int W>
struct SRow {
    T x[W];
};

// Scalar-load W consecutive values at p (uniform).  The opaque copy of the
// pointer keeps the load where it is written (not hoisted ahead of earlier
// rows, which would overflow the SGPRs).
template <typename T, int W>
__device__ __forceinline__ void sload_into(T* dst, cptr<T> p) {
    asm volatile("" : "+s"(p));
#pragma unroll
    for (int j = 0; j < W; ++j) dst[j] = p[j];
}

// Every scalar load issued so far has landed (scalar loads return out of
// order, so only a full wait on the counter is meaningful): lgkmcnt(0).
__device__ __forceinline__ void swait() { __builtin_amdgcn_s_waitcnt(0xC07F); }

// Rows 0..R-1 of a uniform stream: load(r) returns row r, body(r, row)
// consumes it.  With PF, row r + 1 is requested right after row r has landed,
// so its load overlaps body(r); without, each row is loaded, awaited and used
// (fewer SGPRs held, for the widest stages whose registers are full).
template <typename RowT, int R, bool PF, typename L, typename B>
__device__ __forceinline__ void stream_rows(L&& load, B&& body) {
    if constexpr (PF) {
        RowT cur = load(0);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            swait();
            RowT nxt;
            if (r + 1 < R) nxt = load(r + 1);
            body(r, cur);
            cur = nxt;
        }
    } else {
        // two rows per wait: half the exposed latencies for one extra row of SGPRs
#pragma unroll
        for (int r = 0; r < R; r += 2) {
            RowT c0 = load(r), c1;
            if (r + 1 < R) c1 = load(r + 1);
            swait();
            body(r, c0);
            if (r + 1 < R) body(r + 1, c1);
        }
    }
}


}  // namespace pimpc
