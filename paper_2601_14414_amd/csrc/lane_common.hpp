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


// ---- stage matrices of one time-invariant instance held in LDS
// Rows padded to a multiple of four entries (16-byte aligned rows for FP32,
// two 16-byte pieces per four FP64 entries): J [NU][NBP], H and H_{N-1}
// [NB][NBP], the top rows [A_r B_r] [NX][NBP], then ebar, qbar, lb, ub (NBP
// each).  Rows are read with every lane at the same address (broadcast), and
// LDS answers in order, so rows can be requested ahead behind partial waits
// (a scalar-load stream must wait for all its loads at once).
template <int NX, int NU>
struct MatImg {
    static constexpr int NB = NX + NU;
    static constexpr int NBP = (NB + 3) & ~3;
    static constexpr int J = 0;
    static constexpr int H = J + NU * NBP;
    static constexpr int Hb = H + NB * NBP;
    static constexpr int AB = Hb + NB * NBP;
    static constexpr int E = AB + NX * NBP;
    static constexpr int Q = E + NBP;
    static constexpr int LB = Q + NBP;
    static constexpr int UB = LB + NBP;
    static constexpr int TOT = UB + NBP;
};

// One wave copies the matrices at Mg (offsets o of the time-invariant layout)
// into its image; zeros where the wave has no instance and in the padding.
template <typename T, int NX, int NU, typename O>
__device__ __forceinline__ void fill_mat_img(T* img, const T* Mg, const O o, bool have, int lane) {
    using MI = MatImg<NX, NU>;
    constexpr int NB = MI::NB, NBP = MI::NBP;
    for (int e = lane; e < MI::TOT; e += 64) {
        T val = T(0);
        if (have) {
            if (e < MI::AB) {  // J, H, H_{N-1}: rows of NB
                const int blk = e < MI::H ? 0 : (e < MI::Hb ? 1 : 2);
                const int base = blk == 0 ? MI::J : (blk == 1 ? MI::H : MI::Hb);
                const int r = (e - base) / NBP, c = (e - base) % NBP;
                const int64_t src = blk == 0 ? o.J : (blk == 1 ? o.H : o.Hb);
                if (c < NB) val = Mg[src + r * NB + c];
            } else if (e < MI::E) {  // [A_r B_r]
                const int r = (e - MI::AB) / NBP, c = (e - MI::AB) % NBP;
                if (c < NX)
                    val = Mg[o.A + r * NX + c];
                else if (c < NB)
                    val = Mg[o.B + r * NU + (c - NX)];
            } else {
                const int blk = (e - MI::E) / NBP, c = (e - MI::E) % NBP;
                if (blk == 0) {
                    if (c < NX) val = Mg[o.e + c];
                } else if (c < NB) {
                    val = Mg[(blk == 1 ? o.qbar : (blk == 2 ? o.lb : o.ub)) + c];
                }
            }
        }
        img[e] = val;
    }
}

// one padded row from LDS (16-byte pieces)
template <typename T, int NBP>
__device__ __forceinline__ void lds_row(T (&x)[NBP], const T* p) {
    if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int q = 0; q < NBP / 4; ++q) {
            const float4 t = ((const float4*)p)[q];
            x[4 * q] = t.x;
            x[4 * q + 1] = t.y;
            x[4 * q + 2] = t.z;
            x[4 * q + 3] = t.w;
        }
    } else {
#pragma unroll
        for (int q = 0; q < NBP / 2; ++q) {
            const double2 t = ((const double2*)p)[q];
            x[2 * q] = t.x;
            x[2 * q + 1] = t.y;
        }
    }
}

// Rows 0..R-1 of a padded LDS matrix, body(r, row): row r + D is requested
// before body(r) runs, and a scheduling fence after each row keeps the
// compiler from hoisting further rows (each row in flight holds NBP entries
// of VGPRs).
template <typename T, int R, int NBP, int D = 2, typename B>
__device__ __forceinline__ void lds_rows(const T* base, B&& body) {
    T buf[D + 1][NBP];
#pragma unroll
    for (int r = 0; r < D && r < R; ++r) lds_row(buf[r], base + r * NBP);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        if (r + D < R) lds_row(buf[(r + D) % (D + 1)], base + (r + D) * NBP);
        body(r, buf[r % (D + 1)]);
        __builtin_amdgcn_sched_barrier(0);
    }
}

}  // namespace pimpc
