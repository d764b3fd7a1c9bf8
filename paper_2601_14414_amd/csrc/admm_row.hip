// admm_row.hip -- row-per-lane ADMM kernel for long single horizons.
//
// Same iteration as the lane kernel (eqn. (8), Algorithm 1 steps 1-5 of
// arXiv 2601.14414, velocity form of Theorem 2) with a different mapping,
// for horizons longer than one lane-family workgroup (e.g. nx = 24, nu = 11,
// N = 1024, where one lane per stage would also leave most of the chip idle,
// or nx = 2, nu = 1, N = 5000); time-invariant or time-varying stage data
// (with time-varying data each wave or group holds its own stage's rows,
// read once per solve):
//   * a wave owns a block of consecutive stages; lane r owns row r of
//     every stage vector.  Wide stages (more than 16 padded rows) give a wave
//     S stages, processed in turn; narrow stages pack G = 64 / NB stages side
//     by side in the lanes of a wave (lane = g NB + r), so a long horizon of
//     small stages (e.g. the 2-state reactor at N = 5000) costs one stage of
//     work per wave and iteration;
//   * the iteration is evaluated in an algebraically equivalent "fused" form
//     whose only dependence on a neighbouring stage is ONE vector each way:
//       with w_k = z_k - v_k - ebar + lambda_k and d_k = z_k - theta_k of the
//       iterate entering the step (so g_k = Abar' w_k, h_k = qbar + rho (d_k + g_{k+1})),
//       b_k      = beta_k + (Bbar J) (v_k - beta_k)                       [= Bbar du_k + beta_k]
//       xbar_k+1 = H q + rho H d_k + rho (H Abar') w_{k+1}                 [= H_k h_k]
//       c_k      = (Abar H q + ebar) + rho (Abar H) d_{k-1}
//                  + rho (Abar H Abar') w_k - lambda_k                     [= Abar xbar_k + ebar - lambda_k]
//     with c_0 = Abar xbar_0 + ebar - lambda_0 and xbar_N = H_{N-1} (q + rho d_{N-1});
//     the products B J, H Abar', Abar H, Abar H Abar', H q, H_{N-1} q and
//     Abar H q + ebar are formed once per factorisation, in FP64
//     (row_fuse_kernel), and rounded once;
//   * so a block needs, per iteration, only w of the stage after it and d of
//     the stage before it: each wave sends w of its first stage to the left
//     and d of its last stage to the right at the end of an iteration, and
//     after the wait only two dot products (one per halo) and the
//     elementwise update remain on the critical path; everything else of
//     the step runs while the halos are in flight;
//   * lane r keeps row r of H, H Abar' and Abar H in VGPRs and row r of
//     B J, Abar H Abar' and column r of [A B] in LDS (lane-private, float4
//     interleaved, conflict free); dot-product inputs are broadcast through
//     a per-wave LDS buffer;
//   * halos travel as 64-bit words (32-bit value, 32-bit tag = iteration), in
//     LDS between waves of a workgroup and in global memory (agent-scope
//     relaxed atomics, no fences needed: every word carries its own tag)
//     between workgroups; two buffers alternate by iteration parity;
//   * every wait is bounded and checks a global abort flag, so a missing
//     neighbour ends the kernel with an error instead of a hang;
//   * logical block order is XCD-aware (hardware workgroup h runs on XCD
//     h mod 8), so neighbouring blocks mostly share an L2;
//   * residuals reduce in wave order on one wave (deterministic).
#include <hip/hip_runtime.h>

#include "pimpc_row.hpp"
#include "lane_common.hpp"

namespace pimpc {

namespace {

constexpr int kSpinLimit = 1 << 22;  // polls before a wait gives up (seconds at worst)
constexpr int kMboxVecs = 3;         // per buffer: w (to the left), d (to the right), dd (to the left)

// Scratch of one row-family instance (16-byte aligned pieces), cleared
// before every solve: abort flag; per-wave residual words [3][nwaves] (c,
// r_prim, r_dual of the wave, each tag << 32 | float bits); global halo
// mailboxes [nwaves][2 buf][3 vec][NBP] (64-bit words); the reducer waves'
// per-workgroup partials of c [nwg], then the decision word.  The fused
// stage data sit elsewhere (written at factorisation time).
// Device pointers carry the global address space, so that every access is a
// global (not flat) instruction and never waits on the LDS counter.
struct RowScratch {
    gptr<int32_t> abort;
    gptr<uint64_t> red;      // [3][nwaves]
    gptr<uint64_t> mbox;     // [nwaves][2][kMboxVecs][NBP]
    gptr<uint64_t> wg_part;  // [nwg] partials, [nwg] decision word (room for 2 nwaves words)
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) / 16 * 16; }

__host__ __device__ inline size_t row_clear_size(int nwaves, int nbp) {
    return align16(16) + align16(24ull * nwaves) + align16(8ull * nwaves * 2 * kMboxVecs * nbp) +
           align16(16ull * nwaves);
}

// Fused block (floats): BJ | HAt | AH | AHAt  [NB][NB] row-major, then
// Hq | Hbq | cq [NB].
__host__ __device__ inline size_t row_fused_floats(int nbp) { return 4ull * nbp * nbp + 3ull * nbp; }

struct FusedOffsets {
    int BJ, HAt, AH, AHAt, Hq, Hbq, cq;
};
__host__ __device__ inline FusedOffsets fused_offsets(int NB) {
    FusedOffsets f;
    f.BJ = 0;
    f.HAt = NB * NB;
    f.AH = 2 * NB * NB;
    f.AHAt = 3 * NB * NB;
    f.Hq = 4 * NB * NB;
    f.Hbq = f.Hq + NB;
    f.cq = f.Hbq + NB;
    return f;
}

__device__ inline RowScratch row_scratch(gptr<char> base, int nwaves, int nbp) {
    gptr<char> p = base;
    RowScratch s;
    s.abort = (gptr<int32_t>)p;
    p += align16(16);
    s.red = (gptr<uint64_t>)p;
    p += align16(24ull * nwaves);
    s.mbox = (gptr<uint64_t>)p;
    p += align16(8ull * nwaves * 2 * kMboxVecs * nbp);
    s.wg_part = (gptr<uint64_t>)p;
    return s;
}

__device__ inline uint64_t pack(float v, uint32_t tag) {
    return ((uint64_t)tag << 32) | (uint64_t)__float_as_uint(v);
}
__device__ inline float unpack_val(uint64_t w) { return __uint_as_float((uint32_t)w); }
__device__ inline uint32_t unpack_tag(uint64_t w) { return (uint32_t)(w >> 32); }

__device__ inline void gstore(gptr<uint64_t> p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t gload(gptr<uint64_t> p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void lstore(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ inline uint64_t lload(uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ inline bool wave_any(bool p) { return __ballot(p) != 0; }

// A wave-uniform loop invariant held in scalar registers.  The argument block
// is constant memory, so without this the compiler may re-load a value from
// it inside the iteration loop (and wait for that load every iteration)
// rather than keep it live.
template <typename T>
__device__ inline T keep_sgpr(T x) {
    asm volatile("" : "+s"(x));
    return x;
}

template <typename T>
__device__ inline T wsum(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}
template <typename T>
__device__ inline T wmax(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Gathers the words base[c * stride + i], i < n, of NC components c, each
// (tag << 32 | float bits), once they all carry `tag`: lane l takes i = l,
// l + 64, ..., and every word it still waits for is in flight at once in
// each poll, so the wait costs about one memory round trip after the last
// word is stored.  v[c][q] = value of word i = 64 q + lane.  Returns false
// (and raises the abort flag) when the wait gives up.
template <int NC, int PER>
__device__ inline bool gather_tagged(gptr<uint64_t> base, size_t stride, int n, uint32_t tag, float (&v)[NC][PER],
                                     gptr<int32_t> abort) {
    const int lane = threadIdx.x & 63;
    uint64_t need = 0, have = 0;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            v[c][q] = 0.f;
            if (q * 64 + lane < n) need |= 1ull << (c * PER + q);
        }
    bool fail = false;
    int spins = 0;
    for (;;) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int q = 0; q < PER; ++q) {
                const uint64_t bit = 1ull << (c * PER + q);
                if ((need & bit) && !(have & bit)) {
                    const uint64_t w = gload(base + c * stride + q * 64 + lane);
                    if (unpack_tag(w) == tag) {
                        v[c][q] = unpack_val(w);
                        have |= bit;
                    }
                }
            }
        if (have == need) break;
        if (++spins > kSpinLimit ||
            ((spins & 31) == 0 && __hip_atomic_load(abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
            __hip_atomic_store(abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            fail = true;
            break;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return !wave_any(fail);
}

constexpr int kFuseMax = 48;  // largest padded stage size of the row family

// Sums and maxima over the lanes of one stage group: G groups of NB lanes
// per wave (NB a power of two when G > 1, so xor shuffles stay inside the
// group; with G = 1 the group is the wave, lanes past the stage holding 0).
template <int G, int NB>
__device__ inline float gsum(float v) {
    if constexpr (G == 1) {
        return wsum(v);
    } else {
#pragma unroll
        for (int off = NB / 2; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        return v;
    }
}
template <int G, int NB>
__device__ inline float gmax(float v) {
    if constexpr (G == 1) {
        return wmax(v);
    } else {
#pragma unroll
        for (int off = NB / 2; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
        return v;
    }
}

// Projection onto one non-box factor (x_k or u_k) of Xbar = X x U, one
// entry per lane (the sets the proof of Theorem 1 lists; formulas of Parikh
// and Boyd, Ch. 6).  `in`: the lane holds entry j of the factor (j < n);
// a_j: its normal entry (halfspace, hyperplane), pn: b or the l1 radius;
// `first`: lane of the factor's entry 0 in this lane's group.  Every lane of
// the wave calls this (the reductions span the group), with the same kind.
template <int G, int NB>
__device__ inline float project_row_factor(float y, bool in, int j, int n, int kind, float a_j, float pn,
                                           int first) {
    if (kind == 1 || kind == 2) {  // halfspace a'w <= b, hyperplane a'w = b
        const float t = gsum<G, NB>(in ? a_j * y : 0.f) - pn;
        const float aa = gsum<G, NB>(in ? a_j * a_j : 0.f);
        if (in && (kind == 2 || t > 0.f)) y -= (t / aa) * a_j;
    } else if (kind == 3) {  // second-order cone ||w_1..w_{n-1}|| <= w_n
        const float q = gsum<G, NB>((in && j < n - 1) ? y * y : 0.f);
        const float t = gsum<G, NB>((in && j == n - 1) ? y : 0.f);
        const float nq = sqrtf(q);
        if (in && !(nq <= t)) {
            const float al = (nq + t) * 0.5f;
            y = (nq <= -t) ? 0.f : (j < n - 1 ? y * (al / nq) : al);
        }
    } else if (kind == 4) {  // l1 ball ||w||_1 <= r: soft threshold at level theta
        const float m = in ? fabsf(y) : 0.f;
        const float l1 = gsum<G, NB>(m);
        // theta = max_j (sum_{|w_i| >= |w_j|} |w_i| - r) / #{i : |w_i| >= |w_j|}
        float sj = 0.f, cj = 0.f;
        for (int i = 0; i < n; ++i) {
            const float mi = __shfl(m, first + i, 64);
            if (mi >= m) {
                sj += mi;
                cj += 1.f;
            }
        }
        const float theta = gmax<G, NB>(in ? (sj - pn) / cj : -INFINITY);
        if (in && l1 > pn) {
            const float a = m - theta;
            y = a > 0.f ? (y > 0.f ? a : -a) : 0.f;
        }
    }
    return y;
}

}  // namespace

// Fused stage data of one time-invariant row-family instance, from the T
// block (FP32 J, H, H_{N-1}, A, B, e, qbar) with FP64 accumulation:
//   BJ = Bbar J, HAt = H Abar', AH = Abar H, AHAt = Abar H Abar',
//   Hq = H qbar, Hbq = H_{N-1} qbar, cq = Abar H qbar + ebar.
__global__ void __launch_bounds__(256) row_fuse_kernel(const InstDev* __restrict__ inst, int inst_idx,
                                                       const float* __restrict__ mats, float* __restrict__ fused) {
    __shared__ double Ab[kFuseMax * kFuseMax];
    __shared__ double Hs[kFuseMax * kFuseMax];
    __shared__ double AHs[kFuseMax * kFuseMax];
    const InstDev I = inst[inst_idx];
    const int NX = I.nxp, NU = I.nup, NB = I.nbp;
    if (NB > kFuseMax) return;  // host side never launches such a shape
    const MatOffsets o = mat_offsets(NX, NU, I.N, 0);
    const float* bt = mats + I.mat_off;
    const FusedOffsets f = fused_offsets(NB);
    const int t = threadIdx.x;
    for (int idx = t; idx < NB * NB; idx += blockDim.x) {
        const int r = idx / NB, c = idx % NB;
        double a;
        if (r < NX)
            a = (c < NX) ? (double)bt[o.A + r * NX + c] : (double)bt[o.B + r * NU + (c - NX)];
        else
            a = (r == c) ? 1.0 : 0.0;
        Ab[idx] = a;
        Hs[idx] = (double)bt[o.H + idx];
    }
    __syncthreads();
    for (int idx = t; idx < NB * NB; idx += blockDim.x) {
        const int r = idx / NB, c = idx % NB;
        double bj = 0.0, hat = 0.0, ah = 0.0;
        for (int u = 0; u < NU; ++u) {
            const double bb = (r < NX) ? (double)bt[o.B + r * NU + u] : ((r - NX) == u ? 1.0 : 0.0);
            bj += bb * (double)bt[o.J + u * NB + c];
        }
        for (int j = 0; j < NB; ++j) {
            hat += Hs[r * NB + j] * Ab[c * NB + j];
            ah += Ab[r * NB + j] * Hs[j * NB + c];
        }
        fused[f.BJ + idx] = (float)bj;
        fused[f.HAt + idx] = (float)hat;
        fused[f.AH + idx] = (float)ah;
        AHs[idx] = ah;
    }
    __syncthreads();
    for (int idx = t; idx < NB * NB; idx += blockDim.x) {
        const int r = idx / NB, c = idx % NB;
        double s = 0.0;
        for (int j = 0; j < NB; ++j) s += AHs[r * NB + j] * Ab[c * NB + j];
        fused[f.AHAt + idx] = (float)s;
    }
    for (int r = t; r < NB; r += blockDim.x) {
        double hq = 0.0, hbq = 0.0, cq = 0.0;
        for (int j = 0; j < NB; ++j) {
            const double q = (double)bt[o.qbar + j];
            hq += Hs[r * NB + j] * q;
            hbq += (double)bt[o.Hb + r * NB + j] * q;
            cq += AHs[r * NB + j] * q;
        }
        if (r < NX) cq += (double)bt[o.e + r];
        fused[f.Hq + r] = (float)hq;
        fused[f.Hbq + r] = (float)hbq;
        fused[f.cq + r] = (float)cq;
    }
}

// Time-varying stage data: one fused block per stage k (workgroup k), from the
// stage-minor T block (element q of stage k at q N + k):
//   BJ_k = Bbar_k J_k, HAt_k = H_k Abar_{k+1}' (k < N-1), AH_k = Abar_k H_{k-1},
//   AHAt_k = Abar_k H_{k-1} Abar_k', cq_k = Abar_k H_{k-1} qbar + ebar_k (k >= 1),
//   Hq_k = H_k qbar (H_{N-1} qbar for the last stage); Hbq is not used.
__global__ void __launch_bounds__(256) row_fuse_tv_kernel(const InstDev* __restrict__ inst, int inst_idx,
                                                          const float* __restrict__ mats,
                                                          float* __restrict__ fused_all) {
    __shared__ double Ab[kFuseMax * kFuseMax];
    __shared__ double Hs[kFuseMax * kFuseMax];
    __shared__ double AHs[kFuseMax * kFuseMax];
    const InstDev I = inst[inst_idx];
    const int NX = I.nxp, NU = I.nup, NB = I.nbp, N = I.N;
    const int k = blockIdx.x;
    if (NB > kFuseMax || k >= N) return;  // host side never launches such a shape
    const MatOffsets o = mat_offsets(NX, NU, N, 1);
    const float* bt = mats + I.mat_off;
    const FusedOffsets f = fused_offsets(NB);
    float* fused = fused_all + (size_t)k * row_fused_floats(NB);
    const int t = threadIdx.x;
    auto abar = [&](int st, int r, int c) -> double {
        if (r < NX)
            return (c < NX) ? (double)bt[o.A + (int64_t)(r * NX + c) * N + st]
                            : (double)bt[o.B + (int64_t)(r * NU + (c - NX)) * N + st];
        return (r == c) ? 1.0 : 0.0;
    };
    auto hmat = [&](int st, int r, int c) -> double { return (double)bt[o.H + (int64_t)(r * NB + c) * N + st]; };
    // BJ_k
    for (int idx = t; idx < NB * NB; idx += blockDim.x) {
        const int r = idx / NB, c = idx % NB;
        double bj = 0.0;
        for (int u = 0; u < NU; ++u) {
            const double bb = (r < NX) ? (double)bt[o.B + (int64_t)(r * NU + u) * N + k] : ((r - NX) == u ? 1.0 : 0.0);
            bj += bb * (double)bt[o.J + (int64_t)(u * NB + c) * N + k];
        }
        fused[f.BJ + idx] = (float)bj;
    }
    // AH_k, AHAt_k, cq_k from Abar_k and H_{k-1}
    if (k >= 1) {
        for (int idx = t; idx < NB * NB; idx += blockDim.x) {
            const int r = idx / NB, c = idx % NB;
            Ab[idx] = abar(k, r, c);
            Hs[idx] = hmat(k - 1, r, c);
        }
        __syncthreads();
        for (int idx = t; idx < NB * NB; idx += blockDim.x) {
            const int r = idx / NB, c = idx % NB;
            double ah = 0.0;
            for (int j = 0; j < NB; ++j) ah += Ab[r * NB + j] * Hs[j * NB + c];
            AHs[idx] = ah;
            fused[f.AH + idx] = (float)ah;
        }
        __syncthreads();
        for (int idx = t; idx < NB * NB; idx += blockDim.x) {
            const int r = idx / NB, c = idx % NB;
            double s = 0.0;
            for (int j = 0; j < NB; ++j) s += AHs[r * NB + j] * Ab[c * NB + j];
            fused[f.AHAt + idx] = (float)s;
        }
        for (int r = t; r < NB; r += blockDim.x) {
            double cq = 0.0;
            for (int j = 0; j < NB; ++j) cq += AHs[r * NB + j] * (double)bt[o.qbar + j];
            if (r < NX) cq += (double)bt[o.e + (int64_t)r * N + k];
            fused[f.cq + r] = (float)cq;
        }
    } else {
        for (int idx = t; idx < NB * NB; idx += blockDim.x) {
            fused[f.AH + idx] = 0.f;
            fused[f.AHAt + idx] = 0.f;
        }
        for (int r = t; r < NB; r += blockDim.x) fused[f.cq + r] = 0.f;
    }
    __syncthreads();
    // HAt_k from H_k and Abar_{k+1}; Hq_k
    for (int idx = t; idx < NB * NB; idx += blockDim.x) {
        const int r = idx / NB, c = idx % NB;
        Hs[idx] = hmat(k, r, c);
        Ab[idx] = (k + 1 < N) ? abar(k + 1, r, c) : 0.0;
    }
    __syncthreads();
    for (int idx = t; idx < NB * NB; idx += blockDim.x) {
        const int r = idx / NB, c = idx % NB;
        double hat = 0.0;
        for (int j = 0; j < NB; ++j) hat += Hs[r * NB + j] * Ab[c * NB + j];
        fused[f.HAt + idx] = (float)hat;
    }
    for (int r = t; r < NB; r += blockDim.x) {
        double hq = 0.0;
        for (int j = 0; j < NB; ++j) hq += Hs[r * NB + j] * (double)bt[o.qbar + j];
        fused[f.Hq + r] = (float)hq;
        fused[f.Hbq + r] = 0.f;
    }
}

// Kernel geometry: kRowWaves compute waves per workgroup, plus kRecvWaves
// receiver waves that poll the global mailboxes of the two neighbouring
// workgroups and forward each halo word into LDS.  Compute waves then never
// load from global memory inside the iteration loop: their halo waits are
// LDS polls, and a poll never sits behind their own outstanding stores (loads
// and stores share one in-order counter on this architecture), so the halo
// round trip overlaps the local part of the step.
constexpr int kRowWaves = 4;
constexpr int kRecvWaves = 2;
constexpr int kRowThreads = 64 * (kRowWaves + kRecvWaves);
// With restart acceleration (Algorithm 1 steps 6-7) a seventh, reducer wave
// sums c^{i+1} over the workgroup's compute waves (LDS), publishes the
// workgroup's partial, gathers every workgroup's partial in a fixed order
// (so all workgroups reach the same sum and the same decision), applies
// steps 5-7 and hands the decision to the compute waves through LDS.
constexpr int kRowThreadsRed = kRowThreads + 64;

// Stage groups per wave: narrow stages (NB <= 16) share a wave side by side.
__host__ __device__ constexpr int row_groups(int nb) { return nb <= 16 ? 64 / nb : 1; }

// Dynamic LDS of one workgroup: per wave, the broadcast rows [3 S G][NB + 4]
// and the lane-private rows of the rows lanes (H, BJ, AHAt: NB each; column
// of [A B]: NX; time-varying data adds the column of the stage's own [A B])
// as float4 [(3 NB + NX (+ NX)) / 4][groups][NB]; time-invariant stage data
// is the same for every group of a wave, so it is held once.
__host__ __device__ constexpr size_t row_lds_bytes(int NX, int NU, int S, bool TV) {
    return (size_t)kRowWaves * (4 * (3 * S * row_groups(NX + NU)) * (NX + NU + 4) +
                                16 * (NX + NU) * ((3 * (NX + NU) + NX + (TV ? NX : 0)) / 4) *
                                    (TV ? row_groups(NX + NU) : 1));
}

extern __shared__ __align__(16) float row_smem[];

template <int NX, int NU, int S, bool TV, bool RED, bool SETS>
__global__ void __launch_bounds__(RED ? kRowThreadsRed : kRowThreads)
    row_kernel(const RowArgs* __restrict__ ap, int nwaves, int nwg) {
    constexpr int NB = NX + NU;
    constexpr int NB4 = NB / 4;
    constexpr int NX4 = NX / 4;
    constexpr int LD = NB + 4;       // LDS row pitch of a broadcast vector (16-byte multiple)
    constexpr int G = row_groups(NB);  // stage groups side by side in a wave
    constexpr int NV = 3 * S * G;      // broadcast rows: (p, d, w) per stage
    static_assert(NB <= 64, "row kernel needs nx + nu <= 64");
    static_assert(G == 1 || S == 1, "packed narrow stages take one stage per group");
    static_assert(!TV || S == 1, "time-varying stage data: one stage per wave or group");
    static_assert(!SETS || S == 1, "non-box sets: one stage per wave or group");
    constexpr int LG = TV ? G : 1;     // groups with their own lane-private rows
    constexpr int NL4 = 3 * NB4 + NX4 + (TV ? NX4 : 0);  // float4 rows per lane
    static_assert(NB % 4 == 0 && NX % 4 == 0, "padded sizes must be multiples of 4");
    const RowArgs& a = *ap;
    const InstDev I = a.inst[a.inst_idx];
    const int N = I.N;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
    // XCD-aware logical workgroup index: hardware workgroup h runs on XCD h % 8.
    int lwg = blockIdx.x;
    if (nwg % 8 == 0) lwg = (blockIdx.x % 8) * (nwg / 8) + blockIdx.x / 8;
    const int gw = lwg * kRowWaves + wv;  // logical wave (block) index
    const int k0 = gw * S * G;
    // stages in this block (a compute wave, gw < nwaves, has at least one)
    const int ns = (S * G == 1) ? 1 : max(0, min(S * G, N - k0));
    const bool rowl = lane < G * NB;            // lane carries a (padded) row
    const int grp = G > 1 ? lane / NB : 0;      // stage group of the lane
    const int r = rowl ? lane - grp * NB : 0;
    const int tb = grp * S;                     // block position of the lane's first stage
    const int nsl = max(0, min(S, ns - tb));    // stages the lane holds
    const int kl = k0 + tb;                     // index of the lane's first stage
    const float rho = (float)a.rho;
    const float third = 1.0f / 3.0f;
    const int K = keep_sgpr(a.K);
    const double eps = keep_sgpr(a.eps);
    const double rho_d = keep_sgpr(a.rho);
    const int check_every = keep_sgpr(a.check_every);

    const gptr<char> sbase = (gptr<char>)(char*)a.scratch;
    RowScratch sc = row_scratch(sbase, nwaves, NB);
    const gptr<const float> F = (gptr<const float>)(const float*)a.fused;
    const FusedOffsets fo = fused_offsets(NB);

    float(*bc)[LD] = (float(*)[LD])(row_smem + (size_t)wv * NV * LD);
    float4* lrow = (float4*)(row_smem + (size_t)kRowWaves * NV * LD) + (size_t)wv * NL4 * LG * NB;
    const int lg = TV ? grp : 0;
#define LROW(q) lrow[((q) * LG + lg) * NB + r]
#define LH(q) LROW(q)
#define LBJ(q) LROW(NB4 + (q))
#define LAHAT(q) LROW(2 * NB4 + (q))
#define LACOL(q) LROW(3 * NB4 + (q))
#define LBCOL(q) LROW(3 * NB4 + NX4 + (q))
    // (16-byte aligned: a halo vector is also read whole, two words per float4)
    __shared__ __align__(16) uint64_t lmbox[kRowWaves][2][kMboxVecs][NB];  // intra-workgroup mailboxes
    __shared__ __align__(16) uint64_t lin[2][2][NB];  // forwarded external halos: [buf][0: w from the right, 1: d from the left]
    // plain values of the w and d halos, written before their tagged words (LDS
    // operations of one wave complete in order), read whole by the consumer
    __shared__ __align__(16) float lmv[kRowWaves][2][2][NB];
    __shared__ __align__(16) float linv[2][2][NB];
    __shared__ int lstop;               // set by the compute waves when they leave the loop
    // restart acceleration: each compute wave's partial of c^{i+1} (value, then
    // its tag), and the reducer's decision (c, extrapolation coefficient,
    // restart count, then the tag word: tag << 32 | stop | nonfinite << 1)
    __shared__ double lcp[kRowWaves];
    __shared__ uint32_t lcpt[kRowWaves];
    __shared__ double ldec_c;
    __shared__ float ldec_coef;
    __shared__ int ldec_rs;
    __shared__ uint64_t ldec_tag;
    for (int i = threadIdx.x; i < kRowWaves * 2 * kMboxVecs * NB; i += blockDim.x) (&lmbox[0][0][0][0])[i] = 0;
    for (int i = threadIdx.x; i < 2 * 2 * NB; i += blockDim.x) (&lin[0][0][0])[i] = 0;
    if (threadIdx.x < kRowWaves) lcpt[threadIdx.x] = 0;
    if (threadIdx.x == 0) {
        lstop = 0;
        ldec_tag = 0;
    }
    __syncthreads();  // no workgroup barrier below this point

    if constexpr (RED) {
        if (wv == kRowWaves + kRecvWaves) {
            // ---- reducer wave: for every iteration, c^{i+1} (tag i + 2) of the
            // whole horizon, then steps 5-7 of Algorithm 1 (reading R11: the
            // eps stop is tested first; c_prev starts at 1 and takes c^{i+1}
            // after every decision; a restart sets alpha = 1 and hats = the
            // current iterate)
            const int first = lwg * kRowWaves;
            const int nin = min(kRowWaves, nwaves - first);  // compute waves of this workgroup
            const double eta = keep_sgpr(a.eta);
            const bool accel = keep_sgpr(a.accel) != 0;
            double alpha = 1.0, cprev = 1.0;
            int restarts = 0;
            int ck = check_every;
            for (int it = 0; it < K; ++it) {
                // c of this step is reduced every step with acceleration, else
                // every check_every-th step (for the eps stop)
                if (!accel) {
                    if (--ck != 0) continue;
                    ck = check_every;
                }
                const uint32_t tag = (uint32_t)it + 2;
                bool fail = false;
                // this workgroup's partial: its compute waves' partials in wave order
                double part = 0.0;
                for (int w = 0; w < nin && !fail; ++w) {
                    int spins = 0;
                    while (__hip_atomic_load(&lcpt[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != tag) {
                        if ((++spins & 31) == 0) {
                            if (__hip_atomic_load(&lstop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0 ||
                                __hip_atomic_load(sc.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                                fail = true;
                                break;
                            }
                            if (spins > kSpinLimit) {
                                __hip_atomic_store(sc.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                fail = true;
                                break;
                            }
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);  // the value read stays after the tag
                    if (!fail) part += lcp[w];
                }
                if (fail) return;
                // publish this workgroup's partial; the reducer of workgroup 0
                // gathers them all and publishes the decision in one word that
                // the other reducers poll (two hops, but one reader of the
                // partials and one word for the rest: an all-to-all gather has
                // every reducer hammer the same few cache lines).  One slot is
                // enough: a workgroup's next partial needs this decision, which
                // needs every partial of this step to have been read.
                if (lane == 0) gstore(sc.wg_part + lwg, pack((float)part, tag));
                const gptr<uint64_t> dword = sc.wg_part + nwg;  // tag << 32 | payload
                constexpr uint32_t kStopWord = 0xFFFFFFFFu, kNonfiniteWord = 0xFFFFFFFEu;
                bool stop = false, nonfinite = false;
                float coef = 0.f;
                double c = 0.0;
                if (lwg == 0) {
                    // workgroup order (lane l takes l, l + 64, ...), then a fixed
                    // shuffle tree: deterministic
                    float val[1][16];
                    if (!gather_tagged<1, 16>(sc.wg_part, 0, nwg, tag, val, sc.abort)) return;
                    double cs = 0.0;
#pragma unroll
                    for (int q = 0; q < 16; ++q) cs += (double)val[0][q];
                    cs = wsum(cs);
                    c = rho_d * cs;
                    nonfinite = !(c < INFINITY);
                    stop = nonfinite || (eps > 0.0 && c <= eps);
                    if (!stop && accel) {
                        if (c <= eta * cprev) {
                            const double a1 = 0.5 + 0.5 * sqrt(1.0 + 4.0 * alpha * alpha);
                            coef = (float)((alpha - 1.0) / a1);
                            alpha = a1;
                        } else {
                            alpha = 1.0;
                            ++restarts;
                        }
                        cprev = c;
                    }
                    const uint32_t payload = nonfinite ? kNonfiniteWord : (stop ? kStopWord : __float_as_uint(coef));
                    if (lane == 0) gstore(dword, ((uint64_t)tag << 32) | payload);
                } else {
                    uint64_t d = 0;
                    int spins = 0;
                    for (;;) {
                        d = gload(dword);
                        if ((uint32_t)(d >> 32) == tag) break;
                        if (++spins > kSpinLimit ||
                            ((spins & 31) == 0 &&
                             __hip_atomic_load(sc.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)) {
                            __hip_atomic_store(sc.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            return;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                    const uint32_t payload = (uint32_t)d;
                    nonfinite = payload == kNonfiniteWord;
                    stop = nonfinite || payload == kStopWord;
                    coef = stop ? 0.f : __uint_as_float(payload);
                }
                if (lane == 0) {
                    ldec_c = c;  // (workgroup 0 only: the info record's c)
                    ldec_coef = coef;
                    ldec_rs = restarts;
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);  // payload before tag (in-order LDS)
                    __hip_atomic_store(&ldec_tag,
                                       ((uint64_t)tag << 32) | (stop ? 1u : 0u) | (nonfinite ? 2u : 0u),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                if (stop) return;
            }
            return;
        }
    }

    if (wv >= kRowWaves) {
        // ---- receiver wave: side 0 forwards w of the first stage of the right
        // workgroup, side 1 forwards d of the last stage of the left one, for
        // every tag the compute waves will consume (1 .. K)
        const int side = wv - kRowWaves;
        const int first = lwg * kRowWaves;
        const int last = min(first + kRowWaves, nwaves) - 1;
        const int src = side == 0 ? last + 1 : first - 1;
        const bool has = side == 0 ? (last == first + kRowWaves - 1 && src < nwaves) : (first > 0);
        if (!has || lane >= NB) return;
        const int vec = side == 0 ? 0 : 1;
        for (int t = 1; t <= K; ++t) {
            const gptr<uint64_t> p = sc.mbox + ((size_t)(src * 2 + (t & 1)) * kMboxVecs + vec) * NB + lane;
            int spins = 0;
            for (;;) {
                const uint64_t word = gload(p);
                if (unpack_tag(word) == (uint32_t)t) {
                    linv[t & 1][side][lane] = unpack_val(word);
                    __atomic_signal_fence(__ATOMIC_SEQ_CST);  // value before tag (in-order LDS)
                    lstore(&lin[t & 1][side][lane], word);
                    break;
                }
                if ((++spins & 31) == 0) {
                    if (__hip_atomic_load(&lstop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0 ||
                        __hip_atomic_load(sc.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
                        return;
                    if (spins > kSpinLimit) {
                        __hip_atomic_store(sc.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        return;
                    }
                }
            }
        }
        return;
    }
    if (gw >= nwaves) return;

    // ---- per-lane stage data, padded entries are 0.  Time-varying data is
    // that of the lane's own stage ks (its fused block, and element q of the
    // stage-minor T block at q N + ks); a group past the horizon reads the
    // last stage and never uses it.
    const MatOffsets o = mat_offsets(NX, NU, N, TV);
    const gptr<const float> M = (gptr<const float>)((const float*)a.mats + I.mat_off);
    const int ks = TV ? min(kl, N - 1) : 0;
    const int kn = TV ? min(ks + 1, N - 1) : 0;  // the next stage (its Abar enters the dual residual)
    const gptr<const float> Fk = F + (size_t)ks * row_fused_floats(NB);
    auto tvi = [&](int64_t base, int q, int st) -> float {  // element q of a stage-minor block, or row-major
        return TV ? M[base + (int64_t)q * N + st] : M[base + q];
    };
    float HAr[NB], AHr[NB];  // the two matrices of the halo terms stay in VGPRs
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        HAr[j] = rowl ? Fk[fo.HAt + r * NB + j] : 0.f;
        AHr[j] = rowl ? Fk[fo.AH + r * NB + j] : 0.f;
    }
    // With one stage per wave and at most 36 rows, the lane's row of H is
    // held in VGPRs as well (H_{N-1} in the wave of the last stage), so that
    // the local part of a step reads two lane-private rows from LDS instead
    // of three: LDS bandwidth bounds that part, since every compute wave of a
    // CU reads its own rows each iteration.
    constexpr bool RH = S == 1 && NB <= 36;
    const bool last_h = !TV && kl == N - 1;  // time-varying: stage N-1's own H is H_{N-1}
    float Hr[RH ? NB : 1];
    if constexpr (RH) {
#pragma unroll
        for (int j = 0; j < NB; ++j)
            Hr[j] = rowl ? (last_h ? M[o.Hb + r * NB + j] : tvi(o.H, r * NB + j, ks)) : 0.f;
    }
    if (rowl) {
        auto ld4 = [&](gptr<const float> p) { return make_float4(p[0], p[1], p[2], p[3]); };
#pragma unroll
        for (int q = 0; q < NB4; ++q) {
            if constexpr (!RH)
                LH(q) = make_float4(tvi(o.H, r * NB + 4 * q + 0, ks), tvi(o.H, r * NB + 4 * q + 1, ks),
                                    tvi(o.H, r * NB + 4 * q + 2, ks), tvi(o.H, r * NB + 4 * q + 3, ks));
            LAHAT(q) = ld4(Fk + fo.AHAt + r * NB + 4 * q);
            LBJ(q) = ld4(Fk + fo.BJ + r * NB + 4 * q);
        }
    }
    // column r of the top block [A B] (rows i < NX) of stage st
    auto acol = [&](int i, int st) -> float {
        return rowl ? (r < NX ? tvi(o.A, i * NX + r, st) : tvi(o.B, i * NU + (r - NX), st)) : 0.f;
    };
    if (rowl) {
#pragma unroll
        for (int q = 0; q < NX4; ++q)
            LACOL(q) = make_float4(acol(4 * q + 0, kn), acol(4 * q + 1, kn), acol(4 * q + 2, kn), acol(4 * q + 3, kn));
        if constexpr (TV) {
#pragma unroll
            for (int q = 0; q < NX4; ++q)
                LBCOL(q) =
                    make_float4(acol(4 * q + 0, ks), acol(4 * q + 1, ks), acol(4 * q + 2, ks), acol(4 * q + 3, ks));
        }
    }
    const float e_r = (rowl && r < NX) ? tvi(o.e, r, ks) : 0.f;  // ebar_r of the stage
    const float lb_r = rowl ? M[o.lb + r] : 0.f;
    const float ub_r = rowl ? M[o.ub + r] : 0.f;
    const float hbd_r = (rowl && !TV) ? M[o.Hb + r * NB + r] : 0.f;
    // non-box factors: kinds, the lane's entry of the normal and b or r
    const int xkind = SETS ? I.xset : 0, ukind = SETS ? I.uset : 0;
    const bool in_x = SETS && rowl && r < I.nx;
    const bool in_u = SETS && rowl && r >= NX && r - NX < I.nu;
    const float ax_r = in_x ? M[o.sx + r] : 0.f, bx = SETS ? M[o.sx + NX] : 0.f;
    const float au_r = in_u ? M[o.su + (r - NX)] : 0.f, bu = SETS ? M[o.su + NU] : 0.f;
    const float Hq_r = rowl ? Fk[fo.Hq + r] : 0.f;
    const float Hbq_r = rowl ? Fk[fo.Hbq + r] : 0.f;
    const float cq_r = rowl ? Fk[fo.cq + r] : 0.f;
    const bool hb_diag = I.hb_diag != 0;

    // c_0 = Abar xbar_0 + ebar (stage 0 only), xbar_0 = col(x(t), u(t-1))
    float c0_r = 0.f;
    if (k0 == 0 && ns > 0) {
        float xb0 = 0.f;
        if (rowl && r < NX && r < I.nx) xb0 = ((const float*)a.x0)[I.x_off + r];
        if (rowl && r >= NX && r - NX < I.nu && a.uprev) xb0 = ((const float*)a.uprev)[I.u_off + r - NX];
        if (rowl) bc[0][r] = xb0;
        __builtin_amdgcn_wave_barrier();
        if (rowl) {
            float s = e_r;
            if (r < NX) {
#pragma unroll
                for (int j = 0; j < NB; ++j) s += (j < NX ? tvi(o.A, r * NX + j, 0) : tvi(o.B, r * NU + (j - NX), 0)) * bc[0][j];
            } else {
                s = xb0;
            }
            c0_r = s;
        }
        __builtin_amdgcn_wave_barrier();
    }

    // ---- iterate rows of the S stages
    float v[S], z[S], th[S], be[S], la[S], pv[S], xs[S];
    const gptr<float> st = (gptr<float>)((float*)a.state + I.st_off);
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const bool ld = a.warm && rowl && s < nsl;
        const int k = kl + s;
        v[s] = ld ? st[(size_t)(0 * NB + r) * N + k] : 0.f;
        z[s] = ld ? st[(size_t)(1 * NB + r) * N + k] : 0.f;
        th[s] = ld ? st[(size_t)(2 * NB + r) * N + k] : 0.f;
        be[s] = ld ? st[(size_t)(3 * NB + r) * N + k] : 0.f;
        la[s] = ld ? st[(size_t)(4 * NB + r) * N + k] : 0.f;
        pv[s] = 0.f;
        xs[s] = 0.f;
    }
    // Restart acceleration: the previous iterate, and the step-1 products of
    // it.  Step 1 is affine in the hats, and the hats are an affine
    // combination of the current and the previous iterate,
    //   hat = cur + coef (cur - prev),
    // so the products of the hats are the same combination of the products of
    // the two iterates.  The mat-vecs therefore run on the current iterate
    // while the restart decision (which needs c of the whole horizon) is in
    // flight, and the combination is formed once the decision is known.
    constexpr int SA = RED ? S : 1;
    float pvv[SA], pzz[SA], pth[SA], pbe[SA], pla[SA];  // previous iterate
    float lbb[SA], lxl[SA], lcl[SA];                    // products of the previous iterate
#pragma unroll
    for (int s = 0; s < SA; ++s) {
        pvv[s] = v[s];
        pzz[s] = z[s];
        pth[s] = th[s];
        pbe[s] = be[s];
        pla[s] = la[s];
        lbb[s] = lxl[s] = lcl[s] = 0.f;
    }

    const bool has_left = ns > 0 && k0 > 0;
    const bool has_right = ns > 0 && k0 + ns < N;
    const bool left_in_wg = wv > 0;
    const bool right_in_wg = wv < kRowWaves - 1;
    auto mbox_g = [&](int wave, int buf, int vec) -> gptr<uint64_t> {
        return sc.mbox + ((size_t)(wave * 2 + buf) * kMboxVecs + vec) * NB + r;
    };
    auto put = [&](bool in_wg, int buf, int vec, uint64_t word) {
        if (in_wg) {
            if (vec < 2) {
                lmv[wv][buf][vec][r] = unpack_val(word);
                __atomic_signal_fence(__ATOMIC_SEQ_CST);  // value before tag (in-order LDS)
            }
            lstore(&lmbox[wv][buf][vec][r], word);
        } else {
            gstore(mbox_g(gw, buf, vec), word);
        }
    };
    bool failed = false;
    // Stage vectors of the iterate: w = z - v - ebar + lambda, d = z - theta.
    auto wvec = [&](int s) { return z[s] - v[s] - e_r + la[s]; };
    auto dvec = [&](int s) { return z[s] - th[s]; };
    // w of the first stage goes left, d of the last stage goes right (each
    // written by the lanes that hold that stage)
    const int sl = ns - 1 - tb;  // the block's last stage, as an index into the lane's stages
    auto publish = [&](uint32_t tag) {
        if (!rowl) return;
        const int buf = tag & 1;
        if (has_left && tb == 0) put(left_in_wg, buf, 0, pack(wvec(0), tag));
        if (has_right && sl >= 0 && sl < S) {
            float zl = z[0], tl = th[0];
#pragma unroll
            for (int s = 1; s < S; ++s)
                if (s == sl) {
                    zl = z[s];
                    tl = th[s];
                }
            put(right_in_wg, buf, 1, pack(zl - tl, tag));
        }
    };

    publish(1u);  // the initial iterate carries tag 1
    // Let every load of the set-up complete here, so the loop header does not
    // carry a wait for them (which, inside the loop, would also wait for the
    // previous iteration's halo stores).
    __builtin_amdgcn_s_waitcnt(0);

    int iters = 0;
    double c_last = 0.0, rp_last = 0.0, rd_last = 0.0;
    int status = 0;

    // per-lane residual terms of the last step (kept for the final pass with
    // restart acceleration)
    float cpart = 0.f, rpart = 0.f;
    float ddv[S], dzv[S], dvv[S];
#pragma unroll
    for (int s = 0; s < S; ++s) ddv[s] = dzv[s] = dvv[s] = 0.f;
    // Residuals of the step that produced the iterate with tag `tout`:
    // c^{i+1}, r_prim and r_dual of the whole horizon, reduced on wave 0.
    // Each wave has already sent dd of its first stage to the left.
    auto residuals = [&](const uint32_t tout) {
        // dual residual (Section IV-B): du block Bbar_k' dv_k and xbar block
        // dz_{k+1} + Abar_{k+1}' (dz_{k+2} - dv_{k+1}); with the top rows of
        // Abar' as column r of [A B]: (Abar' x)_r = [r >= NX] x_r + sum_i [A B]_{i r} x_i.
        float ddR = 0.f;
        if (has_right && rowl) {
            uint64_t* lp = &lmbox[wv + 1 < kRowWaves ? wv + 1 : wv][tout & 1][2][r];
            const gptr<uint64_t> gp = mbox_g(gw + 1 < nwaves ? gw + 1 : gw, tout & 1, 2);
            int spins = 0;
            for (;;) {
                uint64_t wd;
                if (right_in_wg)
                    wd = lload(lp);
                else
                    wd = gload(gp);
                if (unpack_tag(wd) == tout) {
                    ddR = unpack_val(wd);
                    break;
                }
                if ((++spins & 31) == 0) {
                    if (__hip_atomic_load(sc.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                        spins > kSpinLimit) {
                        __hip_atomic_store(sc.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        failed = true;
                        break;
                    }
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        float rdpart = 0.f;
        // dd of the next stage when it sits in the next group of lanes
        const float ddg = (G > 1) ? __shfl(ddv[0], lane + NB < 64 ? lane + NB : lane, 64) : 0.f;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (s < nsl) {
                const int t = tb + s;
                float ddn = (t + 1 < ns) ? (G > 1 ? ddg : 0.f) : ddR;
#pragma unroll
                for (int u = 1; u < S; ++u)
                    if (u == s + 1 && t + 1 < ns) ddn = ddv[u];
                const bool hasnext = kl + s + 1 < N;
                if (rowl) {
                    bc[3 * tb + 0][r] = dvv[s];
                    bc[3 * tb + 1][r] = ddn;
                }
                __builtin_amdgcn_wave_barrier();
                if (rowl) {
                    float bt = (r >= NX) ? dvv[s] : 0.f;
                    float tg = (r >= NX) ? ddn : 0.f;
#pragma unroll
                    for (int q = 0; q < NX4; ++q) {
                        const float4 c4 = LACOL(q);  // Abar_{k+1} (the next stage's)
                        float4 b4 = c4;                // Bbar_k (this stage's)
                        if constexpr (TV) b4 = LBCOL(q);
                        const float4 x4 = *(const float4*)&bc[3 * tb + 0][4 * q];
                        const float4 y4 = *(const float4*)&bc[3 * tb + 1][4 * q];
                        bt += b4.x * x4.x + b4.y * x4.y + b4.z * x4.z + b4.w * x4.w;
                        tg += c4.x * y4.x + c4.y * y4.y + c4.z * y4.z + c4.w * y4.w;
                    }
                    if (r >= NX) rdpart = fmax(rdpart, fabsf(bt));
                    rdpart = fmax(rdpart, fabsf(dzv[s] + (hasnext ? tg : 0.f)));
                }
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (!rowl) cpart = rpart = rdpart = 0.f;
        const double csum = wsum((double)cpart);
        const double rpm = wmax((double)rpart);
        const double rdm = wmax((double)rdpart);
        if (lane == 0) {
            gstore(sc.red + gw, pack((float)csum, tout));
            gstore(sc.red + nwaves + gw, pack((float)rpm, tout));
            gstore(sc.red + 2 * nwaves + gw, pack((float)rdm, tout));
        }
        if (gw == 0) {
            // deterministic reduction: lane l takes waves l, l + 64, ... in
            // order, then a fixed shuffle tree combines the lanes
            float val[3][16];
            const bool ok = gather_tagged<3, 16>(sc.red, (size_t)nwaves, nwaves, tout, val, sc.abort);
            double cs = 0.0, rp = 0.0, rd = 0.0;
#pragma unroll
            for (int q = 0; q < 16; ++q) {
                cs += (double)val[0][q];
                rp = fmax(rp, (double)val[1][q]);
                rd = fmax(rd, (double)val[2][q]);
            }
            cs = wsum(cs);
            rp = wmax(rp);
            rd = wmax(rd);
            if (lane == 0) {
                c_last = rho_d * cs;
                rp_last = rp;
                rd_last = rho_d * rd;
                if (!(c_last < INFINITY)) status = -4;
                if (!ok) status = -5;
            }
        }
    };

    int ck = check_every;  // steps left until c next goes to the reducer (eps stop)
    const bool accel = RED && keep_sgpr(a.accel) != 0;
    bool pub_prev = false;  // the previous step's c went to the reducer: its decision is due
#pragma unroll 1
    for (int it = 0; it < K; ++it) {
        const uint32_t tin = (uint32_t)it + 1;   // tag of the iterate this step reads
        const uint32_t tout = (uint32_t)it + 2;  // tag of the iterate it produces
        // residuals every check_every-th iteration when stopping on eps, and
        // after the last one
        // the plain kernel (fixed K) forms the residuals after the last step;
        // with a reducer wave, c goes to it after every step (acceleration) or
        // every check_every-th step (eps stop), and r_prim, r_dual are formed
        // once, after the loop
        const bool check = !RED && it == K - 1;
        bool pub = false;
        if constexpr (RED) {
            pub = accel;
            if (!accel && --ck == 0) {
                pub = true;
                ck = check_every;
            }
        }

        // ---- halo mailboxes of the iterate entering this step (LDS only): w of
        // the stage after the block, d of the stage before it, from the
        // neighbouring wave or, across workgroups, as forwarded by a receiver
        const int hbuf = tin & 1;
        uint64_t* prb = right_in_wg ? &lmbox[wv + 1 < kRowWaves ? wv + 1 : wv][hbuf][0][0] : &lin[hbuf][0][0];
        uint64_t* plb = left_in_wg ? &lmbox[wv > 0 ? wv - 1 : 0][hbuf][1][0] : &lin[hbuf][1][0];
        const float* prv = right_in_wg ? &lmv[wv + 1 < kRowWaves ? wv + 1 : wv][hbuf][0][0] : &linv[hbuf][0][0];
        const float* plv = left_in_wg ? &lmv[wv > 0 ? wv - 1 : 0][hbuf][1][0] : &linv[hbuf][1][0];
        uint64_t* pr = prb + r;
        uint64_t* pl = plb + r;
        uint64_t wr = 0, wl = 0;
        auto poll = [&]() {
            if (has_right) wr = lload(pr);
            if (has_left) wl = lload(pl);
        };

        // ---- local part of the step (no halo needed)
        float bb[S], xl[S], cl[S];
        if (rowl) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                if (s < nsl) {
                    const float p_ = v[s] - be[s];
                    if constexpr (!RED) pv[s] = p_;  // with acceleration: from the hats, below
                    bc[3 * (tb + s) + 0][r] = p_;
                    bc[3 * (tb + s) + 1][r] = dvec(s);
                    bc[3 * (tb + s) + 2][r] = wvec(s);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        if (rowl) {
#pragma unroll
            for (int s = 0; s < S; ++s) {
                if (s < nsl) {
                    const int k = kl + s;
                    const int t = tb + s;
                    float ab0 = 0.f, ab1 = 0.f, ah0 = 0.f, ah1 = 0.f, ac0 = 0.f, ac1 = 0.f;
                    if constexpr (RH) {
#pragma unroll
                        for (int q = 0; q < NB4; ++q) {
                            const float4 p4 = *(const float4*)&bc[3 * t + 0][4 * q];
                            const float4 d4 = *(const float4*)&bc[3 * t + 1][4 * q];
                            const float4 w4 = *(const float4*)&bc[3 * t + 2][4 * q];
                            const float4 g = LBJ(q);
                            const float4 m = LAHAT(q);
                            ab0 += g.x * p4.x;
                            ab1 += g.y * p4.y;
                            ab0 += g.z * p4.z;
                            ab1 += g.w * p4.w;
                            ah0 += Hr[4 * q + 0] * d4.x;
                            ah1 += Hr[4 * q + 1] * d4.y;
                            ah0 += Hr[4 * q + 2] * d4.z;
                            ah1 += Hr[4 * q + 3] * d4.w;
                            ac0 += m.x * w4.x;
                            ac1 += m.y * w4.y;
                            ac0 += m.z * w4.z;
                            ac1 += m.w * w4.w;
                            // (unrolled for the register row; the scheduler
                            // may hoist every column's loads: measured 1-4 %
                            // faster than capping it at three columns)
                        }
                    } else {
                    // all operands come from LDS; a partly unrolled loop keeps
                    // the scheduler from hoisting every load (VGPR pressure)
#pragma unroll 3
                    for (int q = 0; q < NB4; ++q) {
                        const float4 p4 = *(const float4*)&bc[3 * t + 0][4 * q];
                        const float4 d4 = *(const float4*)&bc[3 * t + 1][4 * q];
                        const float4 w4 = *(const float4*)&bc[3 * t + 2][4 * q];
                        const float4 g = LBJ(q);
                        const float4 m = LAHAT(q);
                        const float4 h = LH(q);
                        ab0 += g.x * p4.x;
                        ab1 += g.y * p4.y;
                        ab0 += g.z * p4.z;
                        ab1 += g.w * p4.w;
                        ah0 += h.x * d4.x;
                        ah1 += h.y * d4.y;
                        ah0 += h.z * d4.z;
                        ah1 += h.w * d4.w;
                        ac0 += m.x * w4.x;
                        ac1 += m.y * w4.y;
                        ac0 += m.z * w4.z;
                        ac1 += m.w * w4.w;
                    }
                    }
                    bb[s] = be[s] + (ab0 + ab1);
                    if (RH) {  // Hr holds H_{N-1} in the last stage's wave
                        xl[s] = (last_h ? Hbq_r : Hq_r) + rho * (ah0 + ah1);
                    } else if (!TV && k == N - 1) {  // time-varying: the last stage's own H is H_{N-1}
                        // xbar_N = H_{N-1} (q + rho d)
                        float hb = 0.f;
                        if (hb_diag) {
                            hb = hbd_r * bc[3 * t + 1][r];
                        } else {
                            const gptr<const float> Hb = M + o.Hb + r * NB;
#pragma unroll
                            for (int j = 0; j < NB; ++j) hb += Hb[j] * bc[3 * t + 1][j];
                        }
                        xl[s] = Hbq_r + rho * hb;
                    } else {
                        xl[s] = Hq_r + rho * (ah0 + ah1);
                    }
                    cl[s] = (k == 0) ? c0_r - la[s] : cq_r + rho * (ac0 + ac1) - la[s];
                } else {
                    bb[s] = xl[s] = cl[s] = 0.f;
                }
            }
            // neighbours inside the block
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const int t = tb + s;
                if (s < nsl && t + 1 < ns) {  // xbar_{k+1} += rho (H Abar') w_{k+1}
                    float x0 = 0.f, x1 = 0.f;
#pragma unroll
                    for (int q = 0; q < NB4; ++q) {
                        const float4 w4 = *(const float4*)&bc[3 * (t + 1) + 2][4 * q];
                        x0 += HAr[4 * q + 0] * w4.x;
                        x1 += HAr[4 * q + 1] * w4.y;
                        x0 += HAr[4 * q + 2] * w4.z;
                        x1 += HAr[4 * q + 3] * w4.w;
                    }
                    xl[s] += rho * (x0 + x1);
                }
                if (s < nsl && t >= 1) {  // c_k += rho (Abar H) d_{k-1}
                    float x0 = 0.f, x1 = 0.f;
#pragma unroll
                    for (int q = 0; q < NB4; ++q) {
                        const float4 d4 = *(const float4*)&bc[3 * (t - 1) + 1][4 * q];
                        x0 += AHr[4 * q + 0] * d4.x;
                        x1 += AHr[4 * q + 1] * d4.y;
                        x0 += AHr[4 * q + 2] * d4.z;
                        x1 += AHr[4 * q + 3] * d4.w;
                    }
                    cl[s] += rho * (x0 + x1);
                }
            }
        } else {
#pragma unroll
            for (int s = 0; s < S; ++s) bb[s] = xl[s] = cl[s] = 0.f;
        }

        // ---- halos of the iterate entering this step: w of the stage after
        // the block, d of the stage before it.  Both words are loaded together
        // each poll, so a poll costs one memory round trip.
        if ((has_right || has_left) && rowl) {
            int spins = 0;
            poll();
            for (;;) {
                const bool okr = !has_right || unpack_tag(wr) == tin;
                const bool okl = !has_left || unpack_tag(wl) == tin;
                if (okr && okl) break;
                if ((++spins & 31) == 0) {
                    if (__hip_atomic_load(sc.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                        failed = true;
                        break;
                    }
                    if (spins > kSpinLimit) {
                        __hip_atomic_store(sc.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        failed = true;
                        break;
                    }
                }
                __builtin_amdgcn_s_sleep(1);
                poll();
            }
        }
        if (__builtin_amdgcn_readfirstlane((int)failed) || wave_any(failed)) {
            status = -5;
            break;
        }
        // ---- halo terms: xbar of the last stage and c of the first stage.
        // Every lane has seen its own word of both halo vectors carry the tag,
        // and each word's plain value was stored before it by the same wave,
        // so the value arrays are read whole (four values per float4, the
        // same address in every lane).  Both products are always formed (a
        // missing side reads a harmless buffer) and only the existing sides
        // are added.
        __atomic_signal_fence(__ATOMIC_SEQ_CST);  // the value reads stay after the polls
        if (rowl && (has_right || has_left)) {
            float x0 = 0.f, x1 = 0.f, x2 = 0.f, x3 = 0.f, y0 = 0.f, y1 = 0.f, y2 = 0.f, y3 = 0.f;
            float4 wq[NB4], dq[NB4];  // all reads in flight at once
#pragma unroll
            for (int q = 0; q < NB4; ++q) {
                wq[q] = *(const float4*)(prv + 4 * q);
                dq[q] = *(const float4*)(plv + 4 * q);
            }
#pragma unroll
            for (int q = 0; q < NB4; ++q) {
                x0 += HAr[4 * q + 0] * wq[q].x;
                y0 += AHr[4 * q + 0] * dq[q].x;
                x1 += HAr[4 * q + 1] * wq[q].y;
                y1 += AHr[4 * q + 1] * dq[q].y;
                x2 += HAr[4 * q + 2] * wq[q].z;
                y2 += AHr[4 * q + 2] * dq[q].z;
                x3 += HAr[4 * q + 3] * wq[q].w;
                y3 += AHr[4 * q + 3] * dq[q].w;
            }
            if (has_right) {
#pragma unroll
                for (int s = 0; s < S; ++s)
                    if (s == sl) xl[s] += rho * ((x0 + x1) + (x2 + x3));
            }
            if (has_left && tb == 0) cl[0] += rho * ((y0 + y1) + (y2 + y3));
        }

        if constexpr (RED) {
            // ---- steps 6-7: the decision taken on c^{i} of the previous
            // step (none before the first step, where the hats are the
            // initial iterate)
            float coef = 0.f;
            if (pub_prev) {
                const uint64_t want = (uint64_t)(it + 1);
                uint64_t d = 0;
                int spins = 0;
                for (;;) {
                    d = __hip_atomic_load(&ldec_tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    if ((d >> 32) == want) break;
                    if ((++spins & 31) == 0) {
                        if (__hip_atomic_load(sc.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                            spins > kSpinLimit) {
                            __hip_atomic_store(sc.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            failed = true;
                            break;
                        }
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                __atomic_signal_fence(__ATOMIC_SEQ_CST);  // the payload read stays after the tag
                if (failed) {
                    status = -5;
                    break;
                }
                if (d & 2u) status = -4;  // c^{i} is not finite
                if (d & 1u) break;        // step 5: c^{i} <= eps (the iterate stays the current one)
                coef = accel ? ldec_coef : 0.f;
            }
#pragma unroll
            for (int s = 0; s < S; ++s) {
                const float b_ = bb[s], x_ = xl[s], c_ = cl[s];
                bb[s] = b_ + coef * (b_ - lbb[s]);
                xl[s] = x_ + coef * (x_ - lxl[s]);
                cl[s] = c_ + coef * (c_ - lcl[s]);
                lbb[s] = b_;
                lxl[s] = x_;
                lcl[s] = c_;
                auto hat = [&](float& cur, float& prv) {
                    const float h = cur + coef * (cur - prv);
                    prv = cur;
                    cur = h;
                };
                hat(v[s], pvv[s]);
                hat(z[s], pzz[s]);
                hat(th[s], pth[s]);
                hat(be[s], pbe[s]);
                hat(la[s], pla[s]);
                pv[s] = v[s] - be[s];  // du of this step is J (vhat - betahat)
            }
        }

        // ---- steps 2-3 (Theorem 1 closed form, box projection, dual update)
        // (lanes without a row hold zeros throughout: their bounds are [0, 0])
        cpart = 0.f;
        rpart = 0.f;
        float yset = 0.f;  // non-box factors: Theorem 1's point projected factor by factor
        if constexpr (SETS) {
            yset = (2.f * (xl[0] + th[0]) + bb[0] + cl[0]) * third;
            yset = project_row_factor<G, NB>(yset, in_x, r, I.nx, xkind, ax_r, bx, grp * NB);
            yset = project_row_factor<G, NB>(yset, in_u, r - NX, I.nu, ukind, au_r, bu, grp * NB + NX);
        }
#pragma unroll
        for (int s = 0; s < S; ++s) {
            ddv[s] = dzv[s] = dvv[s] = 0.f;
            if (s < nsl) {
                const float bi = bb[s], ci = cl[s], xi = xl[s];
                const float gam = bi - ci;
                // (a non-box factor stores +-inf bounds, so the clamp only zeroes padding)
                const float y = SETS ? yset : (2.f * (xi + th[s]) + bi + ci) * third;
                const float zn = y < lb_r ? lb_r : (y > ub_r ? ub_r : y);
                const float vn = (zn + gam) * 0.5f;
                const float thn = th[s] + xi - zn;
                const float ben = bi - vn;
                const float lan = zn - vn - ci;
                if (check || RED) {
                    const float dv = vn - v[s], dz = zn - z[s];
                    const float dth = thn - th[s], dbe = ben - be[s], dla = lan - la[s];
                    const float dd = dz - dv;
                    cpart += dth * dth + dbe * dbe + dla * dla + dz * dz + dv * dv + dd * dd;
                    rpart = fmax(rpart, fmax(fabsf(dth), fmax(fabsf(dbe), fabsf(dla))));
                    ddv[s] = dd;
                    dzv[s] = dz;
                    dvv[s] = dv;
                }
                xs[s] = xi;
                v[s] = vn;
                z[s] = zn;
                th[s] = thn;
                be[s] = ben;
                la[s] = lan;
            }
        }
        publish(tout);
        ++iters;
        if constexpr (RED) pub_prev = pub;
        if (RED && pub) {
            // this wave's partial of c^{i+1}, for the reducer wave
            const double csum = wsum((double)(rowl ? cpart : 0.f));
            if (lane == 0) {
                lcp[wv] = csum;
                __atomic_signal_fence(__ATOMIC_SEQ_CST);  // value before tag (in-order LDS)
                __hip_atomic_store(&lcpt[wv], tout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }

    }

    // leaving before K iterations (stop decision or failure): no compute wave
    // of this workgroup consumes another halo, so the receivers may end too
    if (iters < K && lane == 0) __hip_atomic_store(&lstop, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);

    // ---- residuals of the last step (after the loop, so that the gather's
    // registers do not weigh on the loop); with a reducer wave, c^{i+1} and
    // the restart count are the reducer's when the last step's c went to it
    int restarts_out = 0;
    if (!failed && iters > 0) {
        const uint32_t tf = (uint32_t)iters + 1;
        if (has_left && rowl && tb == 0) put(left_in_wg, tf & 1, 2, pack(ddv[0], tf));
        residuals(tf);
    }
    if constexpr (RED) {
        if (!failed && iters > 0) {
            const uint32_t tf = (uint32_t)iters + 1;
            if (gw == 0 && pub_prev) {  // the last step's c went to the reducer
                uint64_t d = 0;
                int spins = 0;
                for (;;) {
                    d = __hip_atomic_load(&ldec_tag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                    if ((uint32_t)(d >> 32) == tf) break;
                    if ((++spins & 31) == 0 &&
                        (__hip_atomic_load(sc.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                         spins > kSpinLimit)) {
                        __hip_atomic_store(sc.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        status = -5;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                }
                __atomic_signal_fence(__ATOMIC_SEQ_CST);  // the payload reads stay after the tag
                if (status != -5) {
                    c_last = ldec_c;
                    restarts_out = ldec_rs;
                    if (d & 2u) status = -4;
                }
            }
        }
    }

    // ---- outputs: final iterate; du_k = J_k (v_k - beta_k) and xbar_{k+1}
    // of the last step 1
    float du[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
        du[s] = 0.f;
        if (s < nsl) {
            if (rowl) bc[3 * tb][r] = pv[s];
            __builtin_amdgcn_wave_barrier();
            if (rowl && r < NU) {
                float acc = 0.f;
                for (int j = 0; j < NB; ++j) acc += tvi(o.J, r * NB + j, min(kl + s, N - 1)) * bc[3 * tb][j];
                du[s] = acc;
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (rowl) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (s < nsl) {
                const int k = kl + s;
                st[(size_t)(0 * NB + r) * N + k] = v[s];
                st[(size_t)(1 * NB + r) * N + k] = z[s];
                st[(size_t)(2 * NB + r) * N + k] = th[s];
                st[(size_t)(3 * NB + r) * N + k] = be[s];
                st[(size_t)(4 * NB + r) * N + k] = la[s];
                if (a.write_iters) {
                    const gptr<float> io = (gptr<float>)((float*)a.iters_out + I.it_off);
                    if (r < NU) io[(size_t)r * N + k] = du[s];
                    io[(size_t)(NU + r) * N + k] = xs[s];
                }
            }
        }
    }
    if (k0 == 0 && ns > 0 && lane < I.nu) {
        const float up = a.uprev ? ((const float*)a.uprev)[I.u_off + lane] : 0.f;
        ((float*)a.u0)[I.u_off + lane] = up + du[0];
    }
    if (gw == 0 && lane == 0 && a.info) {
        InfoDev rec;
        rec.iters = iters;
        rec.restarts = restarts_out;
        rec.c = c_last;
        rec.r_prim = rp_last;
        rec.r_dual = rd_last;
        rec.status = (a.fbad && a.fbad[a.inst_idx]) ? -3 : status;  // -3: the factorisation failed (not SPD)
        rec.pad = 0;
        a.info[a.inst_idx] = rec;
    }
#undef LH
#undef LBJ
#undef LAHAT
#undef LACOL
#undef LBCOL
#undef LROW
}

template <typename T>
hipError_t launch_fill(T*, int64_t, T, hipStream_t);

// ------------------------------------------------------------------ host side

namespace {

struct RowCfg {
    int nx, nu;
};
// Padded stage classes of the row family, narrowest first: (4, 4) and (8, 8)
// pack 8 and 4 stages per wave and serve long horizons of small stages (e.g.
// the 2-state, 1-input reactor at N = 5000).
constexpr RowCfg kRowCfgs[] = {{4, 4}, {8, 8}, {24, 12}, {32, 16}};

template <int NX, int NU, int S, bool TV, bool RED, bool SETS>
hipError_t row_launch_t(const RowArgs* a_dev, int nwaves, int nwg, hipStream_t s, int* occ) {
    const size_t lds = row_lds_bytes(NX, NU, S, TV);
    constexpr int threads = RED ? kRowThreadsRed : kRowThreads;
    static bool attr_set = false;
    if (!attr_set) {
        hipError_t e = hipFuncSetAttribute((const void*)row_kernel<NX, NU, S, TV, RED, SETS>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        attr_set = true;
    }
    if (occ)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, row_kernel<NX, NU, S, TV, RED, SETS>, threads, lds);
    hipLaunchKernelGGL((row_kernel<NX, NU, S, TV, RED, SETS>), dim3(nwg), dim3(threads), lds, s, a_dev, nwaves,
                       nwg);
    return hipGetLastError();
}

template <int NX, int NU, bool RED, bool SETS>
hipError_t row_launch_s(int S, bool tv, const RowArgs* a_dev, int nwaves, int nwg, hipStream_t s, int* occ) {
    if (tv) {  // time-varying stage data: one stage per wave or group
        if (S != 1) return hipErrorInvalidValue;
        return row_launch_t<NX, NU, 1, true, RED, SETS>(a_dev, nwaves, nwg, s, occ);
    }
    // packed narrow stages, non-box sets: one stage per wave or group
    if constexpr (SETS || row_groups(NX + NU) > 1) {
        if (S != 1) return hipErrorInvalidValue;
        return row_launch_t<NX, NU, 1, false, RED, SETS>(a_dev, nwaves, nwg, s, occ);
    } else {
        switch (S) {
            case 1:
                return row_launch_t<NX, NU, 1, false, RED, false>(a_dev, nwaves, nwg, s, occ);
            case 2:
                return row_launch_t<NX, NU, 2, false, RED, false>(a_dev, nwaves, nwg, s, occ);
            case 4:
                return row_launch_t<NX, NU, 4, false, RED, false>(a_dev, nwaves, nwg, s, occ);
            default:
                return hipErrorInvalidValue;
        }
    }
}

template <bool RED, bool SETS>
hipError_t row_launch_cls(const InstDev& I, int S, const RowArgs* a_dev, int nwaves, int nwg, hipStream_t s,
                          int* occ) {
    const bool tv = I.tv != 0;
    if (I.nxp == 4 && I.nup == 4) return row_launch_s<4, 4, RED, SETS>(S, tv, a_dev, nwaves, nwg, s, occ);
    if (I.nxp == 8 && I.nup == 8) return row_launch_s<8, 8, RED, SETS>(S, tv, a_dev, nwaves, nwg, s, occ);
    if (I.nxp == 24 && I.nup == 12) return row_launch_s<24, 12, RED, SETS>(S, tv, a_dev, nwaves, nwg, s, occ);
    if (I.nxp == 32 && I.nup == 16) return row_launch_s<32, 16, RED, SETS>(S, tv, a_dev, nwaves, nwg, s, occ);
    return hipErrorInvalidValue;
}

hipError_t row_launch_any(const InstDev& I, int S, const RowArgs* a_dev, hipStream_t s, int* occ) {
    const int per = S * row_groups(I.nbp);  // stages per wave
    const int nwaves = (I.N + per - 1) / per;
    const int nwg = (nwaves + kRowWaves - 1) / kRowWaves;
    const bool sets = I.xset != 0 || I.uset != 0;
    if (I.row_acc)
        return sets ? row_launch_cls<true, true>(I, S, a_dev, nwaves, nwg, s, occ)
                    : row_launch_cls<true, false>(I, S, a_dev, nwaves, nwg, s, occ);
    return sets ? row_launch_cls<false, true>(I, S, a_dev, nwaves, nwg, s, occ)
                : row_launch_cls<false, false>(I, S, a_dev, nwaves, nwg, s, occ);
}

int num_cus() {
    static int n = 0;
    if (!n) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            n = 256;
    }
    return n;
}

}  // namespace

// LDS of one row-kernel workgroup: the dynamic part plus the static mailboxes
// (lmbox, lin, lmv, linv, lstop as declared in the kernel).
constexpr size_t row_total_lds(int NX, int NU, bool tv) {
    const size_t NB = (size_t)(NX + NU);
    return row_lds_bytes(NX, NU, 1, tv) + 8 * NB * (kRowWaves * 2 * kMboxVecs + 4) + 4 * NB * (kRowWaves * 4 + 4) + 16 +
           12 * kRowWaves + 32;
}
constexpr size_t kRowLdsLimit = 160 * 1024;  // per workgroup on gfx950

bool row_supported(int nx, int nu, int N, int tv, int fp64, int* nxp, int* nup) {
    (void)N;
    if (fp64) return false;
    for (const RowCfg& c : kRowCfgs)
        if (nx <= c.nx && nu <= c.nu) {
            // time-varying data keeps a second column set per lane; the widest
            // class then exceeds the workgroup's LDS
            if (tv && row_total_lds(c.nx, c.nu, true) > kRowLdsLimit) return false;
            *nxp = c.nx;
            *nup = c.nu;
            return true;
        }
    return false;
}

// Per-solve scratch sized for one stage per wave (an upper bound for every
// blocking); fused stage data, one block per stage when the stage data is
// time-varying.
size_t row_clear_bytes(const InstDev& I) { return align16(row_clear_size(I.N, I.nbp)); }
size_t row_fused_bytes(const InstDev& I) { return align16(4 * row_fused_floats(I.nbp) * (I.tv ? I.N : 1)); }

// Choose the blocking S (stages per wave): the smallest S whose grid stays
// co-resident (every workgroup must be running for the halo waits to end).
hipError_t row_prepare(int fp64, InstDev& I) {
    (void)fp64;
    const int want = I.row_s > 0 ? I.row_s : 1;
    for (int S : {want, 1, 2, 4}) {
        // packed narrow stages, time-varying data, non-box sets: S = 1
        if (S > 1 && (row_groups(I.nbp) > 1 || I.tv || I.xset != 0 || I.uset != 0)) break;
        int occ = 0;
        hipError_t e = row_launch_any(I, S, nullptr, nullptr, &occ);
        if (e != hipSuccess) return e;
        const int per = S * row_groups(I.nbp);
        const int nwg = ((I.N + per - 1) / per + kRowWaves - 1) / kRowWaves;
        // (the reducer wave of the accelerated kernel gathers at most 1024
        // workgroup partials)
        if (occ > 0 && nwg <= occ * num_cus() && (!I.row_acc || nwg <= 1024)) {
            I.row_s = S;
            return hipSuccess;
        }
    }
    return hipErrorInvalidConfiguration;
}

hipError_t launch_row_fuse(const InstDev* d_inst, int inst_idx, const InstDev& I, const void* mats, void* fused,
                           hipStream_t s) {
    if (I.nbp > kFuseMax) return hipErrorInvalidValue;
    if (I.tv)
        hipLaunchKernelGGL(row_fuse_tv_kernel, dim3(I.N), dim3(256), 0, s, d_inst, inst_idx, (const float*)mats,
                           (float*)fused);
    else
        hipLaunchKernelGGL(row_fuse_kernel, dim3(1), dim3(256), 0, s, d_inst, inst_idx, (const float*)mats,
                           (float*)fused);
    return hipGetLastError();
}

hipError_t launch_row(int fp64, const RowArgs* a_dev, const InstDev& I, void* scratch, hipStream_t s) {
    (void)fp64;
    const int S = I.row_s > 0 ? I.row_s : 1;
    hipError_t e = launch_fill<int32_t>((int32_t*)scratch, (int64_t)(row_clear_size(I.N, I.nbp) / 4), 0, s);
    if (e != hipSuccess) return e;
    return row_launch_any(I, S, a_dev, s, nullptr);
}

}  // namespace pimpc
