// adjoint.hip -- reverse mode through the unrolled ADMM iterations.
//
// Differentiable form of the solver (the paper names a differentiable piMPC
// as future work in its conclusion; the transpose below is derived from the
// closed-form iteration of eqn. (8) / Algorithm 1 steps 1-3).  The loss sees
// u0 = u_prev + du_0 of the K-th step 1, and depends on (x0, diag Q, diag R,
// A, B) of every instance.
//
// Backward kernel (one lane per stage, same bins as the forward):
//   * the taped forward stored the iterate entering every ckpt_every-th
//     iteration; the backward re-runs each segment from its checkpoint into a
//     per-instance tape (per stage and step: d = v - beta, h, the top rows of
//     w and the box mask), then walks it in reverse.  With ckpt_every = 1 the
//     forward wrote that record for every step itself, and the backward only
//     walks it;
//   * per reverse step it applies the exact transpose of steps 2-3, then of
//     step 1, recomputing du = J d and xbar = H h from the record in the same
//     passes over J and H that the transposes make; the halo directions are
//     reversed (the adjoint of xbar_k goes to stage k-1, the adjoint of
//     g_{k+1} to stage k+1);
//   * the stage matrices come from a per-wave LDS image (stages up to 12
//     wide) or stream through SGPRs one row ahead (wider stages);
//   * parameter adjoints are sums over stages and iterations of outer
//     products (e.g. Hbar += xbar_bar h^T).  Each wave stages the vectors of
//     its 64 stages in LDS and contracts over the stages with FP32 MFMA
//     (16x16x4), two products per round, accumulating in 16x16 tiles: the
//     one dense contraction on this path.
// Chain kernel (FP64, one workgroup per instance): maps the adjoints of
// H_a, H_{N-1}, J and the Abar/Bbar blocks to dA, dB, diag Q, diag R through
// M_bar = -H Hbar H and the derivative of J = (Bbar'Bbar)^-1 Bbar'.
#include <hip/hip_runtime.h>

#include "lane_common.hpp"
#include "pimpc_dev.hpp"
#include "pimpc_lane.hpp"
#include "pimpc_adjoint.hpp"

namespace pimpc {

typedef float floatx4 __attribute__((ext_vector_type(4)));


// The backward runs in 256-thread workgroups (bins of at most 4 waves) so that
// each wave may use the whole 512-entry register file of its SIMD.
constexpr int kBwdThreads = 256;
constexpr int kBwdWaves = kBwdThreads / 64;
constexpr int kBBD = kBwdThreads;  // LDS row stride of the halo buffers
extern __shared__ __align__(16) unsigned char bwd_smem[];

// C += V1 V2^T over the 64 stages of this wave.  Each lane passes its stage's
// two 16-vectors; they are staged as [stage][16] and fed to the MFMA so that
// lane l supplies V1[l % 16][4t + l / 16] and V2[l % 16][4t + l / 16].
// The four float4 slots of stage s are rotated by ((s >> 1) + (s >> 3)) mod 4:
// without it the 16-float rows put the even lanes of a 128-bit write on the
// same banks (a 4-way conflict); with it every write and read is
// conflict-free for 32 and for 64 banks.
//
// A wave's staging tile holds six such [64][16] areas: each product's two
// vectors are written to their areas as soon as they are final (so they do
// not stay live in registers through the rest of the step), and one round
// then runs two products' MFMA chains interleaved.  After the areas: the
// last stage's xsb and h (32 floats) and the x0 adjoint (16 floats).
constexpr int kStgArea = 64 * 16;                 // floats per staged vector
constexpr int kStgFloats = 6 * kStgArea + 64;     // six areas + 64 floats
__device__ inline int stage_rot(int s) { return ((s >> 1) + (s >> 3)) & 3; }

__device__ inline void stage_write(float* area, const float (&v)[16], int lane) {
    float4* d = (float4*)(area + lane * 16);
    const int wr = stage_rot(lane);
#pragma unroll
    for (int q = 0; q < 4; ++q) d[(q + wr) & 3] = make_float4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
}

// offset, within an area, of element i = lane % 16 of stage st = 4 t + kk,
// kk = lane / 16: st * 16 + 4 ((i / 4 + stage_rot(st)) mod 4) + i mod 4.
// With st / 2 = 2 t + kk / 2 and st / 8 = t / 2, stage_rot(st) is
// kk / 2 + (2 t + t / 2) mod 4, so the offset is 64 t plus one of four
// per-lane bases (four VGPRs for all sixteen t; 64 t goes into the
// instruction's offset field).
__device__ inline int stage_base(int r, int lane) {
    const int i = lane & 15, kk = lane >> 4;
    return kk * 16 + 4 * (((i >> 2) + (kk >> 1) + r) & 3) + (i & 3);
}
__device__ inline int stage_off(int t, int lane) { return 64 * t + stage_base((2 * t + (t >> 1)) & 3, lane); }

// C += A B^T from two staged areas
__device__ inline void stage_mfma(floatx4& C, const float* A, const float* B, int lane) {
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int off = stage_off(t, lane);
        C = __builtin_amdgcn_mfma_f32_16x16x4f32(A[off], B[off], C, 0, 0, 0);
    }
    __builtin_amdgcn_wave_barrier();
}

// C1 += A1 B1^T and C2 += A2 B2^T, the two chains interleaved
__device__ inline void stage_mfma2(floatx4& C1, const float* A1, const float* B1, floatx4& C2, const float* A2,
                                   const float* B2, int lane) {
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int off = stage_off(t, lane);
        C1 = __builtin_amdgcn_mfma_f32_16x16x4f32(A1[off], B1[off], C1, 0, 0, 0);
        C2 = __builtin_amdgcn_mfma_f32_16x16x4f32(A2[off], B2[off], C2, 0, 0, 0);
    }
    __builtin_amdgcn_wave_barrier();
}

__device__ inline void stage_accum(floatx4& C, const float (&v1)[16], const float (&v2)[16], float* stg,
                                   int lane) {
    stage_write(stg, v1, lane);
    stage_write(stg + kStgArea, v2, lane);
    stage_mfma(C, stg, stg + kStgArea, lane);
}

// The stage matrices of a wave's instance, copied once per bin into the
// wave's own LDS image (MatImg): every class's image fits this slot.
constexpr int kMatFloats = 832;  // the widest class: 4 x 16 + 2 x 16 x 16 + 12 x 16 + 4 x 16

// Where a step reads its stage matrices: the LDS image (LR, stages up to
// twelve floats wide), or the global copy streamed through SGPRs one row
// ahead (wider stages: their per-lane vectors leave no VGPRs for rows).
// body(r, x) gets row r in x[0..NB).
template <int NX, int NU, bool LR>
struct MatView {
    static constexpr int NB = NX + NU;
    static constexpr int NBP = (NB + 3) & ~3;
    using MI = MatImg<NX, NU>;
    using Row = SRow<float, NBP>;
    const float* L;  // the LDS image
    cptr<float> G;   // the global matrices
    MatOffsets o;
    __device__ float e(int i) const { if constexpr (LR) return L[MI::E + i]; else return G[o.e + i]; }
    __device__ float qb(int i) const { if constexpr (LR) return L[MI::Q + i]; else return G[o.qbar + i]; }
    __device__ float lb(int i) const { if constexpr (LR) return L[MI::LB + i]; else return G[o.lb + i]; }
    __device__ float ub(int i) const { if constexpr (LR) return L[MI::UB + i]; else return G[o.ub + i]; }
    __device__ float j(int r, int c) const {
        if constexpr (LR) return L[MI::J + r * NBP + c]; else return G[o.J + r * NB + c];
    }
    template <typename B>
    __device__ __forceinline__ void rowsJ(B&& body) const {
        if constexpr (LR) {
            lds_rows<float, NU, NBP>(L + MI::J, body);
        } else {
            stream_rows<Row, NU, true>(
                [&](int r) {
                    Row x;
                    sload_into<float, NB>(x.x, G + o.J + r * NB);
                    return x;
                },
                [&](int r, const Row& x) { body(r, x.x); });
        }
    }
    // the top rows [A_r B_r]
    template <typename B>
    __device__ __forceinline__ void rowsAB(B&& body) const {
        if constexpr (LR) {
            lds_rows<float, NX, NBP>(L + MI::AB, body);
        } else {
            stream_rows<Row, NX, true>(
                [&](int r) {
                    Row x;
                    sload_into<float, NX>(x.x, G + o.A + r * NX);
                    sload_into<float, NU>(x.x + NX, G + o.B + r * NU);
                    return x;
                },
                [&](int r, const Row& x) { body(r, x.x); });
        }
    }
    // H, or H_{N-1} where `last` (body assigns, so the second pass overwrites)
    template <typename B>
    __device__ __forceinline__ void rowsH(bool last, B&& body) const {
        if constexpr (LR) {
            lds_rows<float, NB, NBP>(L + (last ? MI::Hb : MI::H), body);
        } else {
            auto pass = [&](int64_t off) {
                stream_rows<Row, NB, true>(
                    [&](int r) {
                        Row x;
                        sload_into<float, NB>(x.x, G + off + r * NB);
                        return x;
                    },
                    [&](int r, const Row& x) { body(r, x.x); });
            };
            pass(o.H);
            if (last) pass(o.Hb);
        }
    }
};

// FULL: the forward recorded all K steps (no checkpoints, no re-run); a
// variant of its own, so that the re-running kernel keeps its registers.
template <int NX, int NU, bool FULL>
__device__ __forceinline__ void bwd_run(const BwdArgs& a, int inst_idx, bool have, int gw0,
                                        unsigned leader_mask) {
    constexpr int NB = NX + NU;
    static_assert(NB <= 16, "the backward kernel supports nx + nu <= 16");
    inst_idx = __builtin_amdgcn_readfirstlane(inst_idx);
    gw0 = __builtin_amdgcn_readfirstlane(gw0);
    have = __builtin_amdgcn_readfirstlane((int)have) != 0;
    const InstDev I = ((cptr<InstDev>)uniform_ptr(a.inst))[have ? inst_idx : 0];
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int k = tid - gw0 * 64;
    const int N = have ? I.N : 0;
    const bool act = have && k >= 0 && k < N;
    const float rho = (float)a.rho;
    const float third = 1.0f / 3.0f;
    const MatOffsets o = mat_offsets(NX, NU, have ? N : 1, 0);
    const cptr<float> M0 = (cptr<float>)uniform_ptr(have ? a.mats + I.mat_off : a.mats);
    // LDS: three halo buffers [16][kBBD] (stage to stage: xg towards k - 1,
    // xx and xq towards k + 1), then one staging tile per wave
    float* xg = (float*)bwd_smem;
    float* xx = xg + 16 * kBBD;
    float* xq = xx + 16 * kBBD;
    float* stg0 = xq + 16 * kBBD;
    float* stg = stg0 + wave * kStgFloats;  // this wave's staging tile
    using MI = MatImg<NX, NU>;
    constexpr int NBP = MI::NBP;
    constexpr bool kLdsRows = NBP <= 12;
    float* mw = stg0 + kBwdWaves * kStgFloats + wave * kMatFloats;  // this wave's matrix image
    static_assert(MI::TOT <= kMatFloats, "the matrix image exceeds its LDS slot");
    if constexpr (kLdsRows) {
        fill_mat_img<float, NX, NU>(mw, a.mats + (have ? I.mat_off : 0), o, have, lane);
        __builtin_amdgcn_wave_barrier();
    }

    const cptr<float> x0p = (cptr<float>)uniform_ptr(a.x0 + (have ? I.x_off : 0));
    const cptr<float> upp = (cptr<float>)uniform_ptr(a.uprev ? a.uprev + (have ? I.u_off : 0) : nullptr);
    const int nx_real = have ? I.nx : 0, nu_real = have ? I.nu : 0;
    // xbar_0 = (x0, u_prev), read where stage 0 needs it
    auto xb0 = [&](int i) -> float {
        return i < NX ? (i < nx_real ? x0p[i] : 0.f) : ((upp && i - NX < nu_real) ? upp[i - NX] : 0.f);
    };
    const bool is_last = act && k == N - 1;
    const bool last_wave = have && (N - 1) / 64 == wave - gw0;  // the wave that holds stage N - 1
    // J_bar and the top rows of B_bar share one 16 x 16 tile when they fit:
    // rows dub (NU) then bb (NX), columns d (NB) then du (NU)
    constexpr bool kMergeBJ = NB + NU <= 16;

// the stage matrices behind opaque offsets: their reads stay in the step
// that makes them (not hoisted out of the iteration loops into registers)
#define MATS()                                  \
    int mo_ = 0;                                \
    asm volatile("" : "+s"(mo_));               \
    cptr<float> mg_ = M0;                       \
    asm volatile("" : "+s"(mg_));               \
    const MatView<NX, NU, kLdsRows> mv{mw + mo_, mg_, o};

    float v[NB], z[NB], th[NB], be[NB], la[NB];
    float sv[NB], sz[NB], sth[NB], sbe[NB], sla[NB];  // adjoint of the iterate entering the step
#pragma unroll
    for (int i = 0; i < NB; ++i) sv[i] = sz[i] = sth[i] = sbe[i] = sla[i] = 0.f;
    // [0, 32): the last stage's xsb and h; [32, 48): the x0 adjoint; [48, 64):
    // xbar_0 (read by stage 0 in every step, so kept in LDS rather than
    // re-read through the scalar cache)
    float* lw = stg + 6 * kStgArea;
    if (lane < 16) {
        lw[32 + lane] = 0.f;
        lw[48 + lane] = lane < NB ? xb0(lane) : 0.f;
    }
    __builtin_amdgcn_wave_barrier();
    floatx4 CHa = {0, 0, 0, 0}, CHb = {0, 0, 0, 0}, CJ = {0, 0, 0, 0}, CA = {0, 0, 0, 0}, CB = {0, 0, 0, 0};

    auto load_state = [&](const float* base) {
        const gptr<float> p = (gptr<float>)base;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            v[i] = act ? p[(int64_t)(0 * NB + i) * N + k] : 0.f;
            z[i] = act ? p[(int64_t)(1 * NB + i) * N + k] : 0.f;
            th[i] = act ? p[(int64_t)(2 * NB + i) * N + k] : 0.f;
            be[i] = act ? p[(int64_t)(3 * NB + i) * N + k] : 0.f;
            la[i] = act ? p[(int64_t)(4 * NB + i) * N + k] : 0.f;
        }
    };

    // Step 1 of the iteration from the current iterate: du, h, xbar (two barriers).
    float du[NU], h[NB], xs[NB], d[NB];
    auto step1 = [&]() {
        MATS()
#pragma unroll
        for (int i = 0; i < NB; ++i) d[i] = v[i] - be[i];
        float g[NB];
#pragma unroll
        for (int c = 0; c < NB; ++c) g[c] = (c < NX) ? 0.f : (z[c] - v[c] + la[c]);
        // du = J d, and g = Abar' w from the top rows [A_r B_r]
        mv.rowsJ([&](int r, const float (&x)[NBP]) {
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < NB; ++j) s += x[j] * d[j];
            du[r] = s;
        });
        mv.rowsAB([&](int rr, const float (&x)[NBP]) {
            const float w = z[rr] - v[rr] - mv.e(rr) + la[rr];
#pragma unroll
            for (int c = 0; c < NB; ++c) g[c] += x[c] * w;
        });
#pragma unroll
        for (int c = 0; c < NB; ++c) xg[c * kBBD + tid] = g[c];
        __syncthreads();
        const bool hasnext = act && (k + 1 < N);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const float gv = xg[i * kBBD + tid + 1];
            h[i] = mv.qb(i) + rho * (z[i] - th[i] + (hasnext ? gv : 0.f));
        }
        // xbar_{k+1} = H h (H_{N-1} for the last stage)
        mv.rowsH(is_last, [&](int r, const float (&x)[NBP]) {
            float s = 0.f;
#pragma unroll
            for (int j = 0; j < NB; ++j) s += x[j] * h[j];
            xs[r] = s;
        });
#pragma unroll
        for (int i = 0; i < NB; ++i) xx[i * kBBD + tid] = xs[i];
        __syncthreads();
    };
    // Steps 2-3 given xbar_k (xp): b, c, the projection argument y and its box
    // mask (bit i: lb_i < y_i < ub_i); with `advance`, also the new iterate.
    // One stream of rows [A_i B_i e_i lb_i ub_i] (i < NX), [lb_i ub_i] (i >= NX).
    auto step23 = [&](const float (&xp)[NB], bool advance, uint32_t& mask) {
        MATS()
        mask = 0u;
        // rows i < NX use [A_i B_i]; the input rows i >= NX have none
        auto tail = [&](int i, float bi, float ci) {
            const float lo = mv.lb(i), hi = mv.ub(i);
            const float y = (2.f * (xs[i] + th[i]) + bi + ci) * third;
            if (y > lo && y < hi) mask |= 1u << i;
            if (advance) {
                const float gam = bi - ci;
                const float zn = y < lo ? lo : (y > hi ? hi : y);
                const float vn = (zn + gam) * 0.5f;
                const float thn = th[i] + xs[i] - zn;
                if (act) {
                    v[i] = vn;
                    th[i] = thn;
                    be[i] = bi - vn;
                    la[i] = zn - vn - ci;
                    z[i] = zn;
                }
            }
        };
        mv.rowsAB([&](int i, const float (&x)[NBP]) {
            float bi = be[i];
#pragma unroll
            for (int j = 0; j < NU; ++j) bi += x[NX + j] * du[j];
            float ci = mv.e(i) - la[i];
#pragma unroll
            for (int j = 0; j < NX; ++j) ci += x[j] * xp[j];
#pragma unroll
            for (int j = 0; j < NU; ++j) ci += x[NX + j] * xp[NX + j];
            tail(i, bi, ci);
        });
#pragma unroll
        for (int i = NX; i < NB; ++i) tail(i, du[i - NX] + be[i], xp[i] - la[i]);
    };
    auto get_xp = [&](float (&xp)[NB]) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            const float xv = xx[i * kBBD + tid - 1];
            xp[i] = (k == 0) ? lw[48 + i] : (act ? xv : 0.f);
        }
    };

    // Segment tape: per stage and step, what the transposes need from the
    // forward step -- d = v - beta (the input of du = J d), w = z - v - ebar
    // + lambda (top rows: the input of g = Abar' w), h (the input of xbar =
    // H h) and the box mask of the projection -- rather than the whole
    // iterate: 2 NB + NX + 1 words instead of 5 NB, and the reverse step
    // recomputes only du = J d and xbar = H h instead of steps 1-3.
    constexpr int R = tape_rec_floats(NB, NX);
    float w[NX];
    uint32_t mask = 0u;
    auto store_rec = [&](float* base) {
        if (!act) return;
        const gptr<float> p = (gptr<float>)base;
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            p[(int64_t)i * N + k] = d[i];
            p[(int64_t)(NB + i) * N + k] = h[i];
        }
#pragma unroll
        for (int i = 0; i < NX; ++i) p[(int64_t)(2 * NB + i) * N + k] = w[i];
        p[(int64_t)(2 * NB + NX) * N + k] = __uint_as_float(mask);
    };

    // With a full tape the forward recorded all K steps: one segment, no
    // replay.  Otherwise each segment is re-run from its checkpoint first.
    const int K = a.K;
    constexpr bool full = FULL;
    const int CK = full ? K : a.ckpt_every;
    const int nck = (K + CK - 1) / CK;
    float* tape = have ? a.tape + I.tape_off : a.tape;
#pragma unroll 1
    for (int seg = nck - 1; seg >= 0; --seg) {
        const int i0 = seg * CK;
        const int i1 = min(i0 + CK, K);
        if constexpr (!full) load_state(have ? a.ckpt + I.ck_off + (int64_t)seg * 5 * NB * N : a.ckpt);
        // forward over the segment from its checkpoint, recording each step
#pragma unroll 1
        for (int i = i0; i < (full ? i0 : i1); ++i) {
            step1();
            {
                MATS()
#pragma unroll
                for (int r = 0; r < NX; ++r) w[r] = z[r] - v[r] - mv.e(r) + la[r];
            }
            float xp[NB];
            get_xp(xp);
            step23(xp, i + 1 < i1, mask);
            store_rec(tape + (int64_t)(i - i0) * R * N);
        }
        // reverse sweep.  Each step's record (d, h, the top rows of w, the
        // mask) is loaded one step ahead, during the step before it: at one
        // wave per SIMD nothing else hides the HBM latency (measured: the
        // full-tape backward of the differentiable batch 2.88 -> 2.61 ms).
        float pd[NB], ph[NB], pw[NX], cw[NX];
        uint32_t pmask = 0u;
        auto pre_rec = [&](const float* base) {
            const gptr<float> p = (gptr<float>)base;
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                pd[q] = act ? p[(int64_t)q * N + k] : 0.f;
                ph[q] = act ? p[(int64_t)(NB + q) * N + k] : 0.f;
            }
#pragma unroll
            for (int q = 0; q < NX; ++q) pw[q] = act ? p[(int64_t)(2 * NB + q) * N + k] : 0.f;
            pmask = act ? __float_as_uint(p[(int64_t)(2 * NB + NX) * N + k]) : 0u;
        };
        pre_rec(tape + (int64_t)(i1 - 1 - i0) * R * N);
#pragma unroll 1
        for (int i = i1 - 1; i >= i0; --i) {
#pragma unroll
            for (int q = 0; q < NB; ++q) {
                d[q] = pd[q];
                h[q] = ph[q];
            }
            mask = pmask;
#pragma unroll
            for (int q = 0; q < NX; ++q) cw[q] = pw[q];
            if (i > i0) pre_rec(tape + (int64_t)(i - 1 - i0) * R * N);
            if (i == K - 1) {
                // seed: u0 = u_prev + J (v_0 - beta_0) of the last step 1
                MATS()
                float ub[16], dd[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) ub[q] = dd[q] = 0.f;
                if (act && k == 0) {
#pragma unroll
                    for (int r = 0; r < NU; ++r) ub[r] = r < nu_real ? a.dLdu0[I.u_off + r] : 0.f;
#pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        dd[j] = d[j];
                        float t = 0.f;
#pragma unroll
                        for (int r = 0; r < NU; ++r) t += mv.j(r, j) * ub[r];
                        sv[j] += t;
                        sbe[j] -= t;
                    }
                }
                stage_accum(CJ, ub, dd, stg, lane);
                continue;
            }
            MATS()
            // staging areas of the parameter products: 0 cb | w, 1 xbar_k | gr,
            // 2 [dub; bb] (bb alone when J_bar has its own tile), 3 [d; du] (du),
            // 4 xsb (zero at stage N - 1), 5 h; stages without a stage hold
            // zero adjoints (cb, bb, dub, xsb) and zero tape words, so their
            // rows add nothing
            float* ar0 = stg;
            float* ar1 = stg + kStgArea;
            float* ar2 = stg + 2 * kStgArea;
            float* ar3 = stg + 3 * kStgArea;
            float* ar4 = stg + 4 * kStgArea;
            float* ar5 = stg + 5 * kStgArea;
            auto put = [&](float* area, auto&& f) {
                float t[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) t[q] = f(q);
                stage_write(area, t, lane);
            };
            put(ar5, [&](int q) { return q < NB ? h[q] : 0.f; });
            // ---- transpose of steps 2-3 (sv.. hold the adjoint of the new iterate)
            float nth[NB], xsb[NB], bb[NB], cb[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const bool inside = (mask >> i) & 1u;
                float znb = sz[i] - sth[i];
                nth[i] = sth[i];
                xsb[i] = sth[i];
                float bbi = sbe[i];
                float vnb = sv[i] - sbe[i];
                znb += sla[i];
                vnb -= sla[i];
                float cbi = -sla[i];
                znb += 0.5f * vnb;
                const float gamb = 0.5f * vnb;
                const float yb = inside ? znb : 0.f;
                xsb[i] += (2.f / 3.f) * yb;
                nth[i] += (2.f / 3.f) * yb;
                bbi += yb * third;
                cbi += yb * third;
                bbi += gamb;
                cbi -= gamb;
                bb[i] = act ? bbi : 0.f;
                cb[i] = act ? cbi : 0.f;
            }
            put(ar0, [&](int q) { return q < NX ? cb[q] : 0.f; });
            if constexpr (!kMergeBJ) put(ar2, [&](int q) { return q < NX ? bb[q] : 0.f; });
            // adjoint of the step's input iterate, first contributions
            float nv[NB], nz[NB], nbe[NB], nla[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                nv[i] = 0.f;
                nz[i] = 0.f;
                nbe[i] = bb[i];
                nla[i] = -cb[i];
            }
            // xbar_k adjoint = Abar' cb (to stage k-1, or to xbar_0 at k = 0)
            // and du adjoint = Bbar' bb, from the top rows [A_r B_r]
            float dub[NU];
            {
                float xpb[NB];
#pragma unroll
                for (int cc = 0; cc < NB; ++cc) xpb[cc] = (cc < NX) ? 0.f : cb[cc];
#pragma unroll
                for (int cc = 0; cc < NU; ++cc) dub[cc] = bb[NX + cc];
                mv.rowsAB([&](int r, const float (&x)[NBP]) {
#pragma unroll
                    for (int cc = 0; cc < NB; ++cc) xpb[cc] += x[cc] * cb[r];
#pragma unroll
                    for (int cc = 0; cc < NU; ++cc) dub[cc] += x[NX + cc] * bb[r];
                });
#pragma unroll
                for (int i = 0; i < NB; ++i) xg[i * kBBD + tid] = xpb[i];
                if (act && k == 0) {  // the x0 adjoint (lane of stage 0 only)
#pragma unroll
                    for (int i = 0; i < NB; ++i) lw[32 + i] += xpb[i];
                }
            }
            if constexpr (kMergeBJ)
                put(ar2, [&](int q) { return q < NU ? dub[q] : ((q < NB) ? bb[q - NU] : 0.f); });
            // the step's du = J d (recomputed from the recorded d) and the
            // transpose J' dub, from the J rows
            {
                float jt[NB];
#pragma unroll
                for (int j = 0; j < NB; ++j) jt[j] = 0.f;
                mv.rowsJ([&](int r, const float (&x)[NBP]) {
                    float s = 0.f;
#pragma unroll
                    for (int j = 0; j < NB; ++j) {
                        s += x[j] * d[j];
                        jt[j] += x[j] * dub[r];
                    }
                    du[r] = s;
                });
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    nv[j] += jt[j];
                    nbe[j] -= jt[j];
                }
            }
            if constexpr (kMergeBJ)
                put(ar3, [&](int q) { return q < NB ? d[q] : ((q < NB + NU) ? du[q - NB] : 0.f); });
            else
                put(ar3, [&](int q) { return q < NU ? du[q] : 0.f; });
            __syncthreads();
            // ---- transpose of step 1
            const bool hasnext = act && (k + 1 < N);
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const float t = xg[i * kBBD + tid + 1];
                xsb[i] += hasnext ? t : 0.f;
            }
            put(ar4, [&](int q) { return (q < NB && !is_last) ? xsb[q] : 0.f; });
            // the step's xbar_{k+1} = H h (for stage k + 1) and the h adjoint
            // H' xsb (H symmetric), from the H rows (H_{N-1} at the last stage)
            float hb[NB];
            mv.rowsH(is_last, [&](int r, const float (&x)[NBP]) {
                float s = 0.f, t = 0.f;
#pragma unroll
                for (int j = 0; j < NB; ++j) {
                    s += x[j] * h[j];
                    t += x[j] * xsb[j];
                }
                xs[r] = s;
                hb[r] = t;
            });
            if (last_wave) {  // H_{N-1} += xsb h' of stage N - 1, in the MFMA tile layout
                if (is_last) {
#pragma unroll
                    for (int q = 0; q < 16; ++q) {
                        lw[q] = (q < NB) ? xsb[q] : 0.f;
                        lw[16 + q] = (q < NB) ? h[q] : 0.f;
                    }
                }
                __builtin_amdgcn_wave_barrier();
                const float hv = lw[16 + (lane & 15)];
#pragma unroll
                for (int q = 0; q < 4; ++q) CHb[q] += lw[4 * (lane >> 4) + q] * hv;
                __builtin_amdgcn_wave_barrier();
            }
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const float rh = act ? rho * hb[i] : 0.f;
                nz[i] += rh;
                nth[i] -= rh;
                xx[i * kBBD + tid] = rh;     // adjoint of g_{k+1}, read by stage k+1
                xq[i * kBBD + tid] = xs[i];  // xbar_{k+1}, read by stage k+1
            }
            __syncthreads();
            // g_k = Abar' w_k with w_k = z - v - ebar + lambda: adjoint from
            // stage k-1; xbar_k of the step from stage k-1 (xbar_0 at k = 0)
            put(ar1, [&](int q) {
                if (q >= NB) return 0.f;
                const float xv = xq[q * kBBD + tid - 1];
                return (k == 0) ? lw[48 + q] : (act ? xv : 0.f);
            });
            // round 1: Abar += cb xbar_k' (top rows); J_bar += dub d' and
            // Bbar += bb du' (top rows) in one tile, or Bbar alone
            stage_mfma2(CA, ar0, ar1, kMergeBJ ? CJ : CB, ar2, ar3, lane);
            float gr[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                const float t = xx[i * kBBD + tid - 1];
                gr[i] = (act && k >= 1) ? t : 0.f;
            }
            put(ar0, [&](int q) { return q < NX ? cw[q < NX ? q : 0] : 0.f; });  // w
            put(ar1, [&](int q) { return q < NB ? gr[q] : 0.f; });
            // round 2: H_a += xsb h' (k < N-1); Abar += w_k g_bar' (top rows)
            stage_mfma2(CHa, ar4, ar5, CA, ar0, ar1, lane);
            if constexpr (!kMergeBJ) {  // J_bar += dub d'
                put(ar2, [&](int q) { return q < NU ? dub[q] : 0.f; });
                put(ar3, [&](int q) { return q < NB ? d[q < NB ? q : 0] : 0.f; });  // d
                stage_mfma(CJ, ar2, ar3, lane);
            }
            float wb[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) wb[i] = (i < NX) ? 0.f : gr[i];
            mv.rowsAB([&](int r, const float (&x)[NBP]) {
                float s = 0.f;
#pragma unroll
                for (int cc = 0; cc < NB; ++cc) s += x[cc] * gr[cc];
                wb[r] = s;
            });
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                nz[i] += wb[i];
                nv[i] -= wb[i];
                nla[i] += wb[i];
            }
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                sv[i] = act ? nv[i] : 0.f;
                sz[i] = act ? nz[i] : 0.f;
                sth[i] = act ? nth[i] : 0.f;
                sbe[i] = act ? nbe[i] : 0.f;
                sla[i] = act ? nla[i] : 0.f;
            }
        }
    }

    // ---- reduce the per-wave tiles over the instance's waves, write raw adjoints
    __syncthreads();
    float* red = stg;  // reuse this wave's staging tile
    const floatx4 tiles[5] = {CHa, CHb, CJ, CA, CB};
#pragma unroll
    for (int b5 = 0; b5 < 5; ++b5)
#pragma unroll
        for (int q = 0; q < 4; ++q) red[b5 * 256 + (4 * (lane >> 4) + q) * 16 + (lane & 15)] = tiles[b5][q];
    __syncthreads();
    if (have && wave == gw0) {
        const int nw = (N + 63) >> 6;
        float* out = a.grads + I.gr_off;
        for (int e = lane; e < 5 * 256; e += 64) {
            // with the merged tile (slot 2): J_bar is its rows < NU, columns
            // < NB; the top rows of B_bar are rows NU.., columns NB..
            int src = e;
            bool zero = false;
            if constexpr (kMergeBJ) {
                const int tile = e >> 8, row = (e >> 4) & 15, col = e & 15;
                if (tile == 2) zero = !(row < NU && col < NB);
                if (tile == 4) {
                    src = 2 * 256 + (NU + row) * 16 + NB + col;
                    zero = !(row < NX && col < NU);
                }
            }
            float s = 0.f;
            if (!zero)
                for (int w = gw0; w < gw0 + nw; ++w) s += stg0[w * kStgFloats + src];
            out[e] = s;
        }
        if (k == 0)
            for (int i = 0; i < 16; ++i) out[5 * 256 + i] = i < NB ? lw[32 + i] : 0.f;
    }
    __syncthreads();
    (void)leader_mask;
#undef MATS
}

template <int NX, int NU, bool FULL>
__global__ void __launch_bounds__(kBwdThreads) lane_bwd_kernel(BwdArgs a) {
    __shared__ int s_bin;
    const int wave = threadIdx.x >> 6;
    for (int j = 0;; ++j) {
        int b;
        if (a.bin_counter) {
            if (threadIdx.x == 0) s_bin = atomicAdd(a.bin_counter, 1);
            __syncthreads();
            b = s_bin;
            __syncthreads();
        } else {
            b = blockIdx.x + j * gridDim.x;
        }
        if (b >= a.nbins) break;
        const Bin& bin = a.bins[b];
        int my = -1;
        unsigned leader_mask = 0;
        for (int e = 0; e < bin.n; ++e) {
            leader_mask |= 1u << bin.e[e].wave0;
            if (wave >= bin.e[e].wave0 && wave < bin.e[e].wave0 + bin.e[e].nwaves) my = e;
        }
        my = __builtin_amdgcn_readfirstlane(my);
        // one inlined copy: a wave without an instance shadows the barriers
        const bool have = my >= 0;
        bwd_run<NX, NU, FULL>(a, have ? bin.e[my].inst : 0, have, have ? bin.e[my].wave0 : wave, leader_mask);
        __syncthreads();
    }
}

// ------------------------------------------------------------ FP64 chain

constexpr int kCh = 17;  // LDS pitch of the 16 x 16 work matrices

// In-place Gauss-Jordan inverses of the two stage matrices (order nb) and of G (order nu), all three at once
// by the threads of the workgroup.  The matrices are symmetric positive definite, so no pivoting is needed.
// Each pivot step keeps the old pivot row and column in pr / pc ([3][16]) and then rewrites every element:
// pivot p = 1 / a_kk, row k scaled by p, column k scaled by -p, the rest a_ij - a_ik a_kj p.
__device__ void ch_inverse3(double* M0, double* M1, double* M2, int nb, int nu, double* pr, double* pc) {
    const int t = threadIdx.x;
    for (int k = 0; k < nb; ++k) {
        const int nm = k < nu ? 3 : 2;
        for (int e = t; e < nm * nb; e += blockDim.x) {
            const int m = e / nb, x = e % nb;
            if (m == 2 && x >= nu) continue;
            const double* M = m == 0 ? M0 : (m == 1 ? M1 : M2);
            pr[m * 16 + x] = M[k * kCh + x];
            pc[m * 16 + x] = M[x * kCh + k];
        }
        __syncthreads();
        const int tot = 2 * nb * nb + (nm == 3 ? nu * nu : 0);
        for (int e = t; e < tot; e += blockDim.x) {
            const int m = e < 2 * nb * nb ? e / (nb * nb) : 2;
            const int n = m == 2 ? nu : nb;
            const int r = m == 2 ? e - 2 * nb * nb : e - m * nb * nb;
            const int i = r / n, j = r % n;
            double* M = m == 0 ? M0 : (m == 1 ? M1 : M2);
            const double p = 1.0 / pc[m * 16 + k];
            double v;
            if (i == k && j == k)
                v = p;
            else if (i == k)
                v = pr[m * 16 + j] * p;
            else if (j == k)
                v = -pc[m * 16 + i] * p;
            else
                v = M[i * kCh + j] - pc[m * 16 + i] * pr[m * 16 + j] * p;
            M[i * kCh + j] = v;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(64) chain_kernel(const InstDev* __restrict__ inst, int count,
                                                   const double* __restrict__ mats64,
                                                   const float* __restrict__ grads, double rho, float* dx0,
                                                   float* dQd, float* dRd, float* dA, float* dB) {
    const int ii = blockIdx.x;
    if (ii >= count) return;
    const InstDev I = inst[ii];
    const int NX = I.nxp, NU = I.nup, NB = I.nbp, N = I.N;
    const int nx = I.nx, nu = I.nu;
    const MatOffsets o = mat_offsets(NX, NU, N, 0);
    const double* A = mats64 + I.mat64_off + o.A64;
    const double* B = mats64 + I.mat64_off + o.B64;
    const double* Q = mats64 + I.mat64_off + o.Q64;
    const double* R = mats64 + I.mat64_off + o.R64;
    const float* gr = grads + I.gr_off;
    __shared__ double Ab[16 * kCh], Ha[16 * kCh], Hb[16 * kCh], Gi[16 * kCh], Jm[16 * kCh], T1[16 * kCh],
        Mba[16 * kCh], Mbb[16 * kCh], Gb[16 * kCh], pr[3 * 16], pc[3 * 16];
    // the stage matrices and G are built in Ha, Hb, Gi and inverted in place
    double* Ma = Ha;
    double* Mb = Hb;
    double* G = Gi;
    const int t = threadIdx.x;
    // Abar rows (all NB rows) and the two M matrices
    for (int e = t; e < NB * NB; e += blockDim.x) {
        const int i = e / NB, j = e % NB;
        Ab[i * kCh + j] = (i < NX) ? (j < NX ? A[i * NX + j] : B[i * NU + (j - NX)]) : (i == j ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int e = t; e < NB * NB; e += blockDim.x) {
        const int i = e / NB, j = e % NB;
        double q = (i == j) ? rho : 0.0;
        if (i < NX && j < NX) q += Q[i * NX + j];
        if (i >= NX && j >= NX) q += R[(i - NX) * NU + (j - NX)];
        double s = 0.0;
        for (int r = 0; r < NB; ++r) s += Ab[r * kCh + i] * Ab[r * kCh + j];
        Ma[i * kCh + j] = q + rho * s;
        Mb[i * kCh + j] = q;
    }
    const double* Wd = mats64 + I.mat64_off + o.W64;
    for (int e = t; e < NU * NU; e += blockDim.x) {
        const int i = e / NU, j = e % NU;
        double s = ((i == j) ? 1.0 : 0.0) + Wd[i * NU + j] / rho;
        for (int r = 0; r < NX; ++r) s += B[r * NU + i] * B[r * NU + j];
        G[i * kCh + j] = s;
    }
    __syncthreads();
    ch_inverse3(Ma, Mb, G, NB, NU, pr, pc);
    // J = G^-1 [B' I]
    for (int e = t; e < NU * NB; e += blockDim.x) {
        const int i = e / NB, j = e % NB;
        double s = 0.0;
        for (int r = 0; r < NU; ++r) s += Gi[i * kCh + r] * (j < NX ? B[j * NU + r] : (j - NX == r ? 1.0 : 0.0));
        Jm[i * kCh + j] = s;
    }
    // Mbar = -H Hbar H for both H
    for (int pass = 0; pass < 2; ++pass) {
        const double* H = pass == 0 ? Ha : Hb;
        const float* Hbar = gr + (pass == 0 ? 0 : 256);
        double* Mbar = pass == 0 ? Mba : Mbb;
        __syncthreads();
        for (int e = t; e < NB * NB; e += blockDim.x) {
            const int i = e / NB, j = e % NB;
            double s = 0.0;
            for (int r = 0; r < NB; ++r) s += H[i * kCh + r] * (double)Hbar[r * 16 + j];
            T1[i * kCh + j] = s;
        }
        __syncthreads();
        for (int e = t; e < NB * NB; e += blockDim.x) {
            const int i = e / NB, j = e % NB;
            double s = 0.0;
            for (int r = 0; r < NB; ++r) s += T1[i * kCh + r] * H[r * kCh + j];
            Mbar[i * kCh + j] = (pass == 0 && N == 1) ? 0.0 : -s;
        }
    }
    __syncthreads();
    // Gbar = -G^-1 Jbar J'
    const float* Jbar = gr + 2 * 256;
    for (int e = t; e < NU * NB; e += blockDim.x) {
        const int i = e / NB, j = e % NB;
        double s = 0.0;
        for (int r = 0; r < NU; ++r) s += Gi[i * kCh + r] * (double)Jbar[r * 16 + j];
        T1[i * kCh + j] = s;  // G^-1 Jbar  (NU x NB)
    }
    __syncthreads();
    for (int e = t; e < NU * NU; e += blockDim.x) {
        const int i = e / NU, j = e % NU;
        double s = 0.0;
        for (int r = 0; r < NB; ++r) s += T1[i * kCh + r] * Jm[j * kCh + r];
        Gb[i * kCh + j] = -s;
    }
    __syncthreads();
    const float* Atop = gr + 3 * 256;
    const float* Btop = gr + 4 * 256;
    for (int e = t; e < nx * NB; e += blockDim.x) {
        const int i = e / NB, j = e % NB;
        // Abar_bar top rows: raw + rho Abar (Mbar_a + Mbar_a')
        double s = (double)Atop[i * 16 + j];
        for (int r = 0; r < NB; ++r) s += rho * Ab[i * kCh + r] * (Mba[r * kCh + j] + Mba[j * kCh + r]);
        if (j < NX) {
            if (dA && j < nx) dA[I.ga_off + i * nx + j] = (float)s;
        } else if (j - NX < nu) {
            const int c = j - NX;
            // Bbar_bar top rows: raw + (Jbar' G^-1)[i][c] + (Bbar (Gbar + Gbar'))[i][c]
            double bb = (double)Btop[i * 16 + c] + T1[c * kCh + i];
            for (int r = 0; r < NU; ++r) bb += B[i * NU + r] * (Gb[r * kCh + c] + Gb[c * kCh + r]);
            if (dB) dB[I.gb_off + i * nu + c] = (float)(s + bb);
        }
    }
    for (int i = t; i < nx; i += blockDim.x) {
        if (dQd) dQd[I.x_off + i] = (float)(Mba[i * kCh + i] + Mbb[i * kCh + i]);
        if (dx0) dx0[I.x_off + i] = gr[5 * 256 + i];
    }
    for (int i = t; i < nu; i += blockDim.x)
        if (dRd) dRd[I.u_off + i] = (float)(Mba[(NX + i) * kCh + NX + i] + Mbb[(NX + i) * kCh + NX + i]);
}

// ---------------------------------------------------------------- host side

inline size_t bwd_lds_bytes() {
    return (size_t)3 * 16 * kBBD * sizeof(float) + (size_t)kBwdWaves * (kStgFloats + kMatFloats) * sizeof(float);
}

template <int NX, int NU, bool FULL>
hipError_t launch_bwd_cls(const BwdArgs& a, int grid, hipStream_t s) {
    static bool attr = false;
    if (!attr) {
        hipError_t e = hipFuncSetAttribute((const void*)lane_bwd_kernel<NX, NU, FULL>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)bwd_lds_bytes());
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL((lane_bwd_kernel<NX, NU, FULL>), dim3(grid), dim3(kBwdThreads), bwd_lds_bytes(), s, a);
    return hipGetLastError();
}

template <int NX, int NU>
hipError_t maybe_launch_bwd(const BwdArgs& a, int grid, hipStream_t s) {
    if constexpr (NX + NU <= 16)
        return a.full_tape ? launch_bwd_cls<NX, NU, true>(a, grid, s) : launch_bwd_cls<NX, NU, false>(a, grid, s);
    else
        return hipErrorInvalidValue;
}

// Backward launch for one lane class (time-invariant, FP32, nx + nu <= 16).
hipError_t launch_backward_class(int cls, const BwdArgs& a, int grid, hipStream_t s, bool* handled) {
    *handled = true;
    switch (cls) {
#define PIMPC_BWD(id, nx, nu) \
    case id:                  \
        return maybe_launch_bwd<nx, nu>(a, grid, s);
        PIMPC_LANE_CLASSES(PIMPC_BWD)
#undef PIMPC_BWD
        default:
            break;
    }
    *handled = false;
    return hipErrorInvalidValue;
}

bool backward_class_supported(int cls) {
    switch (cls) {
#define PIMPC_BWD(id, nx, nu) \
    case id:                  \
        return (nx) + (nu) <= 16;
        PIMPC_LANE_CLASSES(PIMPC_BWD)
#undef PIMPC_BWD
        default:
            return false;
    }
}

hipError_t launch_chain(const InstDev* inst, int count, const double* mats64, const float* grads, double rho,
                        float* dx0, float* dQd, float* dRd, float* dA, float* dB, hipStream_t s) {
    hipLaunchKernelGGL(chain_kernel, dim3(count), dim3(64), 0, s, inst, count, mats64, grads, rho, dx0, dQd, dRd,
                       dA, dB);
    return hipGetLastError();
}

}  // namespace pimpc
