// admm_row.hip -- row-per-lane ADMM kernel for long single horizons.
//
// Same iteration as the lane kernel (eqn. (8), Algorithm 1 steps 1-5 of
// arXiv 2601.14414, velocity form of Theorem 2) with a different mapping,
// for instances whose horizon is long and whose stage is wide (e.g. nx = 24,
// nu = 11, N = 1024), where one lane per stage would leave most of the chip
// idle:
//   * a wave owns a block of S consecutive stages; lane r owns row r of
//     every stage vector (v, z, theta, beta, lambda, du, xbar, g);
//   * lane r keeps row r of H, J, [A B] and column r of [A B] in VGPRs for
//     the whole solve (time-invariant data), so every mat-vec is NB FMAs per
//     lane with the input vector broadcast from a per-wave LDS buffer;
//   * a block needs, per iteration, only its neighbours' previous iterate:
//     the right block's first stage (z, v, lambda) gives g of the stage after
//     the block, and the left block's last stage (z, theta) lets the block
//     recompute xbar_k of the stage before it.  So each iteration has ONE
//     halo exchange, sent at the end of the iteration and awaited at the start
//     of the next one;
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

namespace pimpc {

namespace {

constexpr int kSpinLimit = 1 << 22;  // polls before a wait gives up (seconds at worst)

// Scratch layout of one row-family instance (16-byte aligned pieces):
//   abort flag (int), reduction tags, decision word, per-wave partials,
//   global mailboxes: per wave, right_out [2 buf][2 vec][NBP] and
//   left_out [2 buf][4 vec][NBP] 64-bit words.
struct RowScratch {
    int32_t* abort;
    uint64_t* red_tag;   // [nwaves]
    double* red_val;     // [nwaves][3]
    uint64_t* decision;  // [1]
    uint64_t* mbox;      // [nwaves][12][NBP]
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) / 16 * 16; }

__host__ __device__ inline size_t row_scratch_size(int nwaves, int nbp) {
    return align16(16) + align16(8ull * nwaves) + align16(24ull * nwaves) + align16(16) +
           align16(8ull * nwaves * 12 * nbp);
}

__device__ inline RowScratch row_scratch(void* base, int nwaves, int nbp) {
    char* p = (char*)base;
    RowScratch s;
    s.abort = (int32_t*)p;
    p += align16(16);
    s.red_tag = (uint64_t*)p;
    p += align16(8ull * nwaves);
    s.red_val = (double*)p;
    p += align16(24ull * nwaves);
    s.decision = (uint64_t*)p;
    p += align16(16);
    s.mbox = (uint64_t*)p;
    return s;
}

__device__ inline uint64_t pack(float v, uint32_t tag) {
    return ((uint64_t)tag << 32) | (uint64_t)__float_as_uint(v);
}
__device__ inline float unpack_val(uint64_t w) { return __uint_as_float((uint32_t)w); }
__device__ inline uint32_t unpack_tag(uint64_t w) { return (uint32_t)(w >> 32); }

__device__ inline void gstore(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t gload(uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void lstore(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ inline uint64_t lload(uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Wait until *p carries `tag`; returns the value, or 0 after abort/timeout.
// Every wait is bounded and also ends when another wave raised the abort flag.
template <bool LDS>
__device__ inline float wait_word(uint64_t* p, uint32_t tag, int32_t* abort_flag, bool* failed) {
    int spins = 0;
    for (;;) {
        const uint64_t w = LDS ? lload(p) : gload(p);
        if (unpack_tag(w) == tag) return unpack_val(w);
        if ((++spins & 63) == 0) {
            if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                *failed = true;
                return 0.f;
            }
            if (spins > kSpinLimit) {
                __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                *failed = true;
                return 0.f;
            }
        }
        __builtin_amdgcn_s_sleep(1);
    }
}
__device__ inline float wait_lds(uint64_t* p, uint32_t tag, int32_t* ab, bool* f) { return wait_word<true>(p, tag, ab, f); }
__device__ inline float wait_glb(uint64_t* p, uint32_t tag, int32_t* ab, bool* f) { return wait_word<false>(p, tag, ab, f); }

__device__ inline bool wave_any(bool p) { return __ballot(p) != 0; }

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

}  // namespace

// Kernel geometry: kRowWaves waves per workgroup.
constexpr int kRowWaves = 4;

template <int NX, int NU, int S>
__global__ void __launch_bounds__(64 * kRowWaves) row_kernel(const RowArgs* __restrict__ ap, int nwaves,
                                                             int nwg) {
    constexpr int NB = NX + NU;
    constexpr int LD = NB + 4;  // LDS row pitch of a broadcast vector (16-byte multiple)
    static_assert(NB <= 64, "row kernel needs nx + nu <= 64");
    static_assert(LD % 4 == 0, "broadcast rows must stay 16-byte aligned");
    const RowArgs& a = *ap;
    const InstDev I = a.inst[a.inst_idx];
    const int N = I.N;
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    // XCD-aware logical workgroup index: hardware workgroup h runs on XCD h % 8.
    int lwg = blockIdx.x;
    if (nwg % 8 == 0) lwg = (blockIdx.x % 8) * (nwg / 8) + blockIdx.x / 8;
    const int gw = lwg * kRowWaves + wv;  // logical wave (block) index
    const int k0 = gw * S;
    const int ns = max(0, min(S, N - k0));  // stages in this block
    const bool rowl = lane < NB;            // lane carries a (padded) row
    const int r = lane;
    const float rho = (float)a.rho;
    const float third = 1.0f / 3.0f;

    RowScratch sc = row_scratch((char*)a.scratch + (size_t)I.pad0 * 16, nwaves, NB);

    // per-wave broadcast rows: [S + 2][LD] (one row per vector of a round)
    __shared__ __align__(16) float bcast[kRowWaves][S + 2][LD];
    __shared__ uint64_t lmbox[kRowWaves][2][6][NB];  // intra-workgroup mailboxes
    for (int i = threadIdx.x; i < kRowWaves * 2 * 6 * NB; i += blockDim.x) (&lmbox[0][0][0][0])[i] = 0;
    __syncthreads();
    if (gw >= nwaves) return;  // no workgroup barrier below this point

    // ---- per-lane matrix rows (time-invariant data), padded entries are 0
    const MatOffsets o = mat_offsets(NX, NU, N, 0);
    const float* M = (const float*)a.mats + I.mat_off;
    float Hrow[NB], Jrow[NB], Arow[NB], Acol[NX], Brow[NU];
#pragma unroll
    for (int j = 0; j < NB; ++j) {
        Hrow[j] = rowl ? M[o.H + r * NB + j] : 0.f;
        Jrow[j] = (r < NU) ? M[o.J + r * NB + j] : 0.f;
        Arow[j] = (r < NX) ? (j < NX ? M[o.A + r * NX + j] : M[o.B + r * NU + (j - NX)]) : 0.f;
    }
#pragma unroll
    for (int i = 0; i < NX; ++i)  // column r of the top block [A B]
        Acol[i] = rowl ? (r < NX ? M[o.A + i * NX + r] : M[o.B + i * NU + (r - NX)]) : 0.f;
#pragma unroll
    for (int j = 0; j < NU; ++j) Brow[j] = (r < NX) ? M[o.B + r * NU + j] : 0.f;
    const float e_r = (r < NX) ? M[o.e + r] : 0.f;
    const float q_r = rowl ? M[o.qbar + r] : 0.f;
    const float lb_r = rowl ? M[o.lb + r] : 0.f;
    const float ub_r = rowl ? M[o.ub + r] : 0.f;
    const float hbd_r = rowl ? M[o.Hb + r * NB + r] : 0.f;
    const bool hb_diag = I.hb_diag != 0;
    const bool owns_last = ns > 0 && k0 + ns == N;  // block holds stage N-1 (uses H_{N-1})

    float xb0_r = 0.f;  // row r of xbar_0 = col(x(t), u(t-1))
    if (r < NX && r < I.nx) xb0_r = ((const float*)a.x0)[I.x_off + r];
    if (r >= NX && r - NX < I.nu && a.uprev) xb0_r = ((const float*)a.uprev)[I.u_off + r - NX];

    // ---- iterate rows of the S stages
    float v[S], z[S], th[S], be[S], la[S], du[S], xs[S], g[S];
    float* st = (float*)a.state + I.st_off;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const bool ld = a.warm && rowl && s < ns;
        const int k = k0 + s;
        v[s] = ld ? st[(size_t)(0 * NB + r) * N + k] : 0.f;
        z[s] = ld ? st[(size_t)(1 * NB + r) * N + k] : 0.f;
        th[s] = ld ? st[(size_t)(2 * NB + r) * N + k] : 0.f;
        be[s] = ld ? st[(size_t)(3 * NB + r) * N + k] : 0.f;
        la[s] = ld ? st[(size_t)(4 * NB + r) * N + k] : 0.f;
        du[s] = 0.f;
        xs[s] = 0.f;
        g[s] = 0.f;
    }

    const bool has_left = ns > 0 && k0 > 0;
    const bool has_right = ns > 0 && k0 + ns < N;
    const bool left_in_wg = wv > 0;
    const bool right_in_wg = wv < kRowWaves - 1;
    auto put = [&](bool in_wg, int buf, int vec, uint64_t word) {
        if (in_wg)
            lstore(&lmbox[wv][buf][vec][r], word);
        else
            gstore(sc.mbox + ((size_t)gw * 12 + buf * 6 + vec) * NB + r, word);
    };
    bool failed = false;
    auto recv = [&](int nl, int ng, bool in_wg, int vec, uint32_t tag) -> float {
        if (!rowl) return 0.f;
        const int buf = tag & 1;
        if (in_wg) return wait_lds(&lmbox[nl][buf][vec][r], tag, sc.abort, &failed);
        return wait_glb(sc.mbox + ((size_t)ng * 12 + buf * 6 + vec) * NB + r, tag, sc.abort, &failed);
    };
    // left_out (z, v, lambda[, dd]) of the first stage, read by wave gw-1
    auto publish_left = [&](uint32_t tag, bool with_dd, float dd0) {
        if (!has_left || !rowl) return;
        const int buf = tag & 1;
        put(left_in_wg, buf, 0, pack(z[0], tag));
        put(left_in_wg, buf, 1, pack(v[0], tag));
        put(left_in_wg, buf, 2, pack(la[0], tag));
        if (with_dd) put(left_in_wg, buf, 3, pack(dd0, tag));
    };
    // right_out (z, theta) of the last stage, read by wave gw+1
    auto publish_right = [&](uint32_t tag) {
        if (!has_right || !rowl) return;
        const int buf = tag & 1;
        float zl = z[0], tl = th[0];
#pragma unroll
        for (int s = 1; s < S; ++s)
            if (s == ns - 1) {
                zl = z[s];
                tl = th[s];
            }
        put(right_in_wg, buf, 4, pack(zl, tag));
        put(right_in_wg, buf, 5, pack(tl, tag));
    };

    float(*bc)[LD] = bcast[wv];
    // Write this lane's row of up to S + 2 vectors, then make them visible to
    // the wave (LDS operations of one wave complete in order).
#define BC_PUT(row, val)                  \
    do {                                  \
        if (rowl) bc[(row)][r] = (val);   \
    } while (0)
#define BC_SYNC() __builtin_amdgcn_wave_barrier()
#define DOT(acc, coef, row, n)                                  \
    _Pragma("unroll") for (int j_ = 0; j_ < (n); ++j_) (acc) += (coef)[j_] * bc[(row)][j_];

    publish_left(1u, false, 0.f);  // initial iterate carries tag 1
    publish_right(1u);

    int iters = 0;
    double c_last = 0.0, rp_last = 0.0, rd_last = 0.0;
    int status = 0;
    bool stop = false;

    // One update of stage s (steps 2-3) given its xbar_k row `xp`.
    float cpart = 0.f, rpart = 0.f, rdpart = 0.f;
    float ddv[S], dzv[S];
    auto update = [&](int s, bool check) {
        // round 3 inputs (xp, du) are already in bc rows 0 (xp) and 1 (du)
        float ci = 0.f, bi = 0.f;
        DOT(ci, Arow, 0, NB);
        if (r >= NX) ci = bc[0][r];
        ci += e_r - la[s];
        DOT(bi, Brow, 1, NU);
        if (r >= NX) bi = bc[1][r - NX];
        bi += be[s];
        const float gam = bi - ci;
        const float y = (2.f * (xs[s] + th[s]) + bi + ci) * third;
        const float zn = y < lb_r ? lb_r : (y > ub_r ? ub_r : y);
        const float vn = (zn + gam) * 0.5f;
        const float thn = th[s] + xs[s] - zn;
        const float ben = bi - vn;
        const float lan = zn - vn - ci;
        if (check) {
            const float dv = rowl ? vn - v[s] : 0.f, dz = rowl ? zn - z[s] : 0.f;
            const float dth = rowl ? thn - th[s] : 0.f, dbe = rowl ? ben - be[s] : 0.f;
            const float dla = rowl ? lan - la[s] : 0.f;
            const float dd = dz - dv;
            cpart += dth * dth + dbe * dbe + dla * dla + dz * dz + dv * dv + dd * dd;
            rpart = fmax(rpart, fmax(fabsf(dth), fmax(fabsf(dbe), fabsf(dla))));
#pragma unroll
            for (int t = 0; t < S; ++t)
                if (t == s) {
                    ddv[t] = dd;
                    dzv[t] = dz;
                }
            // du block of F'G dq: Bbar' dv = u-rows of Abar' dv
            BC_PUT(2, dv);
            BC_SYNC();
            float bt = (r >= NX) ? dv : 0.f;
            DOT(bt, Acol, 2, NX);
            if (r >= NX && rowl) rdpart = fmax(rdpart, fabsf(bt));
        }
        if (rowl) {
            v[s] = vn;
            z[s] = zn;
            th[s] = thn;
            be[s] = ben;
            la[s] = lan;
        }
    };

#pragma unroll 1
    for (int it = 0; it < a.K && !stop; ++it) {
        const uint32_t tin = (uint32_t)it + 1;   // tag of the iterate this step reads
        const uint32_t tout = (uint32_t)it + 2;  // tag of the iterate it produces
        const bool check = (a.eps > 0.0 && ((it + 1) % a.check_every) == 0) || (it == a.K - 1);
        cpart = rpart = rdpart = 0.f;
#pragma unroll
        for (int s = 0; s < S; ++s) ddv[s] = dzv[s] = 0.f;

        // ---- round 1 (own data only): du_s = J (v - beta), g_s = Abar' (z - v - ebar + lambda)
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (s < ns) {
                BC_PUT(0, v[s] - be[s]);
                BC_PUT(1, z[s] - v[s] - e_r + la[s]);
                BC_SYNC();
                float acc = 0.f;
                DOT(acc, Jrow, 0, NB);
                du[s] = acc;
                float gg = (r >= NX) ? bc[1][r] : 0.f;
                DOT(gg, Acol, 1, NX);
                g[s] = gg;
                BC_SYNC();
            }
        }
        // ---- round 2 for stages whose g_{k+1} is inside the block
#pragma unroll
        for (int s = 0; s + 1 < S; ++s) {
            if (s + 1 < ns) {
                float gn = g[0];
#pragma unroll
                for (int t = 1; t < S; ++t)
                    if (t == s + 1) gn = g[t];
                BC_PUT(0, q_r + rho * (z[s] - th[s] + gn));
                BC_SYNC();
                float acc = 0.f;
                DOT(acc, Hrow, 0, NB);
                xs[s] = acc;
                BC_SYNC();
            }
        }
        // ---- round 3 for interior stages 1 .. ns-2 (xbar_k of the previous stage is inside)
#pragma unroll
        for (int s = 1; s + 1 < S; ++s) {
            if (s + 1 < ns) {
                float xp = xs[0], dus = du[0];
#pragma unroll
                for (int t = 1; t < S; ++t) {
                    if (t == s - 1) xp = xs[t];
                    if (t == s) dus = du[t];
                }
                BC_PUT(0, xp);
                BC_PUT(1, dus);
                BC_SYNC();
                update(s, check);
                BC_SYNC();
            }
        }

        // ---- halos of the previous iterate (needed only by the block's end stages).
        // All five words are loaded together each poll, so a poll costs one
        // memory round trip whatever the number of words.
        float zR = 0.f, vR = 0.f, lR = 0.f, zL = 0.f, tL = 0.f;
        if ((has_right || has_left) && rowl) {
            const int buf = tin & 1;
            uint64_t* pr[3];
            uint64_t* pl[2];
#pragma unroll
            for (int q = 0; q < 3; ++q)
                pr[q] = right_in_wg ? &lmbox[wv + 1 < kRowWaves ? wv + 1 : wv][buf][q][r]
                                    : sc.mbox + ((size_t)(gw + 1) * 12 + buf * 6 + q) * NB + r;
#pragma unroll
            for (int q = 0; q < 2; ++q)
                pl[q] = left_in_wg ? &lmbox[wv > 0 ? wv - 1 : 0][buf][4 + q][r]
                                   : sc.mbox + ((size_t)(gw > 0 ? gw - 1 : 0) * 12 + buf * 6 + 4 + q) * NB + r;
            int spins = 0;
            for (;;) {
                uint64_t wr[3] = {0, 0, 0}, wl[2] = {0, 0};
                if (has_right) {
#pragma unroll
                    for (int q = 0; q < 3; ++q) wr[q] = right_in_wg ? lload(pr[q]) : gload(pr[q]);
                }
                if (has_left) {
#pragma unroll
                    for (int q = 0; q < 2; ++q) wl[q] = left_in_wg ? lload(pl[q]) : gload(pl[q]);
                }
                const bool okr = !has_right || (unpack_tag(wr[0]) == tin && unpack_tag(wr[1]) == tin &&
                                                 unpack_tag(wr[2]) == tin);
                const bool okl = !has_left || (unpack_tag(wl[0]) == tin && unpack_tag(wl[1]) == tin);
                if (okr && okl) {
                    zR = unpack_val(wr[0]);
                    vR = unpack_val(wr[1]);
                    lR = unpack_val(wr[2]);
                    zL = unpack_val(wl[0]);
                    tL = unpack_val(wl[1]);
                    break;
                }
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
            }
        }
        if (__builtin_amdgcn_readfirstlane((int)failed) || wave_any(failed)) {
            status = -5;
            break;
        }
        // g of the stage after the block (right halo)
        float gR = 0.f;
        if (has_right) {
            BC_PUT(0, zR - vR - e_r + lR);
            BC_SYNC();
            gR = (r >= NX) ? bc[0][r] : 0.f;
            DOT(gR, Acol, 0, NX);
            BC_SYNC();
        }
        // ---- round 2 for the last stage (needs gR) and xbar_{k0} from the left halo
        const int sl = ns - 1;  // last stage of the block
        float hlast = 0.f, xlast = 0.f;
        {
            float zl = z[0], tl = th[0];
#pragma unroll
            for (int t = 1; t < S; ++t)
                if (t == sl) {
                    zl = z[t];
                    tl = th[t];
                }
            hlast = q_r + rho * (zl - tl + gR);
            BC_PUT(0, hlast);
            if (has_left) BC_PUT(1, q_r + rho * (zL - tL + g[0]));
            BC_SYNC();
            if (owns_last && hb_diag) {
                xlast = hbd_r * hlast;
            } else if (owns_last) {
                const float* Hb = M + o.Hb + (rowl ? r : 0) * NB;
#pragma unroll
                for (int j = 0; j < NB; ++j) xlast += (rowl ? Hb[j] : 0.f) * bc[0][j];
            } else {
                DOT(xlast, Hrow, 0, NB);
            }
            float xsL = xb0_r;
            if (has_left) {
                xsL = 0.f;
                DOT(xsL, Hrow, 1, NB);
            }
            BC_SYNC();
#pragma unroll
            for (int t = 0; t < S; ++t)
                if (t == sl) xs[t] = xlast;
            // ---- round 3 for the first stage (xp = xbar_{k0}) ...
            BC_PUT(0, xsL);
            BC_PUT(1, du[0]);
            BC_SYNC();
            update(0, check);
            BC_SYNC();
        }
        publish_left(tout, false, 0.f);
        // ... and for the last stage (xp = xbar of the stage before it)
        if (sl > 0) {
            float xp = xs[0], dus = du[0];
#pragma unroll
            for (int t = 1; t < S; ++t) {
                if (t == sl - 1) xp = xs[t];
                if (t == sl) dus = du[t];
            }
            BC_PUT(0, xp);
            BC_PUT(1, dus);
            BC_SYNC();
            update(sl, check);
            BC_SYNC();
        }
        publish_right(tout);
        if (check) publish_left(tout, true, ddv[0]);  // dd of the first stage for the dual residual
        ++iters;

        if (check) {
            // xbar block of F'G dq: dz_{k+1} + Abar_{k+1}' (dz_{k+2} - dv_{k+1})
            float ddR = 0.f;
            if (has_right) ddR = recv(wv + 1, gw + 1, right_in_wg, 3, tout);
#pragma unroll
            for (int s = 0; s < S; ++s) {
                if (s < ns) {
                    float ddn = (s + 1 < ns) ? 0.f : ddR;
#pragma unroll
                    for (int t = 1; t < S; ++t)
                        if (t == s + 1 && t < ns) ddn = ddv[t];
                    const bool hasnext = k0 + s + 1 < N;
                    BC_PUT(0, ddn);
                    BC_SYNC();
                    float tg = (r >= NX) ? bc[0][r] : 0.f;
                    DOT(tg, Acol, 0, NX);
                    BC_SYNC();
                    if (rowl) rdpart = fmax(rdpart, fabsf(dzv[s] + (hasnext ? tg : 0.f)));
                }
            }
            const double csum = wsum((double)cpart);
            const double rpm = wmax((double)rpart);
            const double rdm = wmax((double)rdpart);
            if (lane == 0) {
                sc.red_val[gw * 3 + 0] = csum;
                sc.red_val[gw * 3 + 1] = rpm;
                sc.red_val[gw * 3 + 2] = rdm;
                __hip_atomic_store(&sc.red_tag[gw], (uint64_t)tout, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (gw == 0) {
                // deterministic reduction: lane l accumulates waves l, l+64, ...
                // in order, then a fixed shuffle tree combines the lanes
                double cs = 0.0, rp = 0.0, rd = 0.0;
                bool lfail = false;
                for (int w0 = 0; w0 < nwaves; w0 += 64) {
                    const int w = w0 + lane;
                    if (w < nwaves && !lfail) {
                        int spins = 0;
                        while (__hip_atomic_load(&sc.red_tag[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) !=
                               (uint64_t)tout) {
                            if (++spins > kSpinLimit ||
                                __hip_atomic_load(sc.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                                __hip_atomic_store(sc.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                                lfail = true;
                                break;
                            }
                            __builtin_amdgcn_s_sleep(1);
                        }
                    }
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                    if (w < nwaves && !lfail) {
                        cs += sc.red_val[w * 3 + 0];
                        rp = fmax(rp, sc.red_val[w * 3 + 1]);
                        rd = fmax(rd, sc.red_val[w * 3 + 2]);
                    }
                }
                cs = wsum(cs);
                rp = wmax(rp);
                rd = wmax(rd);
                const bool anyfail = wave_any(lfail);
                if (lane == 0) {
                    c_last = a.rho * cs;
                    rp_last = rp;
                    rd_last = a.rho * rd;
                    int dec = 0;
                    if (!(c_last < INFINITY)) {
                        status = -4;
                        dec = 1;
                    }
                    if (a.eps > 0.0 && c_last <= a.eps) dec = 1;
                    if (anyfail) {
                        status = -5;
                        dec = 1;
                    }
                    __hip_atomic_store(sc.decision, ((uint64_t)tout << 32) | (uint64_t)dec, __ATOMIC_RELEASE,
                                       __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            if (a.eps > 0.0) {  // everyone learns the decision (stop or continue)
                uint64_t d = 0;
                if (lane == 0) {
                    int spins = 0;
                    for (;;) {
                        d = __hip_atomic_load(sc.decision, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                        if ((uint32_t)(d >> 32) == tout) break;
                        if (++spins > kSpinLimit ||
                            __hip_atomic_load(sc.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                            __hip_atomic_store(sc.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            d = 1;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                    }
                }
                d = __shfl(d, 0, 64);
                if ((uint32_t)d & 1u) stop = true;
            }
        }
    }

    // ---- outputs
    if (rowl) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
            if (s < ns) {
                const int k = k0 + s;
                st[(size_t)(0 * NB + r) * N + k] = v[s];
                st[(size_t)(1 * NB + r) * N + k] = z[s];
                st[(size_t)(2 * NB + r) * N + k] = th[s];
                st[(size_t)(3 * NB + r) * N + k] = be[s];
                st[(size_t)(4 * NB + r) * N + k] = la[s];
                if (a.write_iters) {
                    float* io = (float*)a.iters_out + I.it_off;
                    if (r < NU) io[(size_t)r * N + k] = du[s];
                    io[(size_t)(NU + r) * N + k] = xs[s];
                }
            }
        }
    }
    if (k0 == 0 && ns > 0 && r < I.nu) {
        const float up = a.uprev ? ((const float*)a.uprev)[I.u_off + r] : 0.f;
        ((float*)a.u0)[I.u_off + r] = up + du[0];
    }
    if (gw == 0 && lane == 0 && a.info) {
        InfoDev rec;
        rec.iters = iters;
        rec.restarts = 0;
        rec.c = c_last;
        rec.r_prim = rp_last;
        rec.r_dual = rd_last;
        rec.status = status;
        rec.pad = 0;
        a.info[a.inst_idx] = rec;
    }
#undef BC_PUT
#undef BC_SYNC
#undef DOT
}

template <typename T>
hipError_t launch_fill(T*, int64_t, T, hipStream_t);

// ------------------------------------------------------------------ host side

namespace {

struct RowCfg {
    int nx, nu;
};
constexpr RowCfg kRowCfgs[] = {{24, 12}, {32, 16}};

template <int NX, int NU, int S>
hipError_t row_launch_t(const RowArgs* a_dev, int nwaves, int nwg, hipStream_t s, int* occ) {
    if (occ) {
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, row_kernel<NX, NU, S>, 64 * kRowWaves, 0);
    }
    hipLaunchKernelGGL((row_kernel<NX, NU, S>), dim3(nwg), dim3(64 * kRowWaves), 0, s, a_dev, nwaves, nwg);
    return hipGetLastError();
}

template <int NX, int NU>
hipError_t row_launch_s(int S, const RowArgs* a_dev, int nwaves, int nwg, hipStream_t s, int* occ) {
    switch (S) {
        case 1:
            return row_launch_t<NX, NU, 1>(a_dev, nwaves, nwg, s, occ);
        case 2:
            return row_launch_t<NX, NU, 2>(a_dev, nwaves, nwg, s, occ);
        case 4:
            return row_launch_t<NX, NU, 4>(a_dev, nwaves, nwg, s, occ);
        default:
            return hipErrorInvalidValue;
    }
}

hipError_t row_launch_any(const InstDev& I, int S, const RowArgs* a_dev, hipStream_t s, int* occ) {
    const int nwaves = (I.N + S - 1) / S;
    const int nwg = (nwaves + kRowWaves - 1) / kRowWaves;
    if (I.nxp == 24 && I.nup == 12) return row_launch_s<24, 12>(S, a_dev, nwaves, nwg, s, occ);
    if (I.nxp == 32 && I.nup == 16) return row_launch_s<32, 16>(S, a_dev, nwaves, nwg, s, occ);
    return hipErrorInvalidValue;
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

bool row_supported(int nx, int nu, int N, int tv, int fp64, int* nxp, int* nup) {
    (void)N;
    if (tv || fp64) return false;
    for (const RowCfg& c : kRowCfgs)
        if (nx <= c.nx && nu <= c.nu) {
            *nxp = c.nx;
            *nup = c.nu;
            return true;
        }
    return false;
}

size_t row_scratch_bytes(const InstDev& I, int fp64) {
    (void)fp64;
    return align16(row_scratch_size(I.N, I.nbp));  // sized for one stage per wave
}

// Choose the blocking S (stages per wave): the smallest S whose grid stays
// co-resident (every workgroup must be running for the halo waits to end).
hipError_t row_prepare(int fp64, InstDev& I) {
    (void)fp64;
    const int want = I.pad1 > 0 ? I.pad1 : 1;
    for (int S : {want, 1, 2, 4}) {
        int occ = 0;
        hipError_t e = row_launch_any(I, S, nullptr, nullptr, &occ);
        if (e != hipSuccess) return e;
        const int nwg = ((I.N + S - 1) / S + kRowWaves - 1) / kRowWaves;
        if (occ > 0 && nwg <= occ * num_cus()) {
            I.pad1 = S;
            return hipSuccess;
        }
    }
    return hipErrorInvalidConfiguration;
}

hipError_t launch_row(int fp64, const RowArgs* a_dev, const InstDev& I, void* scratch_base, hipStream_t s) {
    (void)fp64;
    const int S = I.pad1 > 0 ? I.pad1 : 1;
    char* scr = (char*)scratch_base + (size_t)I.pad0 * 16;
    hipError_t e = launch_fill<int32_t>((int32_t*)scr, (int64_t)(row_scratch_bytes(I, 0) / 4), 0, s);
    if (e != hipSuccess) return e;
    return row_launch_any(I, S, a_dev, s, nullptr);
}

}  // namespace pimpc
