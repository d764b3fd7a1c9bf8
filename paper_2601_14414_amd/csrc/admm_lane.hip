// admm_lane.hip -- lane-per-stage ADMM kernel for batches of small instances.
//
// Implements the closed-form, parallel-in-horizon iteration of eqn. (8) /
// Algorithm 1 steps 1-5 of arXiv 2601.14414 in the velocity form of
// Theorem 2.  Mapping on gfx950:
//   * one lane owns one horizon stage k and keeps its five iterate vectors
//     (v_k, z_{k+1}, theta_k, beta_k, lambda_k) in VGPRs for all iterations;
//   * an instance occupies ceil(N/64) consecutive waves of a 512-thread
//     workgroup; several instances share a workgroup ("bin");
//   * time-invariant stage data (J, H, A, B, e, bounds) is uniform across the
//     wave, read through the scalar data cache into SGPRs (scalar *loads*
//     only), so every mat-vec FMA takes a matrix operand from an SGPR;
//     time-varying stage data is loaded once into VGPRs per lane;
//   * the two one-stage halos of an iteration (g_{k+1} for step 1 and
//     xbar_k for step 2) go through LDS between two workgroup barriers;
//   * residuals (Algorithm 1 step 4 and Section IV-B) are reduced with
//     cross-lane shuffles, then across the instance's waves in LDS, in a
//     fixed order (deterministic);
//   * the kernel is persistent: each workgroup claims bins from a counter
//     until none is left (largest-cost bins first).
#include <hip/hip_runtime.h>

#include "pimpc_dev.hpp"
#include "pimpc_lane.hpp"
#include "lane_common.hpp"

namespace pimpc {

constexpr int kBD = kBinThreads;  // LDS row stride of the halo buffers

extern __shared__ __align__(16) unsigned char lane_smem[];

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

template <typename T>
__device__ inline T wave_max(T v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

template <typename T>
__device__ inline T clampv(T y, T lo, T hi) {
    return y < lo ? lo : (y > hi ? hi : y);
}

// Run (or, with have = false, only shadow the barrier sequence of) one
// instance on the waves [gw0, gw0 + gnw) of the workgroup.
template <typename T, int NX, int NU, bool TV>
__device__ __forceinline__ void lane_run(const LaneArgs* ap_in, int inst_idx, bool have, int gw0,
                                      unsigned leader_mask) {
    inst_idx = __builtin_amdgcn_readfirstlane(inst_idx);
    gw0 = __builtin_amdgcn_readfirstlane(gw0);
    have = __builtin_amdgcn_readfirstlane((int)have) != 0;
    leader_mask = __builtin_amdgcn_readfirstlane(leader_mask);
    const cptr<LaneArgs> ap = (cptr<LaneArgs>)uniform_ptr(ap_in);
    const LaneArgs a = *ap;
    const InstDev I = ((cptr<InstDev>)uniform_ptr(a.inst))[have ? inst_idx : 0];
    T* xg = (T*)lane_smem;
    T* xx = xg + (size_t)a.nbmax * kBD;
    T* xd = xx + (size_t)a.nbmax * kBD;
    double* red = (double*)(xd + (size_t)a.nbmax * kBD);
    int* gdone = (int*)(red + kBinWaves * 4);
    constexpr int NB = NX + NU;
    const int tid = threadIdx.x;
    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int k = tid - gw0 * 64;  // stage owned by this lane
    const int N = have ? I.N : 0;
    const bool act = have && k >= 0 && k < N;
    const bool leader = have && k == 0;
    const T rho = (T)a.rho;
    const T third = (T)(1.0 / 3.0);

    const MatOffsets o = mat_offsets(NX, NU, have ? N : 1, TV);
    const cptr<T> M0 = (cptr<T>)uniform_ptr(have ? (const T*)a.mats + I.mat_off : (const T*)a.mats);
    // Uniform stage data is re-read through the scalar cache each iteration;
    // an opaque copy of the base pointer keeps the compiler from hoisting
    // hundreds of loads out of the loop (which would overflow the SGPRs).
#define PIMPC_MAT_PTRS(Mp)                          \
    const cptr<T> Jm = (Mp) + o.J;                 \
    const cptr<T> Hm = (Mp) + o.H;                 \
    const cptr<T> Hbm = (Mp) + (TV ? 0 : o.Hb);    \
    const cptr<T> Am = (Mp) + o.A;                 \
    const cptr<T> Bm = (Mp) + o.B;                 \
    const cptr<T> em = (Mp) + o.e;                 \
    const cptr<T> qb = (Mp) + o.qbar;              \
    const cptr<T> lbm = (Mp) + o.lb;               \
    const cptr<T> ubm = (Mp) + o.ub;               \
    (void)Jm; (void)Hm; (void)Hbm; (void)Am; (void)Bm; (void)em; (void)qb; (void)lbm; (void)ubm;

    // per-lane stage data (time-varying only)
    T Jr[TV ? NU * NB : 1], Hr[TV ? NB * NB : 1], Ar[TV ? NX * NX : 1], Br[TV ? NX * NU : 1],
        er[TV ? NX : 1];
    if constexpr (TV) {
        PIMPC_MAT_PTRS(M0)
#pragma unroll
        for (int q = 0; q < NU * NB; ++q) Jr[q] = act ? Jm[(int64_t)q * N + k] : T(0);
#pragma unroll
        for (int q = 0; q < NB * NB; ++q) Hr[q] = act ? Hm[(int64_t)q * N + k] : T(0);
#pragma unroll
        for (int q = 0; q < NX * NX; ++q) Ar[q] = act ? Am[(int64_t)q * N + k] : T(0);
#pragma unroll
        for (int q = 0; q < NX * NU; ++q) Br[q] = act ? Bm[(int64_t)q * N + k] : T(0);
#pragma unroll
        for (int q = 0; q < NX; ++q) er[q] = act ? em[(int64_t)q * N + k] : T(0);
    }
#define JM(r, c) (TV ? Jr[(r) * NB + (c)] : Jm[(r) * NB + (c)])
#define HM(r, c) (TV ? Hr[(r) * NB + (c)] : Hm[(r) * NB + (c)])
#define AM(r, c) (TV ? Ar[(r) * NX + (c)] : Am[(r) * NX + (c)])
#define BM(r, c) (TV ? Br[(r) * NU + (c)] : Bm[(r) * NU + (c)])
#define EM(r) (TV ? er[(r)] : em[(r)])

    // xbar_0 = col(x(t), u(t-1)): uniform over the instance, read through the
    // scalar cache where lane k = 0 needs it.
    const cptr<T> x0p = (cptr<T>)uniform_ptr((const T*)a.x0 + (have ? I.x_off : 0));
    const cptr<T> upp = (cptr<T>)uniform_ptr(a.uprev ? (const T*)a.uprev + (have ? I.u_off : 0) : nullptr);
    const int nx_real = have ? I.nx : 0, nu_real = have ? I.nu : 0;
#define XB0(i) ((i) < NX ? ((i) < nx_real ? x0p[(i)] : T(0)) \
                         : ((upp && (i) - NX < nu_real) ? upp[(i) - NX] : T(0)))

    // iterate (v, z, theta, beta, lambda) of this stage
    T v[NB], z[NB], th[NB], be[NB], la[NB];
    const gptr<T> st = (gptr<T>)(have ? (T*)a.state + I.st_off : (T*)a.state);
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const bool ld = act && a.warm;
        v[i] = ld ? st[(int64_t)(0 * NB + i) * N + k] : T(0);
        z[i] = ld ? st[(int64_t)(1 * NB + i) * N + k] : T(0);
        th[i] = ld ? st[(int64_t)(2 * NB + i) * N + k] : T(0);
        be[i] = ld ? st[(int64_t)(3 * NB + i) * N + k] : T(0);
        la[i] = ld ? st[(int64_t)(4 * NB + i) * N + k] : T(0);
    }
    T du[NU], xs[NB];
#pragma unroll
    for (int i = 0; i < NU; ++i) du[i] = T(0);
#pragma unroll
    for (int i = 0; i < NB; ++i) xs[i] = T(0);

    const bool last_wave = have && ((N - 1) >> 6) == (k >> 6) && k >= 0;
    const bool is_last = act && k == N - 1;
    const bool hb_diag = have && I.hb_diag;

    int iters = 0;
    bool done = !have;
    double c_last = 0.0, rp_last = 0.0, rd_last = 0.0;
    int status = 0;

#pragma unroll 1
    for (int it = 0; it < a.K; ++it) {
        const bool check = (a.eps > 0.0 && ((it + 1) % a.check_every) == 0) || (it == a.K - 1);
        const bool run = !done;
        // taped forward: keep the iterate entering this iteration every ckpt_every steps
        if (a.ckpt_every > 0 && (it % a.ckpt_every) == 0 && act) {
            const gptr<T> ck = (gptr<T>)((T*)a.ckpt + I.ck_off + (int64_t)(it / a.ckpt_every) * 5 * NB * N);
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                ck[(int64_t)(0 * NB + i) * N + k] = v[i];
                ck[(int64_t)(1 * NB + i) * N + k] = z[i];
                ck[(int64_t)(2 * NB + i) * N + k] = th[i];
                ck[(int64_t)(3 * NB + i) * N + k] = be[i];
                ck[(int64_t)(4 * NB + i) * N + k] = la[i];
            }
        }
        // Row pointers are re-made opaque before use so that the scalar loads
        // of one matrix row cannot be hoisted ahead of earlier rows.
#define ROW(base, r, ld) ([&]() { cptr<T> p_ = (base) + (r) * (ld); asm volatile("" : "+s"(p_)); return p_; }())
        cptr<T> Mi = M0;
        asm volatile("" : "+s"(Mi));
        PIMPC_MAT_PTRS(Mi)

        // ---- step 1a: du_k = J_k (v_k - beta_k); g_k = Abar_k' (z_{k+1} - v_k - ebar_k + lambda_k)
        if (run) {
#pragma unroll
            for (int r = 0; r < NU; ++r) {
                const cptr<T> Jrow = ROW(Jm, r, NB);
                T s = T(0);
#pragma unroll
                for (int j = 0; j < NB; ++j) s += (TV ? Jr[r * NB + j] : Jrow[j]) * (v[j] - be[j]);
                du[r] = s;
            }
            T g[NB];
#pragma unroll
            for (int c = 0; c < NB; ++c) g[c] = (c < NX) ? T(0) : (z[c] - v[c] + la[c]);
#pragma unroll
            for (int r = 0; r < NX; ++r) {
                const T w = z[r] - v[r] - EM(r) + la[r];
                const cptr<T> Arow = ROW(Am, r, NX);
                const cptr<T> Brow = ROW(Bm, r, NU);
#pragma unroll
                for (int c = 0; c < NX; ++c) g[c] += (TV ? Ar[r * NX + c] : Arow[c]) * w;
#pragma unroll
                for (int c = 0; c < NU; ++c) g[NX + c] += (TV ? Br[r * NU + c] : Brow[c]) * w;
            }
#pragma unroll
            for (int c = 0; c < NB; ++c) xg[c * kBD + tid] = g[c];
        }
        __syncthreads();

        // ---- step 1b: h_k = qbar + rho (z_{k+1} - theta_k + g_{k+1}); xbar_{k+1} = H_k h_k
        if (run) {
            const bool hasnext = act && (k + 1 < N);
            T h[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                // the read stays inside the LDS allocation for every tid (xx follows xg)
                const T gv = xg[i * kBD + tid + 1];
                const T gn = hasnext ? gv : T(0);
                h[i] = qb[i] + rho * (z[i] - th[i] + gn);
            }
#pragma unroll
            for (int r = 0; r < NB; ++r) {
                const cptr<T> Hrow = ROW(Hm, r, NB);
                T s = T(0);
#pragma unroll
                for (int j = 0; j < NB; ++j) s += (TV ? Hr[r * NB + j] : Hrow[j]) * h[j];
                xs[r] = s;
            }
            if constexpr (!TV) {
                if (last_wave) {  // wave-uniform: only the wave holding stage N-1
                    if (hb_diag) {
#pragma unroll
                        for (int r = 0; r < NB; ++r) xs[r] = is_last ? Hbm[r * NB + r] * h[r] : xs[r];
                    } else {
#pragma unroll
                        for (int r = 0; r < NB; ++r) {
                            const cptr<T> Hrow = ROW(Hbm, r, NB);
                            T s = T(0);
#pragma unroll
                            for (int j = 0; j < NB; ++j) s += Hrow[j] * h[j];
                            xs[r] = is_last ? s : xs[r];
                        }
                    }
                }
            }
#pragma unroll
            for (int i = 0; i < NB; ++i) xx[i * kBD + tid] = xs[i];
        }
        __syncthreads();

        // ---- steps 2-3: Theorem 1 closed form, box projection, dual update
        T rdu[NU];
        T cpart = T(0), rpart = T(0);
        if (run) {
            T xp[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                // tid - 1 >= -1: the read stays inside the LDS allocation (xg precedes xx)
                const T xv = xx[i * kBD + tid - 1];
                xp[i] = (k == 0) ? XB0(i) : (act ? xv : T(0));
            }
#pragma unroll
            for (int c = 0; c < NU; ++c) rdu[c] = T(0);
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                // b_i = (Bbar du)_i + beta_i;  c_i = (Abar xbar_k)_i + ebar_i - lambda_i
                T bi, ci;
                if (i < NX) {
                    const cptr<T> Arow = ROW(Am, i, NX);
                    const cptr<T> Brow = ROW(Bm, i, NU);
                    bi = be[i];
#pragma unroll
                    for (int j = 0; j < NU; ++j) bi += (TV ? Br[i * NU + j] : Brow[j]) * du[j];
                    ci = EM(i) - la[i];
#pragma unroll
                    for (int j = 0; j < NX; ++j) ci += (TV ? Ar[i * NX + j] : Arow[j]) * xp[j];
#pragma unroll
                    for (int j = 0; j < NU; ++j) ci += (TV ? Br[i * NU + j] : Brow[j]) * xp[NX + j];
                } else {
                    bi = du[i - NX] + be[i];
                    ci = xp[i] - la[i];
                }
                const T gam = bi - ci;
                const T y = (T(2) * (xs[i] + th[i]) + bi + ci) * third;
                const T zn = clampv(y, lbm[i], ubm[i]);
                const T vn = (zn + gam) * T(0.5);
                const T thn = th[i] + xs[i] - zn;
                const T ben = bi - vn;
                const T lan = zn - vn - ci;
                if (check) {
                    const T dv = vn - v[i], dz = zn - z[i], dth = thn - th[i], dbe = ben - be[i],
                            dla = lan - la[i];
                    const T dd = dz - dv;
                    cpart += dth * dth + dbe * dbe + dla * dla + dz * dz + dv * dv + dd * dd;
                    rpart = fmax(rpart, fmax(fabs(dth), fmax(fabs(dbe), fabs(dla))));
                    // du block of F'G dq: Bbar_k' dv
                    if (i < NX) {
                        const cptr<T> Brow = ROW(Bm, i, NU);
#pragma unroll
                        for (int c = 0; c < NU; ++c) rdu[c] += (TV ? Br[i * NU + c] : Brow[c]) * dv;
                    } else {
                        rdu[i - NX] += dv;
                    }
                    xd[i * kBD + tid] = dz;  // own slot
                    xg[i * kBD + tid] = dd;  // own slot; nobody reads xg until the next barrier
                }
                v[i] = vn;
                z[i] = zn;
                th[i] = thn;
                be[i] = ben;
                la[i] = lan;
            }
            ++iters;
        }

        if (check) {
            // dual residual, xbar block: dz_{k+1} + Abar_{k+1}' (dz_{k+2} - dv_{k+1})
            T rdpart = T(0);
            if (run) {
#pragma unroll
                for (int c = 0; c < NU; ++c) rdpart = fmax(rdpart, fabs(rdu[c]));
                T tg[NB];
#pragma unroll
                for (int c = 0; c < NB; ++c) tg[c] = (c < NX) ? T(0) : xg[c * kBD + tid];
#pragma unroll
                for (int r = 0; r < NX; ++r) {
                    const T dd = xg[r * kBD + tid];
                    const cptr<T> Arow = ROW(Am, r, NX);
                    const cptr<T> Brow = ROW(Bm, r, NU);
#pragma unroll
                    for (int c = 0; c < NX; ++c) tg[c] += (TV ? Ar[r * NX + c] : Arow[c]) * dd;
#pragma unroll
                    for (int c = 0; c < NU; ++c) tg[NX + c] += (TV ? Br[r * NU + c] : Brow[c]) * dd;
                }
#pragma unroll
                for (int c = 0; c < NB; ++c) xg[c * kBD + tid] = tg[c];
            }
            __syncthreads();
            double csum = 0.0, rpm = 0.0, rdm = 0.0;
            if (run) {
                const bool hasnext = act && (k + 1 < N);
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    const T tv = xg[i * kBD + tid + 1];
                    const T tn = hasnext ? tv : T(0);
                    rdpart = fmax(rdpart, fabs(xd[i * kBD + tid] + tn));
                }
                if (!act) {
                    cpart = T(0);
                    rpart = T(0);
                    rdpart = T(0);
                }
                csum = wave_sum((double)cpart);
                rpm = wave_max((double)rpart);
                rdm = wave_max((double)rdpart);
                if (lane == 0) {
                    red[wave * 4 + 0] = csum;
                    red[wave * 4 + 1] = rpm;
                    red[wave * 4 + 2] = rdm;
                }
            }
            __syncthreads();
            if (run && leader) {
                const int nw = (N + 63) >> 6;
                double cs = 0.0, rp = 0.0, rd = 0.0;
                for (int w = gw0; w < gw0 + nw; ++w) {
                    cs += red[w * 4 + 0];
                    rp = fmax(rp, red[w * 4 + 1]);
                    rd = fmax(rd, red[w * 4 + 2]);
                }
                c_last = a.rho * cs;
                rp_last = rp;
                rd_last = a.rho * rd;
                bool stop = false;
                if (!(c_last < INFINITY)) {  // NaN or Inf
                    status = -4;
                    stop = true;
                }
                if (a.eps > 0.0 && c_last <= a.eps) stop = true;
                gdone[gw0] = stop ? 1 : 0;
            }
            __syncthreads();
            if (run) done = gdone[gw0] != 0;
            bool all_done = true;
            for (unsigned m = leader_mask; m; m &= m - 1) all_done = all_done && (gdone[__ffs(m) - 1] != 0);
            if (all_done) break;
        }
#undef ROW
    }

    // ---- outputs: final iterate, last step-1 results, u0, info
    if (act) {
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            st[(int64_t)(0 * NB + i) * N + k] = v[i];
            st[(int64_t)(1 * NB + i) * N + k] = z[i];
            st[(int64_t)(2 * NB + i) * N + k] = th[i];
            st[(int64_t)(3 * NB + i) * N + k] = be[i];
            st[(int64_t)(4 * NB + i) * N + k] = la[i];
        }
        if (a.write_iters) {
            const gptr<T> io = (gptr<T>)((T*)a.iters_out + I.it_off);
#pragma unroll
            for (int i = 0; i < NU; ++i) io[(int64_t)i * N + k] = du[i];
#pragma unroll
            for (int i = 0; i < NB; ++i) io[(int64_t)(NU + i) * N + k] = xs[i];
        }
    }
    if (leader) {
        const gptr<T> u0 = (gptr<T>)(T*)a.u0;
        const gptr<T> up = (gptr<T>)(T*)a.uprev;
        for (int i = 0; i < I.nu; ++i) u0[I.u_off + i] = (up ? up[I.u_off + i] : T(0)) + du[i];
        if (a.info) {
            InfoDev r;
            r.iters = iters;
            r.restarts = 0;
            r.c = c_last;
            r.r_prim = rp_last;
            r.r_dual = rd_last;
            r.status = status;
            r.pad = 0;
            ((gptr<InfoDev>)a.info)[inst_idx] = r;
        }
    }
#undef JM
#undef HM
#undef AM
#undef BM
#undef EM
#undef XB0
#undef PIMPC_MAT_PTRS
}

// One persistent kernel per class (each gets the whole register file; the
// classes of a batch run as concurrent branches of one graph).  Workgroups
// claim bins of this class from a counter, largest first.
template <typename T, int NX, int NU, bool TV>
__global__ void __launch_bounds__(kBinThreads) lane_kernel(const LaneArgs* __restrict__ ap) {
    const LaneArgs& a = *ap;
    int* gdone = (int*)((double*)((T*)lane_smem + (size_t)3 * a.nbmax * kBD) + kBinWaves * 4);
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
        if (threadIdx.x < kBinWaves) gdone[threadIdx.x] = 1;
        __syncthreads();
        if (my >= 0)
            lane_run<T, NX, NU, TV>(ap, bin.e[my].inst, true, bin.e[my].wave0, leader_mask);
        else
            lane_run<T, NX, NU, TV>(ap, 0, false, wave, leader_mask);
        __syncthreads();
    }
}

// Raise the kernel's dynamic-LDS limit to what this launch needs (only ever
// upwards; the default limit is 64 KiB).
template <typename T, int NX, int NU, bool TV>
hipError_t lane_lds_attr(size_t lds) {
    static size_t set_to = 64 * 1024;
    if (lds <= set_to) return hipSuccess;
    hipError_t e = hipFuncSetAttribute((const void*)lane_kernel<T, NX, NU, TV>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e == hipSuccess) set_to = lds;
    return e;
}

template <typename T, int NX, int NU, bool TV>
hipError_t launch_lane_cls(const LaneArgs* a_dev, int nbmax, int grid, hipStream_t s) {
    const size_t lds = lane_lds_bytes(nbmax, sizeof(T));
    hipError_t e = lane_lds_attr<T, NX, NU, TV>(lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((lane_kernel<T, NX, NU, TV>), dim3(grid), dim3(kBinThreads), lds, s, a_dev);
    return hipGetLastError();
}

template <typename T, int NX, int NU, bool TV>
int lane_occupancy(int nbmax) {
    const size_t lds = lane_lds_bytes(nbmax, sizeof(T));
    if (lane_lds_attr<T, NX, NU, TV>(lds) != hipSuccess) return -1;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lane_kernel<T, NX, NU, TV>, kBinThreads, lds) !=
        hipSuccess)
        return -1;
    return nb > 0 ? nb : 1;
}

// Class dispatch, split into parts compiled separately (PIMPC_LANE_PART of
// PIMPC_LANE_NPARTS) so the per-class kernels build in parallel.
template <int P>
hipError_t lane_dispatch(int fp64, int cls, const LaneArgs* a_dev, int nbmax, int grid, hipStream_t s,
                         int* occ, bool* handled) {
    *handled = false;
#define PIMPC_CASE(id, nx, nu, tv)                                                           \
    if constexpr ((id) % PIMPC_LANE_NPARTS == P) {                                          \
        if (cls == (id)) {                                                                  \
            *handled = true;                                                                \
            if (occ) {                                                                      \
                *occ = fp64 ? lane_occupancy<double, nx, nu, tv>(nbmax)                     \
                            : lane_occupancy<float, nx, nu, tv>(nbmax);                     \
                return *occ > 0 ? hipSuccess : hipErrorInvalidValue;                        \
            }                                                                               \
            return fp64 ? launch_lane_cls<double, nx, nu, tv>(a_dev, nbmax, grid, s)        \
                        : launch_lane_cls<float, nx, nu, tv>(a_dev, nbmax, grid, s);        \
        }                                                                                   \
    }
#define PIMPC_CASE_TI(id, nx, nu) PIMPC_CASE(id, nx, nu, false)
#define PIMPC_CASE_TV(id, nx, nu) PIMPC_CASE(id, nx, nu, true)
    PIMPC_LANE_CLASSES(PIMPC_CASE_TI)
    PIMPC_LANE_TV_CLASSES(PIMPC_CASE_TV)
#undef PIMPC_CASE_TI
#undef PIMPC_CASE_TV
#undef PIMPC_CASE
    return hipSuccess;
}

#ifdef PIMPC_LANE_PART
template hipError_t lane_dispatch<PIMPC_LANE_PART>(int, int, const LaneArgs*, int, int, hipStream_t, int*,
                                                   bool*);
#endif

}  // namespace pimpc
