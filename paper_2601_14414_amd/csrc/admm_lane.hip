// admm_lane.hip -- lane-per-stage ADMM kernel for batches of small instances.
//
// Implements the closed-form, parallel-in-horizon iteration of eqn. (8) /
// Algorithm 1 steps 1-5 of arXiv 2601.14414 in the velocity form of
// Theorem 2.  Mapping on gfx950:
//   * one lane owns one horizon stage k and keeps its five iterate vectors
//     (v_k, z_{k+1}, theta_k, beta_k, lambda_k) in VGPRs for all iterations;
//   * an instance occupies ceil(N/64) consecutive waves of a 512-thread
//     workgroup (256 threads for FP64 classes whose horizons all fit four
//     waves); several instances share a workgroup ("bin");
//   * time-invariant stage data (J, H, A, B, e, bounds) is uniform across the
//     wave.  FP32 box classes up to 19 wide (nu <= 4) copy it once per bin
//     into a per-wave LDS image and read each row as float4 broadcasts (two
//     rows ahead of their use up to 18 wide, one at a time beyond); the other
//     classes and FP64 stream it row by row through SGPRs with scalar loads,
//     one row ahead of its use (each row's load overlaps the previous row's
//     FMAs), so that every mat-vec FMA takes its matrix operand from an SGPR;
//     time-varying stage data is loaded once into VGPRs per lane;
//   * the two one-stage halos of an iteration (g_{k+1} for step 1 and
//     xbar_k for step 2) move between neighbouring lanes with DPP wavefront
//     shifts; only the value crossing a wave boundary goes through a small
//     LDS slot, between two workgroup barriers;
//   * residuals (Algorithm 1 step 4 and Section IV-B) are reduced with
//     cross-lane shuffles, then across the instance's waves in LDS, in a
//     fixed order (deterministic);
//   * the kernel is persistent: each workgroup claims bins from a counter
//     until none is left (largest-cost bins first).
//   * restart acceleration (Algorithm 1 steps 6-7), when on, reduces c every
//     iteration and extrapolates the hats in registers from the previous
//     iterate, kept in a global buffer;
//   * a kernel variant per class (GS) projects onto non-box factor sets
//     (halfspace, hyperplane, second-order cone, l1 ball) once the whole
//     projection argument of a stage is known;
//   * another (REC, FP32 time-invariant boxes) writes, at every step, the
//     record the backward's reverse sweep reads (the full tape).
#include <hip/hip_runtime.h>

#include "pimpc_dev.hpp"
#include "pimpc_lane.hpp"
#include "pimpc_adjoint.hpp"
#include "lane_common.hpp"

namespace pimpc {

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

// Euclidean projection of the factor y[OFF .. OFF + n) (n <= NP real entries
// of a padded factor of NP) onto a non-box set of the proof of Theorem 1
// (closed forms as in Parikh and Boyd, "Proximal Algorithms", Ch. 6); the
// padded entries are left to the box clamp.  par = (a [NP], b) or (., r).
//   1 halfspace a'w <= b, 2 hyperplane a'w = b: w -= (a'w - b)_(+) / |a|^2 a
//   3 second-order cone |w_1..n-1| <= w_n: scale onto the cone surface
//   4 l1 ball |w|_1 <= r: soft threshold at theta = max over j of
//     (sum of the |w_i| >= |w_j|, minus r) / (their count)
template <typename T, int NP, int OFF, int NBT>
__device__ inline void project_factor(T (&y)[NBT], int kind, int n, cptr<T> par) {
    if (kind == 1 || kind == 2) {
        T s = T(0), aa = T(0);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            const T a = par[i];  // zero beyond n
            s += a * y[OFF + i];
            aa += a * a;
        }
        s -= par[NP];
        if (kind == 2 || s > T(0)) {
            const T f = s / aa;
#pragma unroll
            for (int i = 0; i < NP; ++i) y[OFF + i] -= f * par[i];
        }
    } else if (kind == 3) {
        T t = T(0), q = T(0);
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            if (i == n - 1) t = y[OFF + i];
            if (i < n - 1) q += y[OFF + i] * y[OFF + i];
        }
        const T nq = sqrt(q);
        if (nq <= t) return;
        const bool zero = nq <= -t;
        const T al = (nq + t) * T(0.5);
        const T sc = zero ? T(0) : al / nq;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            if (i < n - 1) y[OFF + i] *= sc;
            if (i == n - 1) y[OFF + i] = zero ? T(0) : al;
        }
    } else if (kind == 4) {
        const T r = par[NP];
        T l1 = T(0);
#pragma unroll
        for (int i = 0; i < NP; ++i)
            if (i < n) l1 += fabs(y[OFF + i]);
        if (l1 <= r) return;
        T theta = T(0);
        bool first = true;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            if (j >= n) continue;
            const T mj = fabs(y[OFF + j]);
            T sj = T(0), cj = T(0);
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const T mi = fabs(y[OFF + i]);
                if (i < n && mi >= mj) {
                    sj += mi;
                    cj += T(1);
                }
            }
            const T tj = (sj - r) / cj;
            theta = (first || tj > theta) ? tj : theta;
            first = false;
        }
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            if (i >= n) continue;
            const T a = fabs(y[OFF + i]) - theta;
            y[OFF + i] = a > T(0) ? (y[OFF + i] > T(0) ? a : -a) : T(0);
        }
    }
}

// DPP wavefront shifts by one lane (32-bit moves; a double moves as two
// halves).  shl1: lane i receives lane i + 1 (lane 63 receives 0);
// shr1: lane i receives lane i - 1 (lane 0 receives 0).
__device__ __forceinline__ int dpp_shl1(int x) { return __builtin_amdgcn_update_dpp(0, x, 0x130, 0xf, 0xf, false); }
__device__ __forceinline__ int dpp_shr1(int x) { return __builtin_amdgcn_update_dpp(0, x, 0x138, 0xf, 0xf, false); }
__device__ __forceinline__ float shl1(float x) { return __int_as_float(dpp_shl1(__float_as_int(x))); }
__device__ __forceinline__ float shr1(float x) { return __int_as_float(dpp_shr1(__float_as_int(x))); }
__device__ __forceinline__ double shl1(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = dpp_shl1((int)(b & 0xffffffffll)), hi = dpp_shl1((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double shr1(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = dpp_shr1((int)(b & 0xffffffffll)), hi = dpp_shr1((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Run (or, with have = false, only shadow the barrier sequence of) one
// instance on the waves [gw0, gw0 + gnw) of the workgroup.
// Time-invariant FP32 box classes up to 19 entries wide (nu <= 4) read their
// stage matrices from a per-wave LDS image instead of the SGPR row stream
// (see MatImg).  Up to 18 wide, two rows are in flight behind in-order
// waits; measured per class (batches of 512-1024 instances, 300 iterations):
// (12,1..4) 17-20 % and (16,1..2) 21-23 % faster than SGPR rows, though the
// rows in flight cost the widest of them a few dozen spilled VGPRs.  With
// two rows in flight (16,3) and (16,4) spill 180-230 VGPRs and run 5-31 %
// slower; with one row at a time (16,3) runs 20 % faster.  (16,4) keeps the
// SGPR stream: alone it ran 1-3 % faster on LDS rows, but the 4096-instance
// batch ran 2.7 % faster with it on SGPR rows (with xbar_0 in LDS).  (8,8)
// keeps it too (LDS rows would spill 161 VGPRs there against 24), and so
// does FP64 (measured: the single FP64 chain gains nothing from LDS rows).
template <typename T, int NX, int NU, bool TV, bool GS, int BW>
constexpr bool lane_lds_rows() {
    return !TV && !GS && sizeof(T) == 4 && NX + NU <= 19 && NU <= 4;
}
// Rows the LDS row stream keeps in flight beyond the one in use ((16,3):
// one row at a time).
template <int NX, int NU>
constexpr int lane_row_depth() { return NX + NU > 18 ? 0 : 2; }
template <int NX, int NU>
constexpr int lane_img_stride() { return (MatImg<NX, NU>::TOT + 3) & ~3; }

template <typename T, int NX, int NU, bool TV, bool GS, int BW, bool REC>
__device__ __forceinline__ void lane_run(const LaneArgs* ap_in, int inst_idx, bool have, int gw0,
                                         unsigned leader_mask, T (*bnd_g)[NX + NU], T (*bnd_x)[NX + NU],
                                         T (*dzl)[64 * BW], T (*ddl)[64 * BW], double* red, int* gdone,
                                         T* limg, T (*xb0l)[NX + NU]) {
    inst_idx = __builtin_amdgcn_readfirstlane(inst_idx);
    gw0 = __builtin_amdgcn_readfirstlane(gw0);
    have = __builtin_amdgcn_readfirstlane((int)have) != 0;
    leader_mask = __builtin_amdgcn_readfirstlane(leader_mask);
    // SGPRs are the scarce resource of this kernel (every matrix row streams
    // through them): launch parameters are re-read where they are used, via
    // an opaque copy of the pointer (scalar loads that hit the scalar cache),
    // instead of being held in SGPRs across the iteration loop.
    const cptr<LaneArgs> ap = (cptr<LaneArgs>)uniform_ptr(ap_in);
    const cptr<InstDev> ip = ((cptr<InstDev>)uniform_ptr((*ap).inst)) + (have ? inst_idx : 0);
    auto AP = [&]() {
        cptr<LaneArgs> p = ap;
        asm volatile("" : "+s"(p));
        return p;
    };
    auto IP = [&]() {
        cptr<InstDev> p = ip;
        asm volatile("" : "+s"(p));
        return p;
    };
    constexpr int NB = NX + NU;
    constexpr bool kPF = NB <= 16;  // row prefetch (see stream_rows)
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int k = tid - gw0 * 64;  // stage owned by this lane
    const int N = have ? (*ip).N : 0;
    const bool act = have && k >= 0 && k < N;
    const bool leader = have && k == 0;
    const T rho = (T)(*ap).rho;
    const T third = (T)(1.0 / 3.0);

    const MatOffsets o = mat_offsets(NX, NU, have ? N : 1, TV);
    // matrix block of the instance (re-derived each iteration, see above)
    auto MB = [&]() {
        const T* m = (const T*)(*AP()).mats;
        return (cptr<T>)uniform_ptr(have ? m + (*IP()).mat_off : m);
    };
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

    using MI = MatImg<NX, NU>;
    constexpr int NBP = MI::NBP;
    constexpr bool kLR = lane_lds_rows<T, NX, NU, TV, GS, BW>();
    constexpr int kRD = lane_row_depth<NX, NU>();
    T* img = limg + (kLR ? wave * lane_img_stride<NX, NU>() : 0);  // this wave's matrix image
    if constexpr (kLR) {
        fill_mat_img<T, NX, NU>(img, (const T*)(*ap).mats + (have ? (*ip).mat_off : 0), o, have, lane);
        __builtin_amdgcn_wave_barrier();
    }

    // per-lane stage data (time-varying only)
    T Jr[TV ? NU * NB : 1], Hr[TV ? NB * NB : 1], Ar[TV ? NX * NX : 1], Br[TV ? NX * NU : 1],
        er[TV ? NX : 1];
    if constexpr (TV) {
        PIMPC_MAT_PTRS(MB())
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

    // xbar_0 = col(x(t), u(t-1)): uniform over the instance, read through the
    // scalar cache where lane k = 0 needs it.
#define XB0(i) ((i) < NX ? ((i) < nx_real ? x0p[(i)] : T(0)) \
                         : ((upp && (i) - NX < nu_real) ? upp[(i) - NX] : T(0)))
    // xbar_0, which stage 0 reads at every step 2, goes to this wave's LDS
    // slot once: re-reading it through the scalar cache exposed a round trip
    // per iteration (measured: the single FP64 chain 0.90 -> 0.81 ms, the
    // 4096-instance batch 16.2-16.5 -> 15.2-15.4 ms).  The 24-wide class
    // keeps the scalar loads.
    constexpr bool kXL = NX + NU <= 20;
    if constexpr (kXL) {
        const cptr<T> x0p = (cptr<T>)uniform_ptr((const T*)(*ap).x0 + (have ? (*ip).x_off : 0));
        const T* upraw = (const T*)(*ap).uprev;
        const cptr<T> upp = (cptr<T>)uniform_ptr(upraw ? upraw + (have ? (*ip).u_off : 0) : nullptr);
        const int nx_real = have ? (*ip).nx : 0, nu_real = have ? (*ip).nu : 0;
        if (lane < NB) xb0l[wave][lane] = XB0(lane);
        __builtin_amdgcn_wave_barrier();
    }

    // iterate (v, z, theta, beta, lambda) of this stage
    T v[NB], z[NB], th[NB], be[NB], la[NB];
    auto ST = [&]() { return (gptr<T>)(have ? (T*)(*AP()).state + (*IP()).st_off : (T*)(*AP()).state); };
    const gptr<T> st = ST();
    const bool warm = (*ap).warm != 0;
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        const bool ld = act && warm;
        v[i] = ld ? st[(int64_t)(0 * NB + i) * N + k] : T(0);
        z[i] = ld ? st[(int64_t)(1 * NB + i) * N + k] : T(0);
        th[i] = ld ? st[(int64_t)(2 * NB + i) * N + k] : T(0);
        be[i] = ld ? st[(int64_t)(3 * NB + i) * N + k] : T(0);
        la[i] = ld ? st[(int64_t)(4 * NB + i) * N + k] : T(0);
    }
    // du of the last step 1 is kept for u0; the step-1 outputs of an iteration
    // (du, xbar) are written out on check iterations, which include the last
    // one, so xbar need not stay in registers across iterations
    T du[NU];
#pragma unroll
    for (int i = 0; i < NU; ++i) du[i] = T(0);

    const bool last_wave = have && ((N - 1) >> 6) == (k >> 6) && k >= 0;
    const bool is_last = act && k == N - 1;
    const bool hb_diag = have && (*ip).hb_diag;
    const bool hasnext = act && k + 1 < N;
    const bool from_next_wave = hasnext && lane == 63;  // stage k + 1 is lane 0 of the next wave
    const bool from_prev_wave = act && k > 0 && lane == 0;

    int iters = 0;
    bool done = !have;
    double c_last = 0.0, rp_last = 0.0, rd_last = 0.0;
    int status = 0;
    // restart acceleration state of the instance (the same in all its lanes)
    const bool accel = (*ap).accel != 0;
    double alpha = 1.0, c_prev = 1.0, coef = 0.0;
    int restarts = 0;
    if (accel && act) {  // the iterate entering the first step is the first "previous" one
        const gptr<T> pv = (gptr<T>)((T*)(*AP()).prev + (*IP()).st_off);
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            pv[(int64_t)(0 * NB + i) * N + k] = v[i];
            pv[(int64_t)(1 * NB + i) * N + k] = z[i];
            pv[(int64_t)(2 * NB + i) * N + k] = th[i];
            pv[(int64_t)(3 * NB + i) * N + k] = be[i];
            pv[(int64_t)(4 * NB + i) * N + k] = la[i];
        }
    }

    const int K = (*ap).K;
    const bool use_eps = (*ap).eps > 0.0;
    const int check_every = (*ap).check_every;
    const int ckpt_every = (*ap).ckpt_every;
    // Checkpoints and records are written with non-temporal stores: only a
    // later kernel (the backward) reads them, and the full tape is far larger
    // than the caches (measured: the recording forward 1.5 % faster).
    // REC: a taped forward that records every step (FP32, time-invariant
    // boxes): the reverse sweep's record of the step -- d = v - beta, h, the
    // top rows of w = z - v - ebar + lambda and the box mask of the
    // projection -- so that the backward replays nothing.  A variant of its
    // own: the stores, even skipped, would change the plain kernel's register
    // allocation.
    static_assert(!REC || (sizeof(T) == 4 && !TV && !GS), "recorded steps: FP32, time-invariant, boxes");
    constexpr int kRec = tape_rec_floats(NB, NX);
    auto RECP = [&](int it) {
        return (gptr<T>)((T*)(*AP()).tape + (*IP()).tape_off + (int64_t)it * kRec * N);
    };
#pragma unroll 1
    for (int it = 0; it < K; ++it) {
        const bool check = (use_eps && ((it + 1) % check_every) == 0) || (it == K - 1);
        const bool need_c = check || accel;  // c^{i+1} is needed (accel decides every step)
        const bool run = !done;
        // taped forward: keep the iterate entering this iteration every ckpt_every steps
        if (ckpt_every > 0 && (it % ckpt_every) == 0 && act) {
            const gptr<T> ck =
                (gptr<T>)((T*)(*AP()).ckpt + (*IP()).ck_off + (int64_t)(it / ckpt_every) * 5 * NB * N);
#pragma unroll
            for (int i = 0; i < NB; ++i) {
                __builtin_nontemporal_store(v[i], &ck[(int64_t)(0 * NB + i) * N + k]);
                __builtin_nontemporal_store(z[i], &ck[(int64_t)(1 * NB + i) * N + k]);
                __builtin_nontemporal_store(th[i], &ck[(int64_t)(2 * NB + i) * N + k]);
                __builtin_nontemporal_store(be[i], &ck[(int64_t)(3 * NB + i) * N + k]);
                __builtin_nontemporal_store(la[i], &ck[(int64_t)(4 * NB + i) * N + k]);
            }
        }
        const cptr<T> Mi = MB();
        PIMPC_MAT_PTRS(Mi)
        // the image behind an opaque offset: its reads stay in this iteration
        int mo_ = 0;
        asm volatile("" : "+s"(mo_));
        const T* L = img + mo_;
        (void)L;
        if constexpr (REC) {
            if (act) {
                const gptr<T> tr = RECP(it);
#pragma unroll
                for (int i = 0; i < NB; ++i) __builtin_nontemporal_store(v[i] - be[i], &tr[(int64_t)i * N + k]);
#pragma unroll
                for (int i = 0; i < NX; ++i) {
                    const T ei = kLR ? L[MI::E + i] : (T)em[i];
                    __builtin_nontemporal_store(z[i] - v[i] - ei + la[i], &tr[(int64_t)(2 * NB + i) * N + k]);
                }
            }
        }

        // ---- step 1a: du_k = J_k (v_k - beta_k); g_k = Abar_k' (z_{k+1} - v_k - ebar_k + lambda_k)
        T g[NB], xs[NB];
        if (run) {
#pragma unroll
            for (int c = 0; c < NB; ++c) g[c] = (c < NX) ? T(0) : (z[c] - v[c] + la[c]);
            if constexpr (TV) {
#pragma unroll
                for (int r = 0; r < NU; ++r) {
                    T s = T(0);
#pragma unroll
                    for (int j = 0; j < NB; ++j) s += Jr[r * NB + j] * (v[j] - be[j]);
                    du[r] = s;
                }
#pragma unroll
                for (int r = 0; r < NX; ++r) {
                    const T w = z[r] - v[r] - er[r] + la[r];
#pragma unroll
                    for (int c = 0; c < NX; ++c) g[c] += Ar[r * NX + c] * w;
#pragma unroll
                    for (int c = 0; c < NU; ++c) g[NX + c] += Br[r * NU + c] * w;
                }
            } else if constexpr (kLR) {
                lds_rows<T, NU, NBP, kRD>(L + MI::J, [&](int r, const T (&x)[NBP]) {
                    T s = T(0);
#pragma unroll
                    for (int j = 0; j < NB; ++j) s += x[j] * (v[j] - be[j]);
                    du[r] = s;
                });
                lds_rows<T, NX, NBP, kRD>(L + MI::AB, [&](int i, const T (&x)[NBP]) {
                    const T w = z[i] - v[i] - L[MI::E + i] + la[i];
#pragma unroll
                    for (int c = 0; c < NB; ++c) g[c] += x[c] * w;
                });
            } else {
                // one stream: rows of J (du), then rows [A_r B_r e_r] (g)
                using Row = SRow<T, NB + 1>;
                stream_rows<Row, NU + NX, kPF>(
                    [&](int r) {
                        Row x;
                        if (r < NU) {
                            sload_into<T, NB>(x.x, Jm + r * NB);
                        } else {
                            sload_into<T, NX>(x.x, Am + (r - NU) * NX);
                            sload_into<T, NU>(x.x + NX, Bm + (r - NU) * NU);
                            sload_into<T, 1>(x.x + NB, em + (r - NU));
                        }
                        return x;
                    },
                    [&](int r, const Row& x) {
                        if (r < NU) {
                            T s = T(0);
#pragma unroll
                            for (int j = 0; j < NB; ++j) s += x.x[j] * (v[j] - be[j]);
                            du[r] = s;
                        } else {
                            const int i = r - NU;
                            const T w = z[i] - v[i] - x.x[NB] + la[i];
#pragma unroll
                            for (int c = 0; c < NB; ++c) g[c] += x.x[c] * w;
                        }
                    });
            }
            // g moves one lane down (stage k + 1 -> k); lane 0 of the wave
            // hands its g to the previous wave through LDS
            if (lane == 0) {
#pragma unroll
                for (int c = 0; c < NB; ++c) bnd_g[wave][c] = g[c];
            }
        }
        __syncthreads();
        if (run) {
#pragma unroll
            for (int c = 0; c < NB; ++c) g[c] = shl1(g[c]);  // g[] now holds g_{k+1}
        }

        // ---- step 1b: h_k = qbar + rho (z_{k+1} - theta_k + g_{k+1}); xbar_{k+1} = H_k h_k
        if (run) {
            T h[NB];
            // REC: h is recorded as soon as it is formed; stored after the H
            // rows instead it spilled hundreds of VGPRs in the 12-wide classes
            // ((12,4): 509, and a recording forward 6.9x the plain one)
            if constexpr (kLR) {
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    const T gn = from_next_wave ? bnd_g[wave + 1 < BW ? wave + 1 : wave][i] : g[i];
                    h[i] = L[MI::Q + i] + rho * (z[i] - th[i] + (hasnext ? gn : T(0)));
                }
                if constexpr (REC) {
                    if (act) {
                        const gptr<T> tr = RECP(it);
#pragma unroll
                        for (int i = 0; i < NB; ++i) __builtin_nontemporal_store(h[i], &tr[(int64_t)(NB + i) * N + k]);
                    }
                }
                // H_{N-1} for the last stage
                lds_rows<T, NB, NBP, kRD>(L + (is_last ? MI::Hb : MI::H), [&](int r, const T (&x)[NBP]) {
                    T s = T(0);
#pragma unroll
                    for (int j = 0; j < NB; ++j) s += x[j] * h[j];
                    xs[r] = s;
                });
            } else if constexpr (!TV) {
                T q[NB];
                sload_into<T, NB>(q, qb);
                swait();
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    const T gn = from_next_wave ? bnd_g[wave + 1 < BW ? wave + 1 : wave][i] : g[i];
                    h[i] = q[i] + rho * (z[i] - th[i] + (hasnext ? gn : T(0)));
                }
                if constexpr (REC) {
                    if (act) {
                        const gptr<T> tr = RECP(it);
#pragma unroll
                        for (int i = 0; i < NB; ++i) __builtin_nontemporal_store(h[i], &tr[(int64_t)(NB + i) * N + k]);
                    }
                }
                using Row = SRow<T, NB>;
                stream_rows<Row, NB, kPF>(
                    [&](int r) {
                        Row x;
                        sload_into<T, NB>(x.x, Hm + r * NB);
                        return x;
                    },
                    [&](int r, const Row& x) {
                        T s = T(0);
#pragma unroll
                        for (int j = 0; j < NB; ++j) s += x.x[j] * h[j];
                        xs[r] = s;
                    });
                if (last_wave) {  // wave-uniform: only the wave holding stage N-1
                    if (hb_diag) {
                        T d[NB];
                        cptr<T> Hbp = Hbm;
#pragma unroll
                        for (int r = 0; r < NB; ++r) {
                            asm volatile("" : "+s"(Hbp));
                            d[r] = Hbp[r * NB + r];
                        }
                        swait();
#pragma unroll
                        for (int r = 0; r < NB; ++r) xs[r] = is_last ? d[r] * h[r] : xs[r];
                    } else {
                        stream_rows<Row, NB, kPF>(
                            [&](int r) {
                                Row x;
                                sload_into<T, NB>(x.x, Hbm + r * NB);
                                return x;
                            },
                            [&](int r, const Row& x) {
                                T s = T(0);
#pragma unroll
                                for (int j = 0; j < NB; ++j) s += x.x[j] * h[j];
                                xs[r] = is_last ? s : xs[r];
                            });
                    }
                }
            } else {
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    const T gn = from_next_wave ? bnd_g[wave + 1 < BW ? wave + 1 : wave][i] : g[i];
                    h[i] = qb[i] + rho * (z[i] - th[i] + (hasnext ? gn : T(0)));
                }
#pragma unroll
                for (int r = 0; r < NB; ++r) {
                    T s = T(0);
#pragma unroll
                    for (int j = 0; j < NB; ++j) s += Hr[r * NB + j] * h[j];
                    xs[r] = s;
                }
            }
            // xbar moves one lane up (stage k -> k + 1); lane 63 hands its
            // xbar to the next wave through LDS
            if (lane == 63) {
#pragma unroll
                for (int c = 0; c < NB; ++c) bnd_x[wave][c] = xs[c];
            }
        }
        __syncthreads();

        // ---- steps 2-3: Theorem 1 closed form, box projection, dual update
        T rdu[NU];
        T cpart = T(0), rpart = T(0);
        // check iterations: dz and dd = dz - dv of every component go to LDS planes
        if (run) {
            // shift first, with every lane active (a DPP source lane that is
            // masked off reads as 0), then take the boundary value
            T xp[NB];
#pragma unroll
            for (int i = 0; i < NB; ++i) xp[i] = shr1(xs[i]);
            // xbar_0 = col(x(t), u(t-1)) for stage 0, from the wave's LDS slot
            const int wprev = wave > 0 ? wave - 1 : 0;
            if constexpr (kXL) {
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    const T xv = from_prev_wave ? bnd_x[wprev][i] : xp[i];
                    xp[i] = (k == 0) ? xb0l[wave][i] : (act ? xv : T(0));
                }
            } else {
                const cptr<T> x0p = (cptr<T>)uniform_ptr((const T*)(*AP()).x0 + (have ? (*IP()).x_off : 0));
                const T* upraw = (const T*)(*AP()).uprev;
                const cptr<T> upp = (cptr<T>)uniform_ptr(upraw ? upraw + (have ? (*IP()).u_off : 0) : nullptr);
                const int nx_real = have ? (*IP()).nx : 0, nu_real = have ? (*IP()).nu : 0;
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    const T xv = from_prev_wave ? bnd_x[wprev][i] : xp[i];
                    xp[i] = (k == 0) ? XB0(i) : (act ? xv : T(0));
                }
            }
#pragma unroll
            for (int c = 0; c < NU; ++c) rdu[c] = T(0);
            // the new iterate of component i from b_i, c_i and the projected z_i
            auto finish = [&](int i, T bi, T ci, T zn, auto&& brow) {
                const T gam = bi - ci;
                const T vn = (zn + gam) * T(0.5);
                const T thn = th[i] + xs[i] - zn;
                const T ben = bi - vn;
                const T lan = zn - vn - ci;
                if (need_c) {
                    const T dv = vn - v[i], dz = zn - z[i], dth = thn - th[i], dbe = ben - be[i],
                            dla = lan - la[i];
                    const T dd = dz - dv;
                    cpart += dth * dth + dbe * dbe + dla * dla + dz * dz + dv * dv + dd * dd;
                  if (check) {
                    rpart = fmax(rpart, fmax(fabs(dth), fmax(fabs(dbe), fabs(dla))));
                    // du block of F'G dq: Bbar_k' dv
                    if (i < NX) {
#pragma unroll
                        for (int c = 0; c < NU; ++c) rdu[c] += brow(c) * dv;
                    } else {
                        rdu[i - NX] += dv;
                    }
                    dzl[i][tid] = dz;
                    ddl[i][tid] = dd;
                  }
                }
                v[i] = vn;
                z[i] = zn;
                th[i] = thn;
                be[i] = ben;
                la[i] = lan;
            };
            // general sets: y, b, c of every component, projected after the stream
            T gy[GS ? NB : 1], gbv[GS ? NB : 1], gcv[GS ? NB : 1];
            uint32_t rmask = 0u;  // REC: bit i set where lb_i < y_i < ub_i
            // component i: b_i = (Bbar du)_i + beta_i;  c_i = (Abar xbar_k)_i + ebar_i - lambda_i
            // (rows are passed as accessors, never as addresses, so that they stay in registers)
            auto comp = [&](int i, auto&& arow, auto&& brow, T ei, T lo, T hi) {
                T bi, ci;
                if (i < NX) {
                    bi = be[i];
#pragma unroll
                    for (int j = 0; j < NU; ++j) bi += brow(j) * du[j];
                    ci = ei - la[i];
#pragma unroll
                    for (int j = 0; j < NX; ++j) ci += arow(j) * xp[j];
#pragma unroll
                    for (int j = 0; j < NU; ++j) ci += brow(j) * xp[NX + j];
                } else {
                    bi = du[i - NX] + be[i];
                    ci = xp[i] - la[i];
                }
                const T y = (T(2) * (xs[i] + th[i]) + bi + ci) * third;
                if constexpr (REC) {
                    if (y > lo && y < hi) rmask |= 1u << i;
                }
                if constexpr (GS) {
                    gy[i] = y;
                    gbv[i] = bi;
                    gcv[i] = ci;
                    (void)lo;
                    (void)hi;
                } else {
                    finish(i, bi, ci, clampv(y, lo, hi), brow);
                }
            };
            if constexpr (TV) {
                const cptr<T> lbq = lbm, ubq = ubm;
#pragma unroll
                for (int i = 0; i < NB; ++i)
                    comp(
                        i, [&](int j) { return Ar[(i < NX ? i : 0) * NX + j]; },
                        [&](int j) { return Br[(i < NX ? i : 0) * NU + j]; }, i < NX ? er[i] : T(0), lbq[i], ubq[i]);
            } else if constexpr (kLR) {
                lds_rows<T, NX, NBP, kRD>(L + MI::AB, [&](int i, const T (&x)[NBP]) {
                    comp(
                        i, [&](int j) { return x[j]; }, [&](int j) { return x[NX + j]; }, L[MI::E + i],
                        L[MI::LB + i], L[MI::UB + i]);
                });
#pragma unroll
                for (int i = NX; i < NB; ++i)
                    comp(
                        i, [&](int) { return T(0); }, [&](int) { return T(0); }, T(0), L[MI::LB + i],
                        L[MI::UB + i]);
            } else {
                // one stream over the components: [A_i B_i e_i lb_i ub_i] (i < NX), [lb_i ub_i]
                using Row = SRow<T, NB + 3>;
                stream_rows<Row, NB, kPF>(
                    [&](int i) {
                        Row x;
                        if (i < NX) {
                            sload_into<T, NX>(x.x, Am + i * NX);
                            sload_into<T, NU>(x.x + NX, Bm + i * NU);
                            sload_into<T, 1>(x.x + NB, em + i);
                        }
                        sload_into<T, 1>(x.x + NB + 1, lbm + i);
                        sload_into<T, 1>(x.x + NB + 2, ubm + i);
                        return x;
                    },
                    [&](int i, const Row& x) {
                        comp(
                            i, [&](int j) { return x.x[j]; }, [&](int j) { return x.x[NX + j]; },
                            i < NX ? x.x[NB] : T(0), x.x[NB + 1], x.x[NB + 2]);
                    });
            }
            if constexpr (REC) {
                if (act) __builtin_nontemporal_store(__uint_as_float(rmask), &RECP(it)[(int64_t)(2 * NB + NX) * N + k]);
            }
            if constexpr (GS) {
                // z = Proj_{X x U}(y): the non-box factor (if any) first, then the
                // box clamp (the identity on a non-box factor's real entries,
                // whose bounds are stored as -inf / +inf; zero on padding)
                const int xk = have ? (*IP()).xset : 0, uk = have ? (*IP()).uset : 0;
                const int nxr = have ? (*IP()).nx : 0, nur = have ? (*IP()).nu : 0;
                project_factor<T, NX, 0>(gy, xk, nxr, Mi + o.sx);
                project_factor<T, NU, NX>(gy, uk, nur, Mi + o.su);
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    const T zn = clampv(gy[i], (T)lbm[i], (T)ubm[i]);
                    if constexpr (TV)
                        finish(i, gbv[i], gcv[i], zn, [&](int j) { return Br[(i < NX ? i : 0) * NU + j]; });
                    else
                        finish(i, gbv[i], gcv[i], zn, [&](int j) { return (T)Bm[(i < NX ? i : 0) * NU + j]; });
                }
            }
            ++iters;
            if (check && act && (*AP()).write_iters) {
                const gptr<T> io = (gptr<T>)((T*)(*AP()).iters_out + (*IP()).it_off);
#pragma unroll
                for (int i = 0; i < NU; ++i) io[(int64_t)i * N + k] = du[i];
#pragma unroll
                for (int i = 0; i < NB; ++i) io[(int64_t)(NU + i) * N + k] = xs[i];
            }
        }

        if (check || accel) {  // residuals (uniform over the workgroup: check, accel, K)
            T rdpart = T(0);
            T tg[NB];
            if (check) {
                // dual residual, xbar block: dz_{k+1} + Abar_{k+1}' (dz_{k+2} - dv_{k+1})
                if (run) {
#pragma unroll
                    for (int c = 0; c < NU; ++c) rdpart = fmax(rdpart, fabs(rdu[c]));
                    // Abar_k' dd_k (its next-stage copy enters the xbar block)
#pragma unroll
                    for (int c = 0; c < NB; ++c) tg[c] = (c < NX) ? T(0) : ddl[c][tid];
                    if constexpr (TV) {
#pragma unroll
                        for (int r = 0; r < NX; ++r) {
                            const T dd = ddl[r][tid];
#pragma unroll
                            for (int c = 0; c < NX; ++c) tg[c] += Ar[r * NX + c] * dd;
#pragma unroll
                            for (int c = 0; c < NU; ++c) tg[NX + c] += Br[r * NU + c] * dd;
                        }
                    } else if constexpr (kLR) {
                        lds_rows<T, NX, NBP, kRD>(L + MI::AB, [&](int r, const T (&x)[NBP]) {
                            const T dd = ddl[r][tid];
#pragma unroll
                            for (int c = 0; c < NB; ++c) tg[c] += x[c] * dd;
                        });
                    } else {
                        PIMPC_MAT_PTRS(MB())
                        using Row = SRow<T, NB>;
                        stream_rows<Row, NX, kPF>(
                            [&](int r) {
                                Row x;
                                sload_into<T, NX>(x.x, Am + r * NX);
                                sload_into<T, NU>(x.x + NX, Bm + r * NU);
                                return x;
                            },
                            [&](int r, const Row& x) {
                                const T dd = ddl[r][tid];
#pragma unroll
                                for (int c = 0; c < NB; ++c) tg[c] += x.x[c] * dd;
                            });
                    }
                    if (lane == 0) {  // the g slots are free again (read before the last barrier)
#pragma unroll
                        for (int c = 0; c < NB; ++c) bnd_g[wave][c] = tg[c];
                    }
                }
                __syncthreads();
            }
            if (run) {
                if (check) {
#pragma unroll
                    for (int i = 0; i < NB; ++i) tg[i] = shl1(tg[i]);  // every lane active (see step 2)
                    const int wnext = wave + 1 < BW ? wave + 1 : wave;
#pragma unroll
                    for (int i = 0; i < NB; ++i) {
                        const T tn = from_next_wave ? bnd_g[wnext][i] : tg[i];
                        rdpart = fmax(rdpart, fabs(dzl[i][tid] + (hasnext ? tn : T(0))));
                    }
                }
                if (!act) {
                    cpart = T(0);
                    rpart = T(0);
                    rdpart = T(0);
                }
                const double csum = wave_sum((double)cpart);
                double rpm = 0.0, rdm = 0.0;
                if (check) {
                    rpm = wave_max((double)rpart);
                    rdm = wave_max((double)rdpart);
                }
                if (lane == 0) {
                    red[wave * 4 + 0] = csum;
                    red[wave * 4 + 1] = rpm;
                    red[wave * 4 + 2] = rdm;
                }
            }
            __syncthreads();
            if (run) {
                // every wave of the instance sums the same partials in the same
                // order, so all of them take the same decisions
                const int nw = (N + 63) >> 6;
                double cs = 0.0, rp = 0.0, rd = 0.0;
                for (int w = gw0; w < gw0 + nw; ++w) {
                    cs += red[w * 4 + 0];
                    rp = fmax(rp, red[w * 4 + 1]);
                    rd = fmax(rd, red[w * 4 + 2]);
                }
                const double rho64 = (*AP()).rho;
                const double c_now = rho64 * cs;
                bool stop = false;
                if (check) {
                    c_last = c_now;
                    rp_last = rp;
                    rd_last = rho64 * rd;
                    if (!(c_now < INFINITY)) {  // NaN or Inf
                        status = -4;
                        stop = true;
                    }
                    if (use_eps && c_now <= (*AP()).eps) stop = true;
                }
                // steps 6-7 (restart acceleration): momentum while c keeps
                // falling by the factor eta, else restart (alpha = 1, hats =
                // current iterate); c_prev starts at 1
                if (accel && !stop) {
                    if (c_now <= (*AP()).eta * c_prev) {
                        const double a1 = 0.5 + 0.5 * sqrt(1.0 + 4.0 * alpha * alpha);
                        coef = (alpha - 1.0) / a1;
                        alpha = a1;
                    } else {
                        alpha = 1.0;
                        coef = 0.0;
                        ++restarts;
                    }
                    c_prev = c_now;
                }
                if (leader) gdone[gw0] = stop ? 1 : 0;
            }
            __syncthreads();
            if (run) done = gdone[gw0] != 0;
            bool all_done = true;
            for (unsigned m = leader_mask; m; m &= m - 1) all_done = all_done && (gdone[__ffs(m) - 1] != 0);
            if (all_done) break;
            // hats for the next iteration: new + coef (new - previous); the
            // previous actual iterate moves to `prev` (not after the last step)
            if (accel && run && !done && it + 1 < K && act) {
                const gptr<T> pv = (gptr<T>)((T*)(*AP()).prev + (*IP()).st_off);
                const T cf = (T)coef;
                // the hats are the new iterate itself after a restart (and
                // while alpha is 1): then the previous iterate is only
                // replaced, not read (the decision is uniform over the wave)
                if (cf == T(0)) {
#pragma unroll
                    for (int i = 0; i < NB; ++i) {
                        pv[(int64_t)(0 * NB + i) * N + k] = v[i];
                        pv[(int64_t)(1 * NB + i) * N + k] = z[i];
                        pv[(int64_t)(2 * NB + i) * N + k] = th[i];
                        pv[(int64_t)(3 * NB + i) * N + k] = be[i];
                        pv[(int64_t)(4 * NB + i) * N + k] = la[i];
                    }
                } else
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    const int64_t o0 = (int64_t)(0 * NB + i) * N + k, o1 = (int64_t)(1 * NB + i) * N + k,
                                  o2 = (int64_t)(2 * NB + i) * N + k, o3 = (int64_t)(3 * NB + i) * N + k,
                                  o4 = (int64_t)(4 * NB + i) * N + k;
                    const T p0 = pv[o0], p1 = pv[o1], p2 = pv[o2], p3 = pv[o3], p4 = pv[o4];
                    pv[o0] = v[i];
                    pv[o1] = z[i];
                    pv[o2] = th[i];
                    pv[o3] = be[i];
                    pv[o4] = la[i];
                    v[i] += cf * (v[i] - p0);
                    z[i] += cf * (z[i] - p1);
                    th[i] += cf * (th[i] - p2);
                    be[i] += cf * (be[i] - p3);
                    la[i] += cf * (la[i] - p4);
                }
            }
        }
    }

    // ---- outputs: final iterate, last step-1 results, u0, info
    if (act) {
        const gptr<T> sto = ST();
#pragma unroll
        for (int i = 0; i < NB; ++i) {
            sto[(int64_t)(0 * NB + i) * N + k] = v[i];
            sto[(int64_t)(1 * NB + i) * N + k] = z[i];
            sto[(int64_t)(2 * NB + i) * N + k] = th[i];
            sto[(int64_t)(3 * NB + i) * N + k] = be[i];
            sto[(int64_t)(4 * NB + i) * N + k] = la[i];
        }
        if (iters == 0 && (*AP()).write_iters) {  // no step was taken
            const gptr<T> io = (gptr<T>)((T*)(*AP()).iters_out + (*IP()).it_off);
#pragma unroll
            for (int i = 0; i < NU + NB; ++i) io[(int64_t)i * N + k] = T(0);
        }
    }
    if (leader) {
        const LaneArgs a = *AP();
        const InstDev I = *IP();
        const gptr<T> u0 = (gptr<T>)(T*)a.u0;
        const gptr<T> up = (gptr<T>)(T*)a.uprev;
        for (int i = 0; i < I.nu; ++i) u0[I.u_off + i] = (up ? up[I.u_off + i] : T(0)) + du[i];
        if (a.info) {
            InfoDev r;
            r.iters = iters;
            r.restarts = restarts;
            r.c = c_last;
            r.r_prim = rp_last;
            r.r_dual = rd_last;
            r.status = (a.fbad && a.fbad[inst_idx]) ? -3 : status;  // -3: the factorisation failed (not SPD)
            r.pad = 0;
            ((gptr<InfoDev>)a.info)[inst_idx] = r;
        }
    }
#undef XB0
#undef PIMPC_MAT_PTRS
}

// One persistent kernel per class (each gets the whole register file; the
// classes of a batch run as concurrent branches of one graph).  Workgroups
// claim bins of BW waves of this class from a counter, largest first.
// Narrow FP32 stages fit two 512-thread workgroups per CU (<= 128 VGPRs a
// lane); wider ones take the whole register file with one.  FP64 classes
// whose horizons all fit four waves run 256-thread workgroups, one wave per
// SIMD with up to 512 registers (their doubled vectors spill past 256).
constexpr int lane_waves_per_eu(int nb, int tsize, int bw) {
    return bw == 4 ? 1 : ((tsize == 4 && nb <= 7) ? 4 : 2);
}

template <typename T, int NX, int NU, bool TV, bool GS, int BW, bool REC>
__global__ void __launch_bounds__(64 * BW)
    __attribute__((amdgpu_waves_per_eu(lane_waves_per_eu(NX + NU, sizeof(T), BW))))
    lane_kernel(const LaneArgs* __restrict__ ap) {
    static_assert(BW == 4 || BW == kBinWaves, "bins of four or eight waves");
    const LaneArgs& a = *ap;
    __shared__ T bnd_g[BW][NX + NU];   // g (and the dual-residual term) crossing a wave boundary
    __shared__ T bnd_x[BW][NX + NU];   // xbar crossing a wave boundary
    __shared__ T dzl[NX + NU][64 * BW];  // check iterations: dz of every lane
    __shared__ T ddl[NX + NU][64 * BW];  // check iterations: dz - dv of every lane
    __shared__ double red[BW * 4];       // per-wave residual partials
    __shared__ int gdone[BW];            // per-instance stop flags (indexed by first wave)
    constexpr bool kLR = lane_lds_rows<T, NX, NU, TV, GS, BW>();
    __shared__ __align__(16) T limg[kLR ? BW * lane_img_stride<NX, NU>() : 1];  // matrix images
    __shared__ T xb0l[BW][NX + NU];      // xbar_0 of each wave's instance
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
        if (threadIdx.x < BW) gdone[threadIdx.x] = 1;
        __syncthreads();
        if (my >= 0)
            lane_run<T, NX, NU, TV, GS, BW, REC>(ap, bin.e[my].inst, true, bin.e[my].wave0, leader_mask, bnd_g,
                                            bnd_x, dzl, ddl, red, gdone, limg, xb0l);
        else
            lane_run<T, NX, NU, TV, GS, BW, REC>(ap, 0, false, wave, leader_mask, bnd_g, bnd_x, dzl, ddl, red, gdone,
                                            limg, xb0l);
        __syncthreads();
    }
}

// whether the class has the variant that records every step
template <typename T, int NX, int NU, bool TV>
constexpr bool lane_has_rec() { return sizeof(T) == 4 && !TV && lane_rec_class(NX + NU); }

template <typename T, int NX, int NU, bool TV, int BW>
hipError_t launch_lane_cls(const LaneArgs* a_dev, int grid, hipStream_t s, bool gs, bool rec) {
    if (rec) {
        if constexpr (lane_has_rec<T, NX, NU, TV>()) {
            if (gs) return hipErrorInvalidValue;
            hipLaunchKernelGGL((lane_kernel<T, NX, NU, TV, false, BW, true>), dim3(grid), dim3(64 * BW), 0, s,
                               a_dev);
            return hipGetLastError();
        }
        return hipErrorInvalidValue;
    }
    if (gs)
        hipLaunchKernelGGL((lane_kernel<T, NX, NU, TV, true, BW, false>), dim3(grid), dim3(64 * BW), 0, s, a_dev);
    else
        hipLaunchKernelGGL((lane_kernel<T, NX, NU, TV, false, BW, false>), dim3(grid), dim3(64 * BW), 0, s, a_dev);
    return hipGetLastError();
}

template <typename T, int NX, int NU, bool TV, int BW>
int lane_occupancy(bool gs, bool rec) {
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    if (rec) {
        if constexpr (lane_has_rec<T, NX, NU, TV>())
            if (!gs)
                e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lane_kernel<T, NX, NU, TV, false, BW, true>,
                                                                 64 * BW, 0);
    } else {
        e = gs ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lane_kernel<T, NX, NU, TV, true, BW, false>,
                                                              64 * BW, 0)
               : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, lane_kernel<T, NX, NU, TV, false, BW, false>,
                                                              64 * BW, 0);
    }
    if (e != hipSuccess) return -1;
    return nb > 0 ? nb : 1;
}

// Class dispatch, split into parts compiled separately (PIMPC_LANE_PART of
// PIMPC_LANE_NPARTS) so the per-class kernels build in parallel.
// bw: waves per bin of the class's run (4 only for FP64 classes whose
// horizons all fit four waves); rec: the variant that records every step.
template <int P>
hipError_t lane_dispatch(int fp64, int cls, int gs, bool rec, const LaneArgs* a_dev, int bw, int grid,
                         hipStream_t s, int* occ, bool* handled) {
    *handled = false;
#define PIMPC_CASE(id, nx, nu, tv)                                                                \
    if constexpr ((id) % PIMPC_LANE_NPARTS == P) {                                               \
        if (cls == (id)) {                                                                       \
            *handled = true;                                                                     \
            if (occ) {                                                                           \
                if (!fp64)                                                                       \
                    *occ = lane_occupancy<float, nx, nu, tv, kBinWaves>(gs != 0, rec);           \
                else if constexpr (lane_fp64_class(nx + nu))                                     \
                    *occ = bw == 4 ? lane_occupancy<double, nx, nu, tv, 4>(gs != 0, rec)         \
                                   : lane_occupancy<double, nx, nu, tv, kBinWaves>(gs != 0, rec); \
                else                                                                             \
                    *occ = -1;                                                                   \
                return *occ > 0 ? hipSuccess : hipErrorInvalidValue;                             \
            }                                                                                    \
            if (!fp64) return launch_lane_cls<float, nx, nu, tv, kBinWaves>(a_dev, grid, s, gs != 0, rec); \
            if constexpr (lane_fp64_class(nx + nu)) {                                            \
                if (bw == 4) return launch_lane_cls<double, nx, nu, tv, 4>(a_dev, grid, s, gs != 0, rec); \
                return launch_lane_cls<double, nx, nu, tv, kBinWaves>(a_dev, grid, s, gs != 0, rec); \
            }                                                                                    \
            return hipErrorInvalidValue;                                                         \
        }                                                                                        \
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
template hipError_t lane_dispatch<PIMPC_LANE_PART>(int, int, int, bool, const LaneArgs*, int, int,
                                                   hipStream_t, int*, bool*);
#endif

}  // namespace pimpc
