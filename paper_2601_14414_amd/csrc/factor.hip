// factor.hip -- FP64 stage factorisation (Algorithm 1 "cache") on gfx950.
//
// For each instance and stage (proof of Theorem 2, eqn. (8)):
//   H_k = (Qbar + rho I + rho Abar_{k+1}' Abar_{k+1})^-1   (k < N-1)
//   H_{N-1} = (Qbar + rho I)^-1
//   J_k = (Bbar_k' Bbar_k)^-1 Bbar_k' = (B_k' B_k + I)^-1 [B_k'  I]
// or, with an input-rate weight W (cost 1/2 du' W du, Section V), the minimiser
// of 1/2 du' W du + rho/2 ||Bbar du - (v - beta)||^2:
//   J_k = (W / rho + B_k' B_k + I)^-1 [B_k'  I]
// with Abar = [[A, B], [0, I]], Bbar = [[B], [I]], Qbar = blkdiag(Q, R).
// One 64-thread workgroup builds one matrix in LDS, factors it by a
// right-looking Cholesky (pivot-column scaling and trailing update spread
// over the workgroup) and forms the inverse one column per thread, each
// column solved in LDS beside the factor.  The LDS is sized for the widest
// matrix of the launch (n x (n + 1) doubles twice), not for the widest
// class, so that narrow stages fit many workgroups on a compute unit.  All
// of it in double; results are stored in the iteration precision T.
//
// Also here: the kernels that expand the FP64 stage data into the T layout
// the ADMM kernels read, that load per-instance parameters from device
// tensors (differentiable path), and a plain fill kernel (used instead of
// hipMemsetAsync so the launch sequence can be graph-captured).
#include <hip/hip_runtime.h>

#include <cstring>

#include "pimpc_dev.hpp"

namespace pimpc {

constexpr int kMaxNb = 64;  // widest matrix a launch may hold (one column per thread)

// LDS of one factor workgroup for matrices up to nb wide: the matrix and the
// solution columns, each nb x (nb + 1) doubles (odd leading dimension).
__host__ __device__ inline size_t factor_lds_bytes(int nb) { return 2 * (size_t)nb * (nb + 1) * sizeof(double); }

// Cholesky of the n x n matrix in M (leading dimension ld; lower triangle
// overwritten by L); returns false if a pivot is not strictly positive (or
// not finite).
__device__ bool lds_cholesky(double* M, int n, int ld) {
    __shared__ int ok;
    const int t = threadIdx.x;
    if (t == 0) ok = 1;
    __syncthreads();
    for (int j = 0; j < n; ++j) {
        if (t == 0) {
            const double d = M[j * ld + j];
            if (!(d > 0.0) || !(d < INFINITY)) ok = 0;
            M[j * ld + j] = sqrt(fmax(d, 0.0));
        }
        __syncthreads();
        const double piv = M[j * ld + j];
        for (int i = j + 1 + t; i < n; i += blockDim.x) M[i * ld + j] = M[i * ld + j] / piv;
        __syncthreads();
        const int m = n - j - 1;
        for (int idx = t; idx < m * m; idx += blockDim.x) {
            const int i = j + 1 + idx / m;
            const int l = j + 1 + idx % m;
            if (l <= i) M[i * ld + l] -= M[i * ld + j] * M[l * ld + j];
        }
        __syncthreads();
    }
    return ok != 0;
}

// Solve L L' x = b in place; b is one thread's column, x[i] at x[i * xs]
// (LDS), L with leading dimension ld.
__device__ void chol_solve_col(const double* L, int n, int ld, double* x, int xs) {
    for (int i = 0; i < n; ++i) {
        double s = x[i * xs];
        for (int k = 0; k < i; ++k) s -= L[i * ld + k] * x[k * xs];
        x[i * xs] = s / L[i * ld + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = x[i * xs];
        for (int k = i + 1; k < n; ++k) s -= L[k * ld + i] * x[k * xs];
        x[i * xs] = s / L[i * ld + i];
    }
}

template <typename T>
__global__ void __launch_bounds__(64) factor_kernel(const InstDev* __restrict__ inst,
                                                    const FactorTask* __restrict__ tasks,
                                                    const double* __restrict__ mats64,
                                                    T* __restrict__ mats, double rho,
                                                    int32_t* __restrict__ bad, int32_t* __restrict__ ibad) {
    extern __shared__ double fsm[];  // factor_lds_bytes(widest NB of the launch)
    const FactorTask tk = tasks[blockIdx.x];
    const InstDev I = inst[tk.inst];
    const int NX = I.nxp, NU = I.nup, NB = I.nbp, N = I.N;
    const int ld = NB + 1;       // leading dimension of M and of the solution columns X
    double* M = fsm;
    double* X = fsm + NB * ld;   // column t of the right-hand sides / solutions at X[i * ld + t]
    const MatOffsets o = mat_offsets(NX, NU, N, I.tv);
    const double* b64 = mats64 + I.mat64_off;
    T* bt = mats + I.mat_off;
    const int t = threadIdx.x;

    if (tk.kind <= 1) {
        // M = Qbar + rho I (+ rho Abar_{k+1}' Abar_{k+1})
        const int sn = I.tv ? tk.stage + 1 : 0;
        const double* An = b64 + o.A64 + (int64_t)sn * NX * NX;
        const double* Bn = b64 + o.B64 + (int64_t)sn * NX * NU;
        const double* Q = b64 + o.Q64;
        const double* R = b64 + o.R64;
        for (int idx = t; idx < NB * NB; idx += blockDim.x) {
            const int i = idx / NB, j = idx % NB;
            double s = (i == j) ? rho : 0.0;
            if (i < NX && j < NX) s += Q[i * NX + j];
            if (i >= NX && j >= NX) s += R[(i - NX) * NU + (j - NX)];
            if (tk.kind == 0) {
                double a = 0.0;
                for (int r = 0; r < NX; ++r) {
                    const double ari = (i < NX) ? An[r * NX + i] : Bn[r * NU + (i - NX)];
                    const double arj = (j < NX) ? An[r * NX + j] : Bn[r * NU + (j - NX)];
                    a += ari * arj;
                }
                if (i >= NX && i == j) a += 1.0;
                s += rho * a;
            }
            M[i * ld + j] = s;
        }
        __syncthreads();
        const bool ok = lds_cholesky(M, NB, ld);
        if (!ok && t == 0) {
            bad[blockIdx.x] = 1;
            ibad[tk.inst] = 1;
        }
        if (t < NB) {
            double* x = X + t;
            for (int i = 0; i < NB; ++i) x[i * ld] = (i == t) ? 1.0 : 0.0;
            chol_solve_col(M, NB, ld, x, ld);
            // column t of H (H is symmetric)
            if (!I.tv) {
                T* H = bt + (tk.kind == 0 ? o.H : o.Hb);
                for (int i = 0; i < NB; ++i) H[i * NB + t] = (T)x[i * ld];
            } else {
                T* H = bt + o.H;
                for (int i = 0; i < NB; ++i) H[(int64_t)(i * NB + t) * N + tk.stage] = (T)x[i * ld];
            }
        }
    } else {
        // G = W / rho + B' B + I (NU x NU); J = G^-1 [B' I]
        const int sk = I.tv ? tk.stage : 0;
        const double* Bk = b64 + o.B64 + (int64_t)sk * NX * NU;
        const double* Wd = b64 + o.W64;
        for (int idx = t; idx < NU * NU; idx += blockDim.x) {
            const int i = idx / NU, j = idx % NU;
            double s = ((i == j) ? 1.0 : 0.0) + Wd[i * NU + j] / rho;
            for (int r = 0; r < NX; ++r) s += Bk[r * NU + i] * Bk[r * NU + j];
            M[i * ld + j] = s;
        }
        __syncthreads();
        const bool ok = lds_cholesky(M, NU, ld);
        if (!ok && t == 0) {
            bad[blockIdx.x] = 1;
            ibad[tk.inst] = 1;
        }
        if (t < NB) {
            double* x = X + t;
            for (int i = 0; i < NU; ++i) x[i * ld] = (t < NX) ? Bk[t * NU + i] : ((t - NX) == i ? 1.0 : 0.0);
            chol_solve_col(M, NU, ld, x, ld);
            T* J = bt + o.J;
            if (!I.tv) {
                for (int i = 0; i < NU; ++i) J[i * NB + t] = (T)x[i * ld];
            } else {
                for (int i = 0; i < NU; ++i) J[(int64_t)(i * NB + t) * N + tk.stage] = (T)x[i * ld];
            }
        }
    }
}

// Copy A, B, e from the FP64 block into the T block (row-major for
// time-invariant data, stage-minor for time-varying data).  One thread per
// element; grid-stride over all instances' elements via a flat index table.
template <typename T>
__global__ void expand_kernel(const InstDev* __restrict__ inst, int count,
                              const double* __restrict__ mats64, T* __restrict__ mats) {
    const int i = blockIdx.y;
    if (i >= count) return;
    const InstDev I = inst[i];
    const int NX = I.nxp, NU = I.nup, N = I.N;
    const MatOffsets o = mat_offsets(NX, NU, N, I.tv);
    const double* b64 = mats64 + I.mat64_off;
    T* bt = mats + I.mat_off;
    const int S = I.tv ? N : 1;
    const int per = NX * NX + NX * NU + NX;
    const int total = S * per;  // < 2^31 (checked at setup)
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
        const int k = idx / per;
        const int q = idx - k * per;
        double val;
        int64_t dst;
        if (q < NX * NX) {
            val = b64[o.A64 + (int64_t)k * NX * NX + q];
            dst = I.tv ? o.A + (int64_t)q * N + k : o.A + q;
        } else if (q < NX * NX + NX * NU) {
            const int qq = q - NX * NX;
            val = b64[o.B64 + (int64_t)k * NX * NU + qq];
            dst = I.tv ? o.B + (int64_t)qq * N + k : o.B + qq;
        } else {
            const int qq = q - NX * NX - NX * NU;
            val = b64[o.e64 + (int64_t)k * NX + qq];
            dst = I.tv ? o.e + (int64_t)qq * N + k : o.e + qq;
        }
        bt[dst] = (T)val;
    }
}

// Differentiable path: load per-instance A [nx][nx], B [nx][nu], diag Q,
// diag R (real sizes, context precision) into the padded FP64 block.
template <typename T>
__global__ void params_kernel(const InstDev* __restrict__ inst, int count, const T* __restrict__ A,
                              const T* __restrict__ B, const T* __restrict__ Qd,
                              const T* __restrict__ Rd, double* __restrict__ mats64) {
    const int i = blockIdx.x;
    if (i >= count) return;
    const InstDev I = inst[i];
    const int nx = I.nx, nu = I.nu, NX = I.nxp, NU = I.nup;
    const MatOffsets o = mat_offsets(NX, NU, I.N, 0);
    double* b64 = mats64 + I.mat64_off;
    for (int idx = threadIdx.x; idx < NX * NX; idx += blockDim.x) {
        const int r = idx / NX, c = idx % NX;
        b64[o.A64 + idx] = (r < nx && c < nx) ? (double)A[(int64_t)i * nx * nx + r * nx + c] : 0.0;
        b64[o.Q64 + idx] = (r == c) ? (r < nx ? (double)Qd[(int64_t)i * nx + r] : 1.0) : 0.0;
    }
    for (int idx = threadIdx.x; idx < NX * NU; idx += blockDim.x) {
        const int r = idx / NU, c = idx % NU;
        b64[o.B64 + idx] = (r < nx && c < nu) ? (double)B[(int64_t)i * nx * nu + r * nu + c] : 0.0;
    }
    for (int idx = threadIdx.x; idx < NU * NU; idx += blockDim.x) {
        const int r = idx / NU, c = idx % NU;
        b64[o.R64 + idx] = (r == c) ? (r < nu ? (double)Rd[(int64_t)i * nu + r] : 1.0) : 0.0;
    }
}

// Construction-free update from device memory: copy the caller's packed
// stage data (A_k, B_k, e_k at real sizes, row-major, per instance at the
// packed offsets pk[3 i + 0..2]) into the padded FP64 block; padded entries
// are zero.  Any non-finite value sets *nonfinite.  Grid (blocks, count).
__global__ void stage_import_kernel(const InstDev* __restrict__ inst, int count, const int64_t* __restrict__ pk,
                                    const double* __restrict__ A, const double* __restrict__ B,
                                    const double* __restrict__ e, double* __restrict__ mats64,
                                    int32_t* __restrict__ nonfinite) {
    const int i = blockIdx.y;
    if (i >= count) return;
    const InstDev I = inst[i];
    const int nx = I.nx, nu = I.nu, NX = I.nxp, NU = I.nup, N = I.N;
    const MatOffsets o = mat_offsets(NX, NU, N, I.tv);
    double* b64 = mats64 + I.mat64_off;
    const int S = I.tv ? N : 1;
    const int per = NX * NX + NX * NU + NX;
    const int64_t total = (int64_t)S * per;
    const double* Ai = A + pk[3 * i + 0];
    const double* Bi = B + pk[3 * i + 1];
    const double* ei = e ? e + pk[3 * i + 2] : nullptr;
    bool bad = false;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int k = (int)(idx / per);
        const int q = (int)(idx % per);
        double val = 0.0;
        int64_t dst;
        if (q < NX * NX) {
            const int r = q / NX, c = q % NX;
            if (r < nx && c < nx) val = Ai[(int64_t)k * nx * nx + r * nx + c];
            dst = o.A64 + (int64_t)k * NX * NX + q;
        } else if (q < NX * NX + NX * NU) {
            const int qq = q - NX * NX;
            const int r = qq / NU, c = qq % NU;
            if (r < nx && c < nu) val = Bi[(int64_t)k * nx * nu + r * nu + c];
            dst = o.B64 + (int64_t)k * NX * NU + qq;
        } else {
            const int r = q - NX * NX - NX * NU;
            if (ei && r < nx) val = ei[(int64_t)k * nx + r];
            dst = o.e64 + (int64_t)k * NX + r;
        }
        if (!isfinite(val)) bad = true;
        b64[dst] = val;
    }
    if (bad) *nonfinite = 1;
}

hipError_t launch_stage_import(const InstDev* inst, int count, const int64_t* pk, const double* A,
                               const double* B, const double* e, double* mats64, int32_t* nonfinite,
                               hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(stage_import_kernel, dim3(8, count), dim3(256), 0, s, inst, count, pk, A, B, e, mats64,
                       nonfinite);
    return hipGetLastError();
}

// Host bytes handed to the device as a kernel argument (the kernel argument
// block is copied at launch, and at capture time under graph capture), so a
// caller that may not allocate can still place small structures in device
// memory: one launch per chunk.
constexpr uint32_t kByteChunk = 3072;
struct ByteChunk {
    uint32_t n;
    uint32_t pad;
    unsigned char b[kByteChunk];
};

__global__ void __launch_bounds__(256) bytes_store_kernel(ByteChunk c, unsigned char* __restrict__ dst) {
    for (uint32_t i = threadIdx.x; i < c.n; i += blockDim.x) dst[i] = c.b[i];
}

hipError_t launch_bytes_store(void* dst, const void* src, size_t n, hipStream_t s) {
    for (size_t off = 0; off < n; off += kByteChunk) {
        ByteChunk c;
        c.n = (uint32_t)(n - off < kByteChunk ? n - off : kByteChunk);
        c.pad = 0;
        memcpy(c.b, (const unsigned char*)src + off, c.n);
        hipLaunchKernelGGL(bytes_store_kernel, dim3(1), dim3(256), 0, s, c, (unsigned char*)dst + off);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
__global__ void fill_kernel(T* __restrict__ p, int64_t n, T v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// ---------------------------------------------------------------- launchers

template <typename T>
hipError_t launch_factor(const InstDev* inst, const FactorTask* tasks, int ntasks, int nbmax, const double* mats64,
                         T* mats, double rho, int32_t* bad, int32_t* ibad, hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    if (nbmax < 1 || nbmax > kMaxNb) return hipErrorInvalidValue;
    hipLaunchKernelGGL(factor_kernel<T>, dim3(ntasks), dim3(64), factor_lds_bytes(nbmax), s, inst, tasks, mats64,
                       mats, rho, bad, ibad);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_expand(const InstDev* inst, int count, const double* mats64, T* mats, int tv, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    // time-varying data: N stages per instance, so more workgroups per instance
    hipLaunchKernelGGL(expand_kernel<T>, dim3(tv ? 32 : 4, count), dim3(256), 0, s, inst, count, mats64, mats);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_params(const InstDev* inst, int count, const T* A, const T* B, const T* Qd,
                         const T* Rd, double* mats64, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(params_kernel<T>, dim3(count), dim3(64), 0, s, inst, count, A, B, Qd, Rd, mats64);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T* p, int64_t n, T v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(fill_kernel<T>, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

template hipError_t launch_factor<float>(const InstDev*, const FactorTask*, int, int, const double*, float*,
                                         double, int32_t*, int32_t*, hipStream_t);
template hipError_t launch_factor<double>(const InstDev*, const FactorTask*, int, int, const double*, double*,
                                          double, int32_t*, int32_t*, hipStream_t);

template hipError_t launch_expand<float>(const InstDev*, int, const double*, float*, int, hipStream_t);
template hipError_t launch_expand<double>(const InstDev*, int, const double*, double*, int, hipStream_t);
template hipError_t launch_params<float>(const InstDev*, int, const float*, const float*, const float*,
                                         const float*, double*, hipStream_t);
template hipError_t launch_params<double>(const InstDev*, int, const double*, const double*,
                                          const double*, const double*, double*, hipStream_t);
template hipError_t launch_fill<float>(float*, int64_t, float, hipStream_t);
template hipError_t launch_fill<double>(double*, int64_t, double, hipStream_t);
template hipError_t launch_fill<int32_t>(int32_t*, int64_t, int32_t, hipStream_t);

}  // namespace pimpc
