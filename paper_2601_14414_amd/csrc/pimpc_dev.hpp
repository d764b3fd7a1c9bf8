// pimpc_dev.hpp -- data layout shared by the host runtime and the gfx950
// kernels of the piMPC ADMM path (internal; not part of the C ABI).
//
// Every instance is stored with *padded* sizes (nxp >= nx, nup >= nu) equal
// to one of the compiled kernel classes.  Padding is exact: padded state
// components have zero dynamics, zero coupling, a [0, 0] box and a unit
// weight, so they stay identically zero through every ADMM step.
#pragma once
#include <stdint.h>

namespace pimpc {

// Kernel families.
enum Family : int32_t {
    FAM_LANE = 0,  // one lane per stage, instance-per-wave-group bins
    FAM_ROW = 1,   // one lane per row of a stage, multi-workgroup horizon
};

struct InstDev {
    int32_t nx, nu, nb, N;     // real sizes
    int32_t nxp, nup, nbp;     // padded sizes (kernel class)
    int32_t cls;               // lane-family class index (-1 if row family)
    int32_t tv;                // time-varying stage data
    int32_t hb_diag;           // H_{N-1} is diagonal (time-invariant only)
    int32_t row_acc;           // row family: kernel with a reducer wave (eps stop, restart acceleration)
    int32_t row_s;             // row family: stages per wave (block size S)
    int32_t xset, uset;        // constraint-set kinds of the x and u factors (PIMPC_SET_*)
    int64_t mat_off;           // T matrix block (see layout below)
    int64_t mat64_off;         // FP64 factorisation inputs
    int64_t st_off;            // iterate block [5][nbp][N]
    int64_t it_off;            // last step-1 outputs: du [nup][N], then xbar [nbp][N]
    int64_t x_off, u_off;      // offsets into packed x0 (sum nx) and u (sum nu)
    int64_t ck_off;            // checkpoints [nck][5][nbp][N] (taped forward)
    int64_t tape_off;          // tape [steps][2 nbp + nxp + 1][N]: one segment, or all steps (backward)
    int64_t gr_off;            // raw parameter adjoints [kGradBlocks][16][16] + xbar0 adjoint [16]
    int64_t ga_off, gb_off;    // offsets into the packed dL/dA (sum nx^2) and dL/dB (sum nx nu)
};

// Raw adjoint blocks written by the backward kernel (16 x 16 each, padded):
// H_a (k < N-1), H_{N-1}, J, top rows of Abar, top rows of Bbar; then 16 more
// values for the adjoint of xbar_0.
constexpr int kGradBlocks = 5;
constexpr int kGradStride = kGradBlocks * 256 + 16;

// T matrix block of one instance (padded sizes NX, NU, NB = NX + NU).
// Time-invariant (tv = 0), row-major:
//   J [NU][NB] | Ha [NB][NB] | Hb [NB][NB] | A [NX][NX] | B [NX][NU] | e [NX] |
//   qbar [NB] | lb [NB] | ub [NB] | sx [NX + 1] | su [NU + 1]
// Time-varying (tv = 1), stage-minor ("SoA": element q of stage k at q*N + k):
//   J [NU*NB][N] | H [NB*NB][N] | A [NX*NX][N] | B [NX*NU][N] | e [NX][N] |
//   qbar [NB] | lb [NB] | ub [NB] | sx [NX + 1] | su [NU + 1]
// sx / su: parameters (a padded with zeros, then b or r) of non-box x / u sets.
__host__ __device__ inline int64_t mat_block_size(int32_t NX, int32_t NU, int32_t N, int32_t tv) {
    const int64_t NB = NX + NU;
    if (!tv) return NU * NB + 2 * NB * NB + NX * NX + NX * NU + NX + 4 * NB + 2;
    return (int64_t)N * (NU * NB + NB * NB + NX * NX + NX * NU + NX) + 4 * NB + 2;
}

// FP64 factorisation inputs of one instance (padded):
//   A [S][NX][NX] | B [S][NX][NU] | e [S][NX] | Q [NX][NX] | R [NU][NU] | Wdu [NU][NU]
// with S = tv ? N : 1 (Wdu = input-rate weight, zero when absent).
__host__ __device__ inline int64_t mat64_block_size(int32_t NX, int32_t NU, int32_t N, int32_t tv) {
    const int64_t S = tv ? N : 1;
    return S * (NX * NX + NX * NU + NX) + NX * NX + 2 * NU * NU;
}

// Offsets inside the blocks above.
struct MatOffsets {
    int64_t J, H, Hb, A, B, e, qbar, lb, ub, sx, su;  // T block (Hb unused when tv)
    int64_t A64, B64, e64, Q64, R64, W64;     // FP64 block
};

__host__ __device__ inline MatOffsets mat_offsets(int32_t NX, int32_t NU, int32_t N, int32_t tv) {
    const int64_t NB = NX + NU;
    MatOffsets o;
    if (!tv) {
        o.J = 0;
        o.H = o.J + NU * NB;
        o.Hb = o.H + NB * NB;
        o.A = o.Hb + NB * NB;
        o.B = o.A + NX * NX;
        o.e = o.B + NX * NU;
        o.qbar = o.e + NX;
    } else {
        o.J = 0;
        o.H = o.J + NU * NB * (int64_t)N;
        o.Hb = -1;
        o.A = o.H + NB * NB * (int64_t)N;
        o.B = o.A + NX * NX * (int64_t)N;
        o.e = o.B + NX * NU * (int64_t)N;
        o.qbar = o.e + NX * (int64_t)N;
    }
    o.lb = o.qbar + NB;
    o.ub = o.lb + NB;
    o.sx = o.ub + NB;
    o.su = o.sx + NX + 1;
    const int64_t S = tv ? N : 1;
    o.A64 = 0;
    o.B64 = o.A64 + S * NX * NX;
    o.e64 = o.B64 + S * NX * NU;
    o.Q64 = o.e64 + S * NX;
    o.R64 = o.Q64 + NX * NX;
    o.W64 = o.R64 + NU * NU;
    return o;
}

// One factorisation task: an H_k or J_k of one instance.
struct FactorTask {
    int32_t inst;
    int32_t kind;   // 0 = H with coupling to stage k+1, 1 = H of the last stage, 2 = J
    int32_t stage;  // stage index (time-varying) or 0
    int32_t pad;
};

// A bin of instances that share one 512-thread workgroup of the lane kernel;
// instance j occupies waves [wave0, wave0 + nwaves).
constexpr int kBinThreads = 512;
constexpr int kBinWaves = kBinThreads / 64;
struct BinEntry {
    int32_t inst;
    int16_t wave0;
    int16_t nwaves;
};
struct Bin {
    int32_t n;
    int32_t pad;
    BinEntry e[kBinWaves];
};

// Device-side result record; identical layout to pimpc_info.
struct InfoDev {
    int32_t iters;
    int32_t restarts;
    double c;
    double r_prim;
    double r_dual;
    int32_t status;
    int32_t pad;
};

// Compiled lane-family classes (padded nx, nu).  X(id, NX, NU).
// Time-invariant, both precisions.
#define PIMPC_LANE_CLASSES(X) \
    X(0, 2, 1)                \
    X(1, 2, 2)                \
    X(2, 4, 1)                \
    X(3, 4, 2)                \
    X(4, 4, 3)                \
    X(5, 4, 4)                \
    X(6, 8, 1)                \
    X(7, 8, 2)                \
    X(8, 8, 3)                \
    X(9, 8, 4)                \
    X(10, 12, 1)              \
    X(11, 12, 2)              \
    X(12, 12, 3)              \
    X(13, 12, 4)              \
    X(14, 16, 1)              \
    X(15, 16, 2)              \
    X(16, 16, 3)              \
    X(17, 16, 4)              \
    X(18, 8, 8)               \
    X(19, 16, 8)
constexpr int kLaneClasses = 20;

// Time-varying classes (stage matrices held in registers): X(id, NX, NU).
// Ids continue after the time-invariant ones.
#define PIMPC_LANE_TV_CLASSES(X) \
    X(20, 2, 1)                  \
    X(21, 2, 2)                  \
    X(22, 4, 1)                  \
    X(23, 4, 2)
constexpr int kLaneTvFirst = 20;
constexpr int kLaneAllClasses = 24;

}  // namespace pimpc
