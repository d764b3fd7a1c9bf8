// runtime.cpp -- host runtime and C ABI of the piMPC solver (include/pimpc.h).
//
// Owns validation, device memory layout, the FP64 stage factorisation
// launches, the batch schedule (bins of instances per class, LPT order), the
// per-class persistent ADMM launches forked over a few streams and joined
// back, hipGraph capture/replay of that launch sequence, and the conversion
// of iterates between the caller's packed layout and the device layout.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "pimpc.h"
#include "pimpc_dev.hpp"
#include "pimpc_lane.hpp"
#include "pimpc_row.hpp"
#include "pimpc_adjoint.hpp"

namespace pimpc {
template <typename T>
hipError_t launch_factor(const InstDev*, const FactorTask*, int, int, const double*, T*, double, int32_t*,
                         int32_t*, hipStream_t);
hipError_t launch_stage_import(const InstDev*, int, const int64_t*, const double*, const double*, const double*,
                               double*, int32_t*, hipStream_t);
hipError_t launch_bytes_store(void*, const void*, size_t, hipStream_t);
template <typename T>
hipError_t launch_expand(const InstDev*, int, const double*, T*, int, hipStream_t);
template <typename T>
hipError_t launch_params(const InstDev*, int, const T*, const T*, const T*, const T*, double*, hipStream_t);
template <typename T>
hipError_t launch_fill(T*, int64_t, T, hipStream_t);

}  // namespace pimpc

using namespace pimpc;

namespace {

thread_local std::string g_setup_err;

struct ClassDesc {
    int id, nx, nu, tv;
};
const ClassDesc kClassTable[] = {
#define PIMPC_CD(id, nx, nu) {id, nx, nu, 0},
    PIMPC_LANE_CLASSES(PIMPC_CD)
#undef PIMPC_CD
#define PIMPC_CD(id, nx, nu) {id, nx, nu, 1},
        PIMPC_LANE_TV_CLASSES(PIMPC_CD)
#undef PIMPC_CD
};

inline int64_t stage_fma(int nx, int nu) {
    const int64_t nb = nx + nu;
    return nb * nb + nu * nb + 2LL * nx * nx + 3LL * nx * nu;
}

hipError_t lane_dispatch_any(int fp64, int cls, int gs, bool rec, const LaneArgs* a, int bw, int grid,
                             hipStream_t s, int* occ) {
    bool handled = false;
    hipError_t e;
#define PIMPC_TRY(P)                                                            \
    e = lane_dispatch<P>(fp64, cls, gs, rec, a, bw, grid, s, occ, &handled);   \
    if (handled) return e;
    PIMPC_TRY(0)
    PIMPC_TRY(1)
    PIMPC_TRY(2)
    PIMPC_TRY(3)
    PIMPC_TRY(4)
    PIMPC_TRY(5)
#undef PIMPC_TRY
    return hipErrorInvalidValue;
}

size_t pin_align(size_t x) { return (x + 15) / 16 * 16; }

template <typename T>
T* dmalloc(size_t n, hipError_t* err) {
    T* p = nullptr;
    if (n == 0) n = 1;
    *err = hipMalloc((void**)&p, n * sizeof(T));
    return p;
}

}  // namespace

// ---------------------------------------------- scratch of the no-alloc solve
//
// pimpc_solve_batch_noalloc keeps every per-call buffer (kernel arguments,
// bin counters, row-family mailboxes and reduction words) in this array
// instead of memory the library allocates.  Each GPU holds its own copy, at
// its own address, from module load until the process ends.  Host code never
// passes `scratch` itself (on the host it only names the symbol): the device
// address is looked up once per device with hipGetSymbolAddress, at the first
// pimpc_setup on that device, and kept in g_scratch_dev.
static __device__ __align__(256) unsigned char scratch[PIMPC_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once).
hipError_t scratch_init(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (g_scratch_dev[dev]) return hipSuccess;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[dev] = ptr;
    return hipSuccess;
}

void* scratch_dev(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    return g_scratch_dev[dev];
}
}  // namespace

// One distinct argument set of the batched launch sequence (device copies
// of the per-class kernel arguments and, once captured, its graph).
struct LaunchSet {
    const void* x0 = nullptr;
    const void* up = nullptr;
    void* u0 = nullptr;
    void* info = nullptr;
    int warm = 0;
    int write_iters = 0;
    hipStream_t stream = nullptr;
    LaneArgs* d_args = nullptr;  // one per present lane class
    RowArgs* d_rargs = nullptr;  // one per row-family instance
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    uint64_t last_use = 0;  // for the least-recently-used eviction of the set cache
};

// Distinct argument sets (each with its device arguments and graph) a
// context keeps; the least recently used one is released beyond this.
constexpr size_t kMaxLaunchSets = 8;

struct ClassRun {
    int cls = 0;
    int nbmax = 0;
    int bw = kBinWaves;  // waves per bin (the launch's workgroup size / 64)
    int bin_first = 0;
    int nbins = 0;
    int occ = 1;
    int gs = 0;        // some instance of the class has a non-box constraint set
    int64_t cost = 0;  // sum over bins of waves * stage FMAs (for stream balancing)
};

struct pimpc_ctx_s {
    std::string err;
    int device = 0;  // the device current at pimpc_setup
    hipStream_t stream = nullptr;
    hipStream_t aux[3] = {nullptr, nullptr, nullptr};
    hipEvent_t ev_fork = nullptr;
    hipEvent_t ev_join[3] = {nullptr, nullptr, nullptr};
    pimpc_options opt{};
    int fp64 = 0;
    size_t tsize = 4;
    int count = 0;
    int tv = 0;
    int num_cus = 256;
    std::vector<InstDev> inst;
    int64_t mat_elems = 0, mat64_elems = 0, st_elems = 0, it_elems = 0, sum_nx = 0, sum_nu = 0;
    // device memory
    InstDev* d_inst = nullptr;
    void* d_mats = nullptr;
    double* d_mats64 = nullptr;
    // host copy of d_mats64, current unless device-side parameters replaced it
    std::vector<double> h_mats64;
    bool h_mats64_valid = false;
    // pinned staging of pimpc_solve: x0 | u_prev | u0 | info (16-byte aligned parts)
    char* h_pin = nullptr;
    void* d_state = nullptr;
    void* d_prev = nullptr;  // restart acceleration: the previous actual iterate (state layout)
    void* d_iters = nullptr;
    void* d_x0 = nullptr;
    void* d_up = nullptr;
    void* d_u0 = nullptr;
    InfoDev* d_info = nullptr;
    FactorTask* d_tasks = nullptr;
    int ntasks = 0;
    int nb_max = 1;  // widest padded stage (nx + nu) of the context: the factor kernel's LDS
    int32_t* d_bad = nullptr;       // per factorisation task: not SPD
    int32_t* d_ibad = nullptr;      // per instance: some stage matrix not SPD (read by the solve kernels)
    int32_t* d_nonfinite = nullptr; // device stage import saw NaN/Inf
    int64_t* d_pack_off = nullptr;  // per instance: offsets of A, B, e in the caller's packed arrays
    Bin* d_bins = nullptr;
    int32_t* d_counters = nullptr;
    std::vector<ClassRun> runs;
    std::vector<int> bin_waves;  // waves of each bin (host copy of the schedule, for the autotuner)
    std::vector<int> row_insts;  // instances handled by the row family
    void* d_row_clear = nullptr;   // per-solve scratch of the row-family instances (cleared every solve)
    void* d_row_fused = nullptr;   // fused stage data of the row-family instances
    std::vector<size_t> row_clear_off, row_fused_off;  // per row-family instance (bytes)
    size_t row_clear_total = 0;
    int schedule = 1;            // 1 = dynamic counter, 2 = static striding
    int nstreams = 1;
    int grid_div = 1;            // resident workgroups of a class launch: (occupancy x CUs) / grid_div
    int has_state = 0;
    std::vector<std::unique_ptr<LaunchSet>> sets;
    // differentiable path (ckpt_every > 0)
    void* d_ckpt = nullptr;
    float* d_tape = nullptr;
    float* d_grads = nullptr;
    Bin* d_bwd_bins = nullptr;
    int32_t* d_bwd_counters = nullptr;
    std::vector<ClassRun> bwd_runs;
    uint64_t tape_id = 0;    // id of the tape pimpc_backward may use (0: none)
    uint64_t tape_count = 0; // taped forwards so far (ids are 1, 2, ...)
    uint64_t set_clock = 0;  // launch-set use counter
    std::vector<LaneArgs> na_args;  // host staging of pimpc_solve_batch_noalloc's arguments
    std::vector<RowArgs> na_rargs;
    const void* tape_x0 = nullptr;
    const void* tape_up = nullptr;

    int fail(int32_t code, const char* fmt, ...) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof(buf), fmt, ap);
        va_end(ap);
        err = buf;
        return code;
    }
};

#define HIPCHK(ctx, expr)                                                                     \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return (ctx)->fail(PIMPC_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_));    \
    } while (0)

namespace {

bool finite_arr(const double* p, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

// Symmetric PSD test: symmetry to a relative tolerance, then a Cholesky of
// M + delta I with delta = 1e-12 (1 + max|M|).
bool sym_psd(const double* M, int n, bool* sym) {
    double mx = 0.0;
    for (int i = 0; i < n * n; ++i) mx = std::max(mx, std::fabs(M[i]));
    *sym = true;
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < i; ++j)
            if (std::fabs(M[i * n + j] - M[j * n + i]) > 1e-10 * (1.0 + mx)) *sym = false;
    if (!*sym) return false;
    std::vector<double> L(M, M + n * n);
    const double delta = 1e-12 * (1.0 + mx);
    for (int i = 0; i < n; ++i) L[i * n + i] += delta;
    for (int j = 0; j < n; ++j) {
        double d = L[j * n + j];
        for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
        if (!(d > 0.0)) return false;
        const double l = std::sqrt(d);
        L[j * n + j] = l;
        for (int i = j + 1; i < n; ++i) {
            double s = L[i * n + j];
            for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
            L[i * n + j] = s / l;
        }
    }
    return true;
}

int pick_class(int nx, int nu, int tv, size_t tsize) {
    int best = -1;
    int64_t best_cost = 0;
    for (const ClassDesc& c : kClassTable) {
        if (c.tv != tv || c.nx < nx || c.nu < nu) continue;
        if (!lane_class_fits(c.nx + c.nu, tsize)) continue;
        const int64_t cost = stage_fma(c.nx, c.nu);
        if (best < 0 || cost < best_cost) {
            best = c.id;
            best_cost = cost;
        }
    }
    return best;
}

const ClassDesc* class_desc(int id) {
    for (const ClassDesc& c : kClassTable)
        if (c.id == id) return &c;
    return nullptr;
}

}  // namespace

// --------------------------------------------------------------- data upload

// Build the padded FP64 block (A, B, e, Q, R, Wdu) of every instance from
// packed caller arrays; only the stage data (A, B, e) when `stage_only`.
static void build_mats64(pimpc_ctx ctx, const double* A, const double* B, const double* e,
                         const double* Q, const double* R, const double* Wdu, std::vector<double>& out,
                         bool stage_only) {
    if (!stage_only) out.assign(ctx->mat64_elems, 0.0);
    int64_t oa = 0, ob = 0, oe = 0, oq = 0, orr = 0;
    for (int i = 0; i < ctx->count; ++i) {
        const InstDev& I = ctx->inst[i];
        const int nx = I.nx, nu = I.nu, NX = I.nxp, NU = I.nup, N = I.N;
        const MatOffsets o = mat_offsets(NX, NU, N, I.tv);
        double* b = out.data() + I.mat64_off;
        const int S = I.tv ? N : 1;
        for (int k = 0; k < S; ++k) {
            for (int r = 0; r < NX; ++r) {
                for (int c = 0; c < NX; ++c)
                    b[o.A64 + (int64_t)k * NX * NX + r * NX + c] =
                        (r < nx && c < nx) ? A[oa + (int64_t)k * nx * nx + r * nx + c] : 0.0;
                for (int c = 0; c < NU; ++c)
                    b[o.B64 + (int64_t)k * NX * NU + r * NU + c] =
                        (r < nx && c < nu) ? B[ob + (int64_t)k * nx * nu + r * nu + c] : 0.0;
                b[o.e64 + (int64_t)k * NX + r] = (e && r < nx) ? e[oe + (int64_t)k * nx + r] : 0.0;
            }
        }
        oa += (int64_t)S * nx * nx;
        ob += (int64_t)S * nx * nu;
        oe += (int64_t)S * nx;
        if (!stage_only) {
            for (int r = 0; r < NX; ++r)
                for (int c = 0; c < NX; ++c)
                    b[o.Q64 + r * NX + c] = (r < nx && c < nx) ? Q[oq + r * nx + c] : (r == c ? 1.0 : 0.0);
            for (int r = 0; r < NU; ++r)
                for (int c = 0; c < NU; ++c)
                    b[o.R64 + r * NU + c] = (r < nu && c < nu) ? R[orr + r * nu + c] : (r == c ? 1.0 : 0.0);
            for (int r = 0; r < NU; ++r)
                for (int c = 0; c < NU; ++c)
                    b[o.W64 + r * NU + c] = (Wdu && r < nu && c < nu) ? Wdu[orr + r * nu + c] : 0.0;
            oq += (int64_t)nx * nx;
            orr += (int64_t)nu * nu;
        }
    }
}

template <typename T>
static int upload_t_block(pimpc_ctx ctx, const double* qbar, const double* xmin, const double* xmax,
                          const double* umin, const double* umax, const double* xpar, const double* upar) {
    std::vector<T> h(ctx->mat_elems, T(0));
    int64_t ox = 0, ou = 0;
    for (int i = 0; i < ctx->count; ++i) {
        const InstDev& I = ctx->inst[i];
        const int nx = I.nx, nu = I.nu, NX = I.nxp, NU = I.nup, NB = I.nbp;
        const MatOffsets o = mat_offsets(NX, NU, I.N, I.tv);
        T* b = h.data() + I.mat_off;
        for (int r = 0; r < NB; ++r) {
            const bool isx = r < NX;
            const int rr = isx ? r : r - NX;
            const bool real = isx ? rr < nx : rr < nu;
            double q = 0.0, lo = 0.0, hi = 0.0;  // padded rows: [0, 0] box, zero linear term
            if (real) {
                lo = isx ? xmin[ox + rr] : umin[ou + rr];
                hi = isx ? xmax[ox + rr] : umax[ou + rr];
                if ((isx ? I.xset : I.uset) != PIMPC_SET_BOX) {  // the set's own projection applies
                    lo = -INFINITY;
                    hi = INFINITY;
                }
            }
            b[o.lb + r] = (T)lo;
            b[o.ub + r] = (T)hi;
            b[o.qbar + r] = (T)q;
        }
        // non-box set parameters: (a, b) or (., r), a padded with zeros
        if (I.xset != PIMPC_SET_BOX && xpar) {
            for (int r = 0; r < nx; ++r) b[o.sx + r] = (T)xpar[ox + i + r];
            b[o.sx + NX] = (T)xpar[ox + i + nx];
        }
        if (I.uset != PIMPC_SET_BOX && upar) {
            for (int r = 0; r < nu; ++r) b[o.su + r] = (T)upar[ou + i + r];
            b[o.su + NU] = (T)upar[ou + i + nu];
        }
        if (qbar) {
            const int64_t qo = ox + ou;  // qbar packed as (nx + nu) per instance
            for (int r = 0; r < nx; ++r) b[o.qbar + r] = (T)qbar[qo + r];
            for (int r = 0; r < nu; ++r) b[o.qbar + NX + r] = (T)qbar[qo + nx + r];
        }
        ox += nx;
        ou += nu;
    }
    HIPCHK(ctx, hipMemcpy(ctx->d_mats, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    return PIMPC_OK;
}

// Fused stage data of the row-family instances (once their scratch exists).
static hipError_t fuse_rows(pimpc_ctx ctx, hipStream_t s) {
    if (!ctx->d_row_fused) return hipSuccess;
    for (size_t j = 0; j < ctx->row_insts.size(); ++j) {
        const int i = ctx->row_insts[j];
        hipError_t e = launch_row_fuse(ctx->d_inst, i, ctx->inst[i], ctx->d_mats,
                                       (char*)ctx->d_row_fused + ctx->row_fused_off[j], s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Expand the FP64 stage data into the T layout, factor, check the SPD flags.
static int refactor(pimpc_ctx ctx, bool sync_check) {
    hipStream_t s = ctx->stream;
    HIPCHK(ctx, launch_fill<int32_t>(ctx->d_bad, std::max(ctx->ntasks, 1), 0, s));
    HIPCHK(ctx, launch_fill<int32_t>(ctx->d_ibad, ctx->count, 0, s));
    if (ctx->fp64) {
        HIPCHK(ctx, launch_expand<double>(ctx->d_inst, ctx->count, ctx->d_mats64, (double*)ctx->d_mats, ctx->tv, s));
        HIPCHK(ctx, launch_factor<double>(ctx->d_inst, ctx->d_tasks, ctx->ntasks, ctx->nb_max, ctx->d_mats64,
                                          (double*)ctx->d_mats, ctx->opt.rho, ctx->d_bad, ctx->d_ibad, s));
    } else {
        HIPCHK(ctx, launch_expand<float>(ctx->d_inst, ctx->count, ctx->d_mats64, (float*)ctx->d_mats, ctx->tv, s));
        HIPCHK(ctx, launch_factor<float>(ctx->d_inst, ctx->d_tasks, ctx->ntasks, ctx->nb_max, ctx->d_mats64,
                                         (float*)ctx->d_mats, ctx->opt.rho, ctx->d_bad, ctx->d_ibad, s));
    }
    HIPCHK(ctx, fuse_rows(ctx, s));
    if (sync_check) {
        std::vector<int32_t> bad(std::max(ctx->ntasks, 1));
        HIPCHK(ctx, hipMemcpyAsync(bad.data(), ctx->d_bad, bad.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        for (int t = 0; t < ctx->ntasks; ++t)
            if (bad[t]) return ctx->fail(PIMPC_E_NOT_PSD, "stage matrix of factorisation task %d is not SPD", t);
    }
    return PIMPC_OK;
}

// ------------------------------------------------------------ batch schedule

// Bins of at most cap_waves waves; with fp64_narrow, FP64 classes whose
// horizons all fit four waves get bins of four (256-thread workgroups, one
// wave per SIMD with the whole register file).
static void build_bins(pimpc_ctx ctx, std::vector<Bin>& bins, std::vector<ClassRun>& runs, int cap_waves,
                       bool fp64_narrow) {
    bins.clear();
    runs.clear();
    for (const ClassDesc& cd : kClassTable) {
        std::vector<int> members;
        for (int i = 0; i < ctx->count; ++i)
            if (ctx->inst[i].cls == cd.id) members.push_back(i);
        if (members.empty()) continue;
        std::sort(members.begin(), members.end(), [&](int a, int b) {
            if (ctx->inst[a].N != ctx->inst[b].N) return ctx->inst[a].N > ctx->inst[b].N;
            return a < b;
        });
        const int cap = (fp64_narrow && ctx->inst[members[0]].N <= 4 * 64) ? 4 : cap_waves;
        // first-fit decreasing on waves
        std::vector<Bin> cb;
        std::vector<int> used;
        for (int i : members) {
            const int w = (ctx->inst[i].N + 63) / 64;
            int tgt = -1;
            for (size_t b = 0; b < cb.size(); ++b)
                if (used[b] + w <= cap && cb[b].n < cap) {
                    tgt = (int)b;
                    break;
                }
            if (tgt < 0) {
                Bin nb{};
                cb.push_back(nb);
                used.push_back(0);
                tgt = (int)cb.size() - 1;
            }
            Bin& bb = cb[tgt];
            bb.e[bb.n].inst = i;
            bb.e[bb.n].wave0 = (int16_t)used[tgt];
            bb.e[bb.n].nwaves = (int16_t)w;
            bb.n++;
            used[tgt] += w;
        }
        // largest bins first (LPT order for the claiming counter)
        std::vector<int> order(cb.size());
        for (size_t b = 0; b < cb.size(); ++b) order[b] = (int)b;
        std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return used[a] > used[b]; });
        ClassRun run;
        run.cls = cd.id;
        for (int i : members)
            if (ctx->inst[i].xset != 0 || ctx->inst[i].uset != 0) run.gs = 1;
        run.nbmax = cd.nx + cd.nu;
        run.bw = cap;
        run.bin_first = (int)bins.size();
        run.nbins = (int)cb.size();
        int64_t waves = 0;
        for (int b : order) {
            bins.push_back(cb[b]);
            waves += used[b];
        }
        run.cost = waves * stage_fma(cd.nx, cd.nu);
        runs.push_back(run);
    }
}

// Whether the lane kernels record every step for the backward (a taped
// forward with ckpt_every = 1) rather than checkpoints.
static bool rec_steps(pimpc_ctx ctx) { return ctx->opt.ckpt_every == 1; }

// Grid size of a class launch under the current schedule.
static int class_grid(pimpc_ctx ctx, const ClassRun& r) {
    if (ctx->schedule == 3) return r.nbins;  // one workgroup per bin, hardware dispatch order
    const int cap = std::max(1, r.occ * ctx->num_cus / std::max(1, ctx->grid_div));
    return std::max(1, std::min(r.nbins, cap));
}

// Where the per-solve scratch of a launch lives: the bin counters of the lane
// classes and the per-solve part of every row-family instance's scratch.
struct SolveScratch {
    int32_t* counters;
    char* row_clear;  // row-family instance j at row_clear + ctx->row_clear_off[j]
};

static SolveScratch ctx_scratch(pimpc_ctx ctx) { return {ctx->d_counters, (char*)ctx->d_row_clear}; }

// Kernel arguments of one batched solve (host copies).
static void build_args(pimpc_ctx ctx, const void* x0, const void* up, void* u0, void* info, int warm,
                       int write_iters, const SolveScratch& sc, std::vector<LaneArgs>& args,
                       std::vector<RowArgs>& rargs) {
    args.assign(ctx->runs.size(), LaneArgs{});
    for (size_t c = 0; c < ctx->runs.size(); ++c) {
        const ClassRun& r = ctx->runs[c];
        LaneArgs& a = args[c];
        memset(&a, 0, sizeof(a));
        a.inst = ctx->d_inst;
        a.bins = ctx->d_bins + r.bin_first;
        a.nbins = r.nbins;
        a.bin_counter = (ctx->schedule == 1) ? sc.counters + c : nullptr;
        a.mats = ctx->d_mats;
        a.state = ctx->d_state;
        a.iters_out = ctx->d_iters;
        a.x0 = x0;
        a.uprev = up;
        a.u0 = u0;
        a.info = (InfoDev*)info;
        a.rho = ctx->opt.rho;
        a.eps = ctx->opt.eps;
        a.K = ctx->opt.max_iter;
        a.check_every = ctx->opt.check_every;
        a.warm = warm;
        a.nbmax = r.nbmax;
        a.write_iters = write_iters;
        a.ckpt_every = rec_steps(ctx) ? 0 : ctx->opt.ckpt_every;
        a.ckpt = ctx->d_ckpt;
        a.tape = rec_steps(ctx) ? ctx->d_tape : nullptr;
        a.accel = ctx->opt.accel;
        a.eta = ctx->opt.eta;
        a.prev = ctx->d_prev;
        a.fbad = ctx->d_ibad;
    }
    rargs.assign(ctx->row_insts.size(), RowArgs{});
    for (size_t j = 0; j < ctx->row_insts.size(); ++j) {
        RowArgs& a = rargs[j];
        memset(&a, 0, sizeof(a));
        a.inst = ctx->d_inst;
        a.inst_idx = ctx->row_insts[j];
        a.mats = ctx->d_mats;
        a.state = ctx->d_state;
        a.iters_out = ctx->d_iters;
        a.x0 = x0;
        a.uprev = up;
        a.u0 = u0;
        a.info = (InfoDev*)info;
        a.rho = ctx->opt.rho;
        a.eps = ctx->opt.eps;
        a.K = ctx->opt.max_iter;
        a.check_every = ctx->opt.check_every;
        a.warm = warm;
        a.write_iters = write_iters;
        a.scratch = sc.row_clear + ctx->row_clear_off[j];
        a.fused = (const char*)ctx->d_row_fused + ctx->row_fused_off[j];
        a.fbad = ctx->d_ibad;
        a.eta = ctx->opt.eta;
        a.accel = ctx->opt.accel;
    }
}

static int fill_set_args(pimpc_ctx ctx, LaunchSet* ls) {
    std::vector<LaneArgs> args;
    std::vector<RowArgs> rargs;
    build_args(ctx, ls->x0, ls->up, ls->u0, ls->info, ls->warm, ls->write_iters, ctx_scratch(ctx), args, rargs);
    if (!args.empty())
        HIPCHK(ctx, hipMemcpy(ls->d_args, args.data(), args.size() * sizeof(LaneArgs), hipMemcpyHostToDevice));
    if (!rargs.empty())
        HIPCHK(ctx, hipMemcpy(ls->d_rargs, rargs.data(), rargs.size() * sizeof(RowArgs), hipMemcpyHostToDevice));
    return PIMPC_OK;
}

static void release_set(LaunchSet* ls) {
    // a graph launch of this set may still run on its stream
    if (ls->stream) (void)hipStreamSynchronize(ls->stream);
    else (void)hipDeviceSynchronize();
    if (ls->exec) (void)hipGraphExecDestroy(ls->exec);
    if (ls->graph) (void)hipGraphDestroy(ls->graph);
    if (ls->d_args) (void)hipFree(ls->d_args);
    if (ls->d_rargs) (void)hipFree(ls->d_rargs);
    ls->exec = nullptr;
    ls->graph = nullptr;
    ls->d_args = nullptr;
    ls->d_rargs = nullptr;
}

static LaunchSet* get_set(pimpc_ctx ctx, const void* x0, const void* up, void* u0, void* info, int warm,
                          int write_iters, hipStream_t s, int* rc) {
    for (auto& p : ctx->sets) {
        LaunchSet* ls = p.get();
        if (ls->x0 == x0 && ls->up == up && ls->u0 == u0 && ls->info == info && ls->warm == warm &&
            ls->write_iters == write_iters && ls->stream == s) {
            ls->last_use = ++ctx->set_clock;
            return ls;
        }
    }
    if (ctx->sets.size() >= kMaxLaunchSets) {  // release the least recently used set
        size_t lru = 0;
        for (size_t j = 1; j < ctx->sets.size(); ++j)
            if (ctx->sets[j]->last_use < ctx->sets[lru]->last_use) lru = j;
        release_set(ctx->sets[lru].get());
        ctx->sets.erase(ctx->sets.begin() + lru);
    }
    auto ls = std::make_unique<LaunchSet>();
    ls->last_use = ++ctx->set_clock;
    ls->x0 = x0;
    ls->up = up;
    ls->u0 = u0;
    ls->info = info;
    ls->warm = warm;
    ls->write_iters = write_iters;
    ls->stream = s;
    hipError_t e = hipSuccess;
    ls->d_args = dmalloc<LaneArgs>(std::max<size_t>(ctx->runs.size(), 1), &e);
    if (e != hipSuccess) {
        *rc = ctx->fail(PIMPC_E_NOMEM, "hipMalloc of launch arguments failed");
        return nullptr;
    }
    ls->d_rargs = dmalloc<RowArgs>(std::max<size_t>(ctx->row_insts.size(), 1), &e);
    if (e != hipSuccess) {
        *rc = ctx->fail(PIMPC_E_NOMEM, "hipMalloc of launch arguments failed");
        return nullptr;
    }
    *rc = fill_set_args(ctx, ls.get());
    if (*rc != PIMPC_OK) return nullptr;
    ctx->sets.push_back(std::move(ls));
    return ctx->sets.back().get();
}

static void free_set_graphs(pimpc_ctx ctx) {
    for (auto& p : ctx->sets) {
        if (p->exec) (void)hipGraphExecDestroy(p->exec);
        if (p->graph) (void)hipGraphDestroy(p->graph);
        p->exec = nullptr;
        p->graph = nullptr;
    }
}

// Enqueue the whole batched ADMM launch sequence on `s`, with the kernel
// arguments at d_args / d_rargs (device) and the per-solve scratch `sc`.
static int enqueue_launches(pimpc_ctx ctx, const LaneArgs* d_args, const RowArgs* d_rargs, const SolveScratch& sc,
                            hipStream_t s) {
    const int ncls = (int)ctx->runs.size();
    if (ctx->schedule == 1 && ncls > 0) HIPCHK(ctx, launch_fill<int32_t>(sc.counters, ncls, 0, s));
    // A row-family kernel needs every workgroup of its grid resident at once
    // (its halo waits cross workgroups).  Beside another row kernel each
    // could hold part of the GPU and wait for the rest; beside a long lane
    // batch its resident workgroups could wait longer than their bounded
    // polls allow.  So the row-family instances run first, one after the
    // other on the first stream, and the lane classes start after them.
    for (size_t rj = 0; rj < ctx->row_insts.size(); ++rj)
        HIPCHK(ctx, launch_row(ctx->fp64, d_rargs + rj, ctx->inst[ctx->row_insts[rj]],
                               sc.row_clear + ctx->row_clear_off[rj], s));
    const int ns = std::min(ctx->nstreams, std::max(1, ncls));
    if (ns > 1) {
        HIPCHK(ctx, hipEventRecord(ctx->ev_fork, s));
        for (int j = 0; j < ns - 1; ++j) HIPCHK(ctx, hipStreamWaitEvent(ctx->aux[j], ctx->ev_fork, 0));
    }
    // the lane classes, whose workgroups never wait on each other: LPT over
    // the streams by class cost
    std::vector<int> order(ncls);
    for (int c = 0; c < ncls; ++c) order[c] = c;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return ctx->runs[a].cost > ctx->runs[b].cost; });
    std::vector<int64_t> load(ns, 0);
    auto stream_of = [&](int j) { return j == 0 ? s : ctx->aux[j - 1]; };
    for (int c : order) {
        const ClassRun& r = ctx->runs[c];
        const int j = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[j] += r.cost;
        HIPCHK(ctx, lane_dispatch_any(ctx->fp64, r.cls, r.gs, rec_steps(ctx), d_args + c, r.bw, class_grid(ctx, r),
                                      stream_of(j), nullptr));
    }
    if (ns > 1) {
        for (int j = 0; j < ns - 1; ++j) {
            HIPCHK(ctx, hipEventRecord(ctx->ev_join[j], ctx->aux[j]));
            HIPCHK(ctx, hipStreamWaitEvent(s, ctx->ev_join[j], 0));
        }
    }
    return PIMPC_OK;
}

static int enqueue_solve(pimpc_ctx ctx, LaunchSet* ls, hipStream_t s) {
    return enqueue_launches(ctx, ls->d_args, ls->d_rargs, ctx_scratch(ctx), s);
}

static int run_set(pimpc_ctx ctx, LaunchSet* ls, hipStream_t s, bool graph) {
    // The legacy default stream cannot be captured: launch directly there.
    if (!graph || s == nullptr) return enqueue_solve(ctx, ls, s);
    if (!ls->exec) {
        HIPCHK(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
        int rc = enqueue_solve(ctx, ls, s);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(s, &g);
        if (rc != PIMPC_OK) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return ctx->fail(PIMPC_E_HIP, "graph capture failed: %s", hipGetErrorString(e));
        ls->graph = g;
        HIPCHK(ctx, hipGraphInstantiate(&ls->exec, g, nullptr, nullptr, 0));
    }
    HIPCHK(ctx, hipGraphLaunch(ls->exec, s));
    return PIMPC_OK;
}

// Each class launch split in two, at the bin where the waves of its
// (largest-first) bins reach half of the class's: twice as many, smaller
// launches for the streams to balance.  Costs split in proportion.
static std::vector<ClassRun> split_runs(pimpc_ctx ctx, const std::vector<ClassRun>& base) {
    std::vector<ClassRun> out;
    for (const ClassRun& r : base) {
        if (r.nbins < 2) {
            out.push_back(r);
            continue;
        }
        int64_t total = 0;
        for (int b = 0; b < r.nbins; ++b) total += ctx->bin_waves[r.bin_first + b];
        int64_t acc = 0;
        int cut = 1;
        for (int b = 0; b < r.nbins - 1; ++b) {
            acc += ctx->bin_waves[r.bin_first + b];
            cut = b + 1;
            if (2 * acc >= total) break;
        }
        int64_t w0 = 0;
        for (int b = 0; b < cut; ++b) w0 += ctx->bin_waves[r.bin_first + b];
        ClassRun a = r, c = r;
        a.nbins = cut;
        c.bin_first = r.bin_first + cut;
        c.nbins = r.nbins - cut;
        a.cost = std::max<int64_t>(1, r.cost * w0 / std::max<int64_t>(total, 1));
        c.cost = std::max<int64_t>(1, r.cost - a.cost);
        out.push_back(a);
        out.push_back(c);
    }
    return out;
}

// Time one enqueued solve (or one class alone) on the context's stream.
static int time_launch(pimpc_ctx ctx, LaunchSet* ls, int only_class, hipEvent_t t0, hipEvent_t t1, float* ms) {
    HIPCHK(ctx, hipEventRecord(t0, ctx->stream));
    if (only_class < 0) {
        const int rc = enqueue_solve(ctx, ls, ctx->stream);
        if (rc != PIMPC_OK) return rc;
    } else {
        const ClassRun& r = ctx->runs[only_class];
        if (ctx->schedule == 1) HIPCHK(ctx, launch_fill<int32_t>(ctx->d_counters + only_class, 1, 0, ctx->stream));
        HIPCHK(ctx, lane_dispatch_any(ctx->fp64, r.cls, r.gs, rec_steps(ctx), ls->d_args + only_class, r.bw,
                                      class_grid(ctx, r),
                                      ctx->stream, nullptr));
    }
    HIPCHK(ctx, hipEventRecord(t1, ctx->stream));
    HIPCHK(ctx, hipEventSynchronize(t1));
    HIPCHK(ctx, hipEventElapsedTime(ms, t0, t1));
    return PIMPC_OK;
}

// The batch schedule, picked by measurement on the real batch at setup:
//   1. each class launch is timed alone; its measured time is the
//      alternative to the FMA-count estimate as its cost in the
//      longest-processing-time assignment of class launches to streams (the
//      classes' throughputs differ: narrow stages use the lanes less well);
//   2. candidates -- bin claiming (atomic counter, static striding, one
//      workgroup per bin), 1 to 4 streams, class launches whole or split in
//      two, FMA-count or measured costs, grids of all resident workgroups or
//      of a half or a quarter of them -- are each timed once on the full
//      batch; the fastest is kept.
static int autotune(pimpc_ctx ctx) {
    struct Cand {
        int schedule, nstreams, split, measured, grid_div;
    };
    const Cand cands[] = {{1, 4, 0, 0, 1}, {1, 1, 0, 0, 1}, {2, 4, 0, 0, 1}, {3, 4, 0, 0, 1},
                          {1, 4, 1, 1, 1}, {1, 3, 1, 1, 1}, {1, 2, 1, 1, 1}, {3, 4, 1, 1, 1},
                          {1, 4, 0, 1, 1}, {3, 4, 0, 1, 1}, {1, 4, 0, 0, 2}, {1, 4, 0, 0, 4},
                          {2, 4, 0, 0, 2}, {1, 4, 0, 1, 2}};
    const int ncand = (int)(sizeof(cands) / sizeof(cands[0]));
    const std::vector<ClassRun> base = ctx->runs;
    if (ctx->opt.schedule > 0) {  // a fixed candidate; split launches take their costs from the FMA model
        const Cand& c = cands[(ctx->opt.schedule - 1) % ncand];
        ctx->schedule = c.schedule;
        ctx->nstreams = c.nstreams;
        ctx->grid_div = c.grid_div;
        if (c.split) ctx->runs = split_runs(ctx, base);
        return PIMPC_OK;
    }
    int64_t total_waves = 0;
    for (const InstDev& I : ctx->inst) total_waves += (I.N + 63) / 64;
    if (ctx->count == 1 || total_waves <= 64 || base.empty()) {  // nothing to balance
        ctx->schedule = 2;
        ctx->nstreams = 1;
        return PIMPC_OK;
    }
    hipError_t e = hipSuccess;
    hipEvent_t t0, t1;
    HIPCHK(ctx, hipEventCreate(&t0));
    HIPCHK(ctx, hipEventCreate(&t1));
    auto make_set = [&](LaunchSet& ls) -> int {
        ls.x0 = ctx->d_x0;
        ls.up = ctx->d_up;
        ls.u0 = ctx->d_u0;
        ls.info = ctx->d_info;
        ls.d_args = dmalloc<LaneArgs>(std::max<size_t>(ctx->runs.size(), 1), &e);
        ls.d_rargs = dmalloc<RowArgs>(std::max<size_t>(ctx->row_insts.size(), 1), &e);
        if (e != hipSuccess) return ctx->fail(PIMPC_E_NOMEM, "hipMalloc failed in autotune");
        return fill_set_args(ctx, &ls);
    };
    auto free_set = [&](LaunchSet& ls) {
        (void)hipFree(ls.d_args);
        (void)hipFree(ls.d_rargs);
    };
    // 1. measured class costs (after one warm-up solve)
    {
        ctx->schedule = 1;
        ctx->nstreams = 4;
        ctx->grid_div = 1;
        LaunchSet ls;
        int rc = make_set(ls);
        float ms = 0.f;
        if (rc == PIMPC_OK) rc = time_launch(ctx, &ls, -1, t0, t1, &ms);
        for (size_t c = 0; c < ctx->runs.size() && rc == PIMPC_OK; ++c) {
            rc = time_launch(ctx, &ls, (int)c, t0, t1, &ms);
            ctx->runs[c].cost = std::max<int64_t>(1, (int64_t)(ms * 1e6f));  // ns
        }
        free_set(ls);
        if (rc != PIMPC_OK) return rc;
    }
    const std::vector<ClassRun> measured = ctx->runs;
    const std::vector<ClassRun> halves = split_runs(ctx, measured);
    const std::vector<ClassRun> base_halves = split_runs(ctx, base);
    auto runs_of = [&](const Cand& c) -> const std::vector<ClassRun>& {
        return c.split ? (c.measured ? halves : base_halves) : (c.measured ? measured : base);
    };
    // 2. candidates on the full batch
    float best = 1e30f;
    Cand bestc = cands[0];
    for (const Cand& c : cands) {
        ctx->schedule = c.schedule;
        ctx->nstreams = c.nstreams;
        ctx->grid_div = c.grid_div;
        ctx->runs = runs_of(c);
        LaunchSet ls;
        int rc = make_set(ls);
        float ms = 0.f;
        if (rc == PIMPC_OK) rc = time_launch(ctx, &ls, -1, t0, t1, &ms);  // warm-up
        if (rc == PIMPC_OK) rc = time_launch(ctx, &ls, -1, t0, t1, &ms);
        free_set(ls);
        if (rc != PIMPC_OK) return rc;
        if (ms < best) {
            best = ms;
            bestc = c;
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    ctx->schedule = bestc.schedule;
    ctx->nstreams = bestc.nstreams;
    ctx->grid_div = bestc.grid_div;
    ctx->runs = runs_of(bestc);
    return PIMPC_OK;
}

template <typename T>
static void to_t(const double* src, int64_t n, std::vector<char>& buf) {
    buf.resize(std::max<int64_t>(n, 1) * sizeof(T));
    T* d = (T*)buf.data();
    for (int64_t i = 0; i < n; ++i) d[i] = (T)src[i];
}

// ------------------------------------------------------------------ C ABI

extern "C" {

void pimpc_default_options(pimpc_options* o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->rho = 1.0;
    o->max_iter = 200;
    o->eps = 0.0;
    o->check_every = 1;
    o->precision = PIMPC_FP32;
    o->accel = 0;
    o->eta = 0.999;
    o->warm_start = 0;
    o->ckpt_every = 0;
    o->schedule = 0;
    o->family = PIMPC_FAMILY_AUTO;
}

int32_t pimpc_version(void) { return PIMPC_VERSION; }

const char* pimpc_last_error(pimpc_ctx ctx) {
    if (!ctx) return g_setup_err.c_str();
    return ctx->err.c_str();
}

static void destroy_ctx(pimpc_ctx ctx) {
    if (!ctx) return;
    // Only release what was created: a context that failed host validation
    // never touched the HIP runtime and must not start it here.
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    free_set_graphs(ctx);
    auto rel = [](void* p) {
        if (p) (void)hipFree(p);
    };
    for (auto& p : ctx->sets) {
        rel(p->d_args);
        rel(p->d_rargs);
    }
    rel(ctx->d_inst);
    rel(ctx->d_mats);
    rel(ctx->d_mats64);
    rel(ctx->d_state);
    rel(ctx->d_prev);
    rel(ctx->d_iters);
    rel(ctx->d_x0);
    rel(ctx->d_up);
    rel(ctx->d_u0);
    rel(ctx->d_info);
    rel(ctx->d_tasks);
    rel(ctx->d_bad);
    rel(ctx->d_bins);
    rel(ctx->d_counters);
    rel(ctx->d_row_clear);
    rel(ctx->d_row_fused);
    rel(ctx->d_ibad);
    rel(ctx->d_nonfinite);
    rel(ctx->d_pack_off);
    rel(ctx->d_ckpt);
    rel(ctx->d_tape);
    rel(ctx->d_grads);
    if (ctx->h_pin) (void)hipHostFree(ctx->h_pin);
    rel(ctx->d_bwd_bins);
    rel(ctx->d_bwd_counters);
    for (int j = 0; j < 3; ++j) {
        if (ctx->aux[j]) (void)hipStreamDestroy(ctx->aux[j]);
        if (ctx->ev_join[j]) (void)hipEventDestroy(ctx->ev_join[j]);
    }
    if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
    delete ctx;
}

void pimpc_destroy(pimpc_ctx ctx) { destroy_ctx(ctx); }

static int setup_impl(pimpc_ctx ctx, const pimpc_problem* p, const pimpc_options* o) {
    // ---------------- validation (host only, before any HIP call)
    if (!p || !o) return ctx->fail(PIMPC_E_ARG, "problem and options are required");
    if (p->count < 1) return ctx->fail(PIMPC_E_ARG, "count must be >= 1");
    if (p->count > 65535)  // the setup kernels give each instance one row of their grid
        return ctx->fail(PIMPC_E_DIM, "count must be <= 65535 (got %d)", p->count);
    if (!p->nx || !p->nu || !p->N || !p->A || !p->B || !p->Q || !p->R || !p->xmin || !p->xmax || !p->umin ||
        !p->umax)
        return ctx->fail(PIMPC_E_ARG, "a required problem array is NULL");
    if (p->time_varying != 0 && p->time_varying != 1) return ctx->fail(PIMPC_E_ARG, "time_varying must be 0 or 1");
    if (!(o->rho > 0.0) || !std::isfinite(o->rho)) return ctx->fail(PIMPC_E_ARG, "rho must be finite and > 0");
    if (o->max_iter < 1) return ctx->fail(PIMPC_E_ARG, "max_iter must be >= 1");
    if (o->check_every < 1) return ctx->fail(PIMPC_E_ARG, "check_every must be >= 1");
    if (std::isnan(o->eps)) return ctx->fail(PIMPC_E_ARG, "eps is NaN");
    if (o->precision != PIMPC_FP32 && o->precision != PIMPC_FP64)
        return ctx->fail(PIMPC_E_ARG, "precision must be PIMPC_FP32 or PIMPC_FP64");
    if (o->accel != 0 && o->accel != 1) return ctx->fail(PIMPC_E_ARG, "accel must be 0 or 1");
    if (o->accel == 1 && !(o->eta > 0.0 && o->eta <= 1.0)) return ctx->fail(PIMPC_E_ARG, "eta must be in (0, 1]");
    if (o->accel == 1 && o->ckpt_every > 0)
        return ctx->fail(PIMPC_E_UNSUPPORTED, "the taped forward differentiates plain ADMM (accel = 0)");
    if (o->warm_start != 0 && o->warm_start != 1) return ctx->fail(PIMPC_E_ARG, "warm_start must be 0 or 1");
    if (o->ckpt_every < 0) return ctx->fail(PIMPC_E_ARG, "ckpt_every must be >= 0");
    if (o->ckpt_every > 0 && o->eps > 0.0)
        return ctx->fail(PIMPC_E_UNSUPPORTED, "the taped forward runs exactly max_iter iterations (eps <= 0)");
    if (o->schedule < 0) return ctx->fail(PIMPC_E_ARG, "schedule must be >= 0");
    if (o->family < PIMPC_FAMILY_AUTO || o->family > PIMPC_FAMILY_ROW)
        return ctx->fail(PIMPC_E_ARG, "family must be PIMPC_FAMILY_AUTO, _LANE or _ROW");
    const int count = p->count;
    const int tv = p->time_varying;
    int64_t sA = 0, sB = 0, se = 0, sQ = 0, sR = 0, snx = 0, snu = 0;
    for (int i = 0; i < count; ++i) {
        const int nx = p->nx[i], nu = p->nu[i], N = p->N[i];
        if (nx < 1 || nu < 1 || N < 1) return ctx->fail(PIMPC_E_DIM, "instance %d: nx, nu, N must be >= 1", i);
        if (nx > 48 || nu > 16 || nx + nu > 64)
            return ctx->fail(PIMPC_E_DIM, "instance %d: nx <= 48, nu <= 16, nx + nu <= 64 supported", i);
        if (N > (1 << 20)) return ctx->fail(PIMPC_E_DIM, "instance %d: N too large", i);
        const int64_t S = tv ? N : 1;
        sA += S * nx * nx;
        sB += S * nx * nu;
        se += S * nx;
        sQ += (int64_t)nx * nx;
        sR += (int64_t)nu * nu;
        snx += nx;
        snu += nu;
    }
    if (!finite_arr(p->A, sA) || !finite_arr(p->B, sB) || (p->e && !finite_arr(p->e, se)) ||
        !finite_arr(p->Q, sQ) || !finite_arr(p->R, sR) || (p->qbar && !finite_arr(p->qbar, snx + snu)) ||
        (p->Wdu && !finite_arr(p->Wdu, sR)))
        return ctx->fail(PIMPC_E_NONFINITE, "problem data contains NaN or Inf");
    for (int64_t j = 0; j < snx; ++j)
        if (std::isnan(p->xmin[j]) || std::isnan(p->xmax[j]) || p->xmin[j] > p->xmax[j])
            return ctx->fail(PIMPC_E_ARG, "state bound %lld: need xmin <= xmax (no NaN)", (long long)j);
    for (int64_t j = 0; j < snu; ++j)
        if (std::isnan(p->umin[j]) || std::isnan(p->umax[j]) || p->umin[j] > p->umax[j])
            return ctx->fail(PIMPC_E_ARG, "input bound %lld: need umin <= umax (no NaN)", (long long)j);
    {
        int64_t oq = 0, orr = 0;
        for (int i = 0; i < count; ++i) {
            bool sym = true;
            if (!sym_psd(p->Q + oq, p->nx[i], &sym))
                return ctx->fail(PIMPC_E_NOT_PSD, "instance %d: Q is not %s", i, sym ? "PSD" : "symmetric");
            if (!sym_psd(p->R + orr, p->nu[i], &sym))
                return ctx->fail(PIMPC_E_NOT_PSD, "instance %d: R is not %s", i, sym ? "PSD" : "symmetric");
            if (p->Wdu && !sym_psd(p->Wdu + orr, p->nu[i], &sym))
                return ctx->fail(PIMPC_E_NOT_PSD, "instance %d: Wdu is not %s", i, sym ? "PSD" : "symmetric");
            oq += (int64_t)p->nx[i] * p->nx[i];
            orr += (int64_t)p->nu[i] * p->nu[i];
        }
    }
    {  // constraint sets of the x and u factors
        int64_t ox = 0, ou = 0;
        for (int i = 0; i < count; ++i) {
            for (int side = 0; side < 2; ++side) {
                const int kind = side == 0 ? (p->xset ? p->xset[i] : 0) : (p->uset ? p->uset[i] : 0);
                const int n = side == 0 ? p->nx[i] : p->nu[i];
                const double* par = side == 0 ? (p->xset_par ? p->xset_par + ox + i : nullptr)
                                              : (p->uset_par ? p->uset_par + ou + i : nullptr);
                const char* nm = side == 0 ? "xset" : "uset";
                if (kind < PIMPC_SET_BOX || kind > PIMPC_SET_L1BALL)
                    return ctx->fail(PIMPC_E_ARG, "instance %d: unknown %s kind %d", i, nm, kind);
                if (kind == PIMPC_SET_BOX) continue;
                if (kind == PIMPC_SET_SOC && n < 2)
                    return ctx->fail(PIMPC_E_DIM, "instance %d: a second-order cone %s needs >= 2 entries", i, nm);
                if (kind != PIMPC_SET_SOC && !par)
                    return ctx->fail(PIMPC_E_ARG, "instance %d: %s_par is required for this set", i, nm);
                if (par && !finite_arr(par, n + 1))
                    return ctx->fail(PIMPC_E_NONFINITE, "instance %d: %s_par contains NaN or Inf", i, nm);
                if (kind == PIMPC_SET_HALFSPACE || kind == PIMPC_SET_HYPERPLANE) {
                    double aa = 0.0;
                    for (int r = 0; r < n; ++r) aa += par[r] * par[r];
                    if (!(aa > 0.0)) return ctx->fail(PIMPC_E_ARG, "instance %d: %s normal a is zero", i, nm);
                }
                if (kind == PIMPC_SET_L1BALL && !(par[n] >= 0.0))
                    return ctx->fail(PIMPC_E_ARG, "instance %d: %s radius must be >= 0", i, nm);
                if (o->ckpt_every > 0)
                    return ctx->fail(PIMPC_E_UNSUPPORTED,
                                     "instance %d: the taped forward differentiates box constraints only", i);
            }
            ox += p->nx[i];
            ou += p->nu[i];
        }
    }

    // ---------------- layout
    ctx->opt = *o;
    ctx->fp64 = o->precision == PIMPC_FP64;
    ctx->tsize = ctx->fp64 ? sizeof(double) : sizeof(float);
    ctx->count = count;
    ctx->tv = tv;
    ctx->inst.resize(count);
    int64_t mo = 0, m64 = 0, so = 0, io = 0, xo = 0, uo = 0, oq = 0, orr = 0, ga = 0, gb = 0;
    std::vector<FactorTask> tasks;
    for (int i = 0; i < count; ++i) {
        InstDev& I = ctx->inst[i];
        memset(&I, 0, sizeof(I));
        I.nx = p->nx[i];
        I.nu = p->nu[i];
        I.nb = I.nx + I.nu;
        I.N = p->N[i];
        I.tv = tv;
        I.xset = p->xset ? p->xset[i] : PIMPC_SET_BOX;
        I.uset = p->uset ? p->uset[i] : PIMPC_SET_BOX;
        const int cls = (I.N <= kBinThreads) ? pick_class(I.nx, I.nu, tv, ctx->fp64 ? 8 : 4) : -1;
        int rnx = 0, rnu = 0;
        const bool row_ok = row_supported(I.nx, I.nu, I.N, tv, ctx->fp64, &rnx, &rnu);
        bool lane = cls >= 0;
        if (o->family == PIMPC_FAMILY_LANE) {
            if (cls < 0)
                return ctx->fail(PIMPC_E_UNSUPPORTED,
                                 "instance %d (nx=%d, nu=%d, N=%d): no lane-family class holds it", i, I.nx,
                                 I.nu, I.N);
        } else if (o->family == PIMPC_FAMILY_ROW) {
            lane = false;
        } else if (count == 1 && row_ok && I.xset == PIMPC_SET_BOX && I.uset == PIMPC_SET_BOX &&
                   o->ckpt_every == 0) {
            // One instance alone: a row of the stage per lane gives a much
            // shorter iteration than one lane walking every row of its stage.
            lane = false;
        }
        if (lane) {
            const ClassDesc* cd = class_desc(cls);
            I.cls = cls;
            I.nxp = cd->nx;
            I.nup = cd->nu;
        } else {
            if (!row_ok)
                return ctx->fail(PIMPC_E_UNSUPPORTED,
                                 "instance %d (nx=%d, nu=%d, N=%d, %s, %s) has no compiled kernel", i, I.nx, I.nu,
                                 I.N, tv ? "time-varying" : "time-invariant", ctx->fp64 ? "fp64" : "fp32");
            I.cls = -1;
            I.nxp = rnx;
            I.nup = rnu;
            // the kernel variant with a reducer wave serves the eps stop and
            // restart acceleration
            I.row_acc = (o->accel == 1 || o->eps > 0.0) ? 1 : 0;
            ctx->row_insts.push_back(i);
        }
        I.nbp = I.nxp + I.nup;
        // H_{N-1} = (Qbar + rho I)^-1 is diagonal when Q and R are
        bool diag = !tv;
        for (int r = 0; r < I.nx && diag; ++r)
            for (int c = 0; c < I.nx; ++c)
                if (r != c && p->Q[oq + r * I.nx + c] != 0.0) diag = false;
        for (int r = 0; r < I.nu && diag; ++r)
            for (int c = 0; c < I.nu; ++c)
                if (r != c && p->R[orr + r * I.nu + c] != 0.0) diag = false;
        I.hb_diag = diag ? 1 : 0;
        oq += (int64_t)I.nx * I.nx;
        orr += (int64_t)I.nu * I.nu;
        I.mat_off = mo;
        mo += (mat_block_size(I.nxp, I.nup, I.N, tv) + 15) / 16 * 16;
        I.mat64_off = m64;
        m64 += (mat64_block_size(I.nxp, I.nup, I.N, tv) + 15) / 16 * 16;
        I.st_off = so;
        so += 5LL * I.nbp * I.N;
        I.it_off = io;
        io += (int64_t)(I.nup + I.nbp) * I.N;
        I.x_off = xo;
        xo += I.nx;
        I.u_off = uo;
        uo += I.nu;
        I.ga_off = ga;
        ga += (int64_t)I.nx * I.nx;
        I.gb_off = gb;
        gb += (int64_t)I.nx * I.nu;
        // the expansion of the stage data indexes one instance's A, B, e in 32 bits
        if ((int64_t)(tv ? I.N : 1) * (I.nxp * I.nxp + I.nxp * I.nup + I.nxp) >= INT32_MAX)
            return ctx->fail(PIMPC_E_DIM, "instance %d: time-varying stage data too large (N=%d)", i, I.N);
        if (!tv) {
            if (I.N > 1) tasks.push_back({i, 0, 0, 0});
            tasks.push_back({i, 1, I.N - 1, 0});
            tasks.push_back({i, 2, 0, 0});
        } else {
            for (int k = 0; k < I.N; ++k) {
                tasks.push_back({i, k < I.N - 1 ? 0 : 1, k, 0});
                tasks.push_back({i, 2, k, 0});
            }
        }
    }
    ctx->mat_elems = mo;
    ctx->mat64_elems = m64;
    ctx->st_elems = so;
    ctx->it_elems = io;
    ctx->sum_nx = xo;
    ctx->sum_nu = uo;
    ctx->ntasks = (int)tasks.size();
    for (const InstDev& I : ctx->inst) ctx->nb_max = std::max(ctx->nb_max, I.nbp);

    // ---------------- device
    int dev = 0;
    HIPCHK(ctx, hipGetDevice(&dev));
    ctx->device = dev;
    HIPCHK(ctx, hipDeviceGetAttribute(&ctx->num_cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHK(ctx, scratch_init(dev));  // the no-alloc solve's scratch on this device
    for (int j = 0; j < 3; ++j) {
        HIPCHK(ctx, hipStreamCreateWithFlags(&ctx->aux[j], hipStreamNonBlocking));
        HIPCHK(ctx, hipEventCreateWithFlags(&ctx->ev_join[j], hipEventDisableTiming));
    }
    HIPCHK(ctx, hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming));
    hipError_t e = hipSuccess;
    const size_t ts = ctx->tsize;
#define DALLOC(ptr, type, n)                                                                  \
    do {                                                                                      \
        ptr = (decltype(ptr))dmalloc<type>((size_t)(n), &e);                                  \
        if (e != hipSuccess) return ctx->fail(PIMPC_E_NOMEM, "hipMalloc(%s) failed", #ptr);     \
    } while (0)
    DALLOC(ctx->d_inst, InstDev, count);
    DALLOC(ctx->d_mats, char, ctx->mat_elems * ts);
    DALLOC(ctx->d_mats64, double, ctx->mat64_elems);
    DALLOC(ctx->d_state, char, ctx->st_elems * ts);
    DALLOC(ctx->d_iters, char, ctx->it_elems * ts);
    DALLOC(ctx->d_x0, char, ctx->sum_nx * ts);
    DALLOC(ctx->d_up, char, ctx->sum_nu * ts);
    DALLOC(ctx->d_u0, char, ctx->sum_nu * ts);
    DALLOC(ctx->d_info, InfoDev, count);
    {
        const size_t pin = pin_align(ctx->sum_nx * 8) + 2 * pin_align(ctx->sum_nu * 8) + pin_align(count * sizeof(InfoDev));
        e = hipHostMalloc((void**)&ctx->h_pin, pin, hipHostMallocDefault);
        if (e != hipSuccess) return ctx->fail(PIMPC_E_NOMEM, "pinned host staging allocation failed");
    }
    DALLOC(ctx->d_tasks, FactorTask, ctx->ntasks);
    DALLOC(ctx->d_bad, int32_t, ctx->ntasks);
    DALLOC(ctx->d_ibad, int32_t, count);
    DALLOC(ctx->d_nonfinite, int32_t, 1);
    {
        // offsets of every instance's A, B, e in the caller's packed arrays
        // (the device-side stage import of pimpc_linearize reads them)
        std::vector<int64_t> pk(3 * (size_t)count);
        int64_t oa = 0, ob = 0, oe = 0;
        for (int i = 0; i < count; ++i) {
            const int64_t S = tv ? ctx->inst[i].N : 1;
            pk[3 * i + 0] = oa;
            pk[3 * i + 1] = ob;
            pk[3 * i + 2] = oe;
            oa += S * ctx->inst[i].nx * ctx->inst[i].nx;
            ob += S * ctx->inst[i].nx * ctx->inst[i].nu;
            oe += S * ctx->inst[i].nx;
        }
        DALLOC(ctx->d_pack_off, int64_t, pk.size());
        HIPCHK(ctx, hipMemcpy(ctx->d_pack_off, pk.data(), pk.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    }
    HIPCHK(ctx, hipMemcpy(ctx->d_inst, ctx->inst.data(), count * sizeof(InstDev), hipMemcpyHostToDevice));
    HIPCHK(ctx, hipMemcpy(ctx->d_tasks, tasks.data(), tasks.size() * sizeof(FactorTask), hipMemcpyHostToDevice));
    HIPCHK(ctx, hipMemset(ctx->d_state, 0, ctx->st_elems * ts));
    if (o->accel == 1) DALLOC(ctx->d_prev, char, ctx->st_elems * ts);
    HIPCHK(ctx, hipMemset(ctx->d_iters, 0, ctx->it_elems * ts));
    HIPCHK(ctx, hipMemset(ctx->d_up, 0, ctx->sum_nu * ts));

    std::vector<double>& m64v = ctx->h_mats64;
    build_mats64(ctx, p->A, p->B, p->e, p->Q, p->R, p->Wdu, m64v, false);
    HIPCHK(ctx, hipMemcpy(ctx->d_mats64, m64v.data(), m64v.size() * sizeof(double), hipMemcpyHostToDevice));
    ctx->h_mats64_valid = true;
    int rc = ctx->fp64
                 ? upload_t_block<double>(ctx, p->qbar, p->xmin, p->xmax, p->umin, p->umax, p->xset_par, p->uset_par)
                 : upload_t_block<float>(ctx, p->qbar, p->xmin, p->xmax, p->umin, p->umax, p->xset_par, p->uset_par);
    if (rc != PIMPC_OK) return rc;
    rc = refactor(ctx, true);
    if (rc != PIMPC_OK) return rc;

    // ---------------- schedule
    std::vector<Bin> bins;
    build_bins(ctx, bins, ctx->runs, kBinWaves, ctx->fp64 != 0);
    if (!bins.empty()) {
        DALLOC(ctx->d_bins, Bin, bins.size());
        HIPCHK(ctx, hipMemcpy(ctx->d_bins, bins.data(), bins.size() * sizeof(Bin), hipMemcpyHostToDevice));
    }
    for (const Bin& b : bins) {
        int w = 0;
        for (int j = 0; j < b.n; ++j) w += b.e[j].nwaves;
        ctx->bin_waves.push_back(w);
    }
    // (the autotuner may split every class launch in two)
    DALLOC(ctx->d_counters, int32_t, std::max<size_t>(2 * ctx->runs.size(), 1));
    for (ClassRun& r : ctx->runs) {
        int occ = 1;
        // (a class without a backward is refused below, with its reason)
        const bool rec = rec_steps(ctx) && !ctx->fp64 && !tv && r.gs == 0 && backward_class_supported(r.cls);
        HIPCHK(ctx, lane_dispatch_any(ctx->fp64, r.cls, r.gs, rec, nullptr, r.bw, 0, ctx->stream, &occ));
        r.occ = occ;
    }
    if (!ctx->row_insts.empty()) {
        size_t cbytes = 0, fbytes = 0;
        for (int i : ctx->row_insts) {
            ctx->row_clear_off.push_back(cbytes);
            ctx->row_fused_off.push_back(fbytes);
            cbytes += row_clear_bytes(ctx->inst[i]);
            fbytes += row_fused_bytes(ctx->inst[i]);
        }
        ctx->row_clear_total = cbytes;
        DALLOC(ctx->d_row_clear, char, cbytes);
        DALLOC(ctx->d_row_fused, char, fbytes);
        HIPCHK(ctx, hipMemset(ctx->d_row_clear, 0, cbytes));
        HIPCHK(ctx, hipMemset(ctx->d_row_fused, 0, fbytes));
        const char* env_s = getenv("PIMPC_ROW_STAGES");
        for (int i : ctx->row_insts) {
            ctx->inst[i].row_s = env_s ? atoi(env_s) : 1;
            const hipError_t e = row_prepare(ctx->fp64, ctx->inst[i]);
            if (e == hipErrorInvalidConfiguration)
                return ctx->fail(PIMPC_E_UNSUPPORTED,
                                 "instance %d: horizon N=%d does not fit one co-resident grid of the row "
                                 "family at up to 4 stages per wave",
                                 i, ctx->inst[i].N);
            HIPCHK(ctx, e);
        }
        HIPCHK(ctx, hipMemcpy(ctx->d_inst, ctx->inst.data(), count * sizeof(InstDev), hipMemcpyHostToDevice));
        HIPCHK(ctx, hipDeviceSynchronize());  // the scratch clear above is complete
        HIPCHK(ctx, fuse_rows(ctx, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    if (o->ckpt_every > 0) {
        if (ctx->fp64 || tv || !ctx->row_insts.empty())
            return ctx->fail(PIMPC_E_UNSUPPORTED, "the taped forward / backward needs FP32, time-invariant "
                                                  "instances of the lane family");
        // ckpt_every = 1: the forward records all max_iter steps, no checkpoints;
        // otherwise checkpoints and a tape of one segment
        const bool all = o->ckpt_every == 1;
        int64_t ck = 0, tp = 0;
        const int nck = all ? 0 : (o->max_iter + o->ckpt_every - 1) / o->ckpt_every;
        const int seg = all ? o->max_iter : o->ckpt_every;
        for (int i = 0; i < count; ++i) {
            InstDev& I = ctx->inst[i];
            if (!backward_class_supported(I.cls) || I.N > 256)
                return ctx->fail(PIMPC_E_UNSUPPORTED, "instance %d: backward supports nx + nu <= 16 (padded) "
                                                      "and N <= 256", i);
            I.ck_off = ck;
            ck += (int64_t)nck * 5 * I.nbp * I.N;
            I.tape_off = tp;
            tp += (int64_t)seg * tape_rec_floats(I.nbp, I.nxp) * I.N;
            I.gr_off = (int64_t)i * kGradStride;
        }
        DALLOC(ctx->d_ckpt, float, ck);
        DALLOC(ctx->d_tape, float, tp);
        DALLOC(ctx->d_grads, float, (int64_t)count * kGradStride);
        HIPCHK(ctx, hipMemcpy(ctx->d_inst, ctx->inst.data(), count * sizeof(InstDev), hipMemcpyHostToDevice));
        std::vector<Bin> bb;
        build_bins(ctx, bb, ctx->bwd_runs, 4, false);
        DALLOC(ctx->d_bwd_bins, Bin, bb.size());
        HIPCHK(ctx, hipMemcpy(ctx->d_bwd_bins, bb.data(), bb.size() * sizeof(Bin), hipMemcpyHostToDevice));
        DALLOC(ctx->d_bwd_counters, int32_t, std::max<size_t>(ctx->bwd_runs.size(), 1));
    }
#undef DALLOC
    rc = autotune(ctx);
    if (rc != PIMPC_OK) return rc;
    ctx->na_args.reserve(ctx->runs.size());
    ctx->na_rargs.reserve(ctx->row_insts.size());
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return PIMPC_OK;
}

// Output form of eqn. (1): the cost 1/2 ||C x_{k+1} - r_y||^2_Wy +
// 1/2 ||u_k - r_u||^2_R expands (constant terms dropped) to
// 1/2 x'(C' Wy C) x - (C' Wy r_y)' x + 1/2 u'R u - (R r_u)' u, which is the
// velocity-form cost with Q + C' Wy C and qbar + (C' Wy r_y, R r_u).  A bound
// on an output that selects one state (y_i = c_ij x_j) is a bound on x_j.
// Writes the folded problem to *q (pointing into f); the caller's arrays
// are not touched.
struct Folded {
    std::vector<double> Q, qbar, xmin, xmax;
};

static int fold_outputs(pimpc_ctx ctx, const pimpc_problem* p, pimpc_problem* q, Folded& f) {
    *q = *p;
    if (!p || (!p->ny && !p->ru)) return PIMPC_OK;
    if (p->count < 1 || !p->nx || !p->nu || !p->R || !p->xmin || !p->xmax)
        return ctx->fail(PIMPC_E_ARG, "a required problem array is NULL");
    if (!p->Q && !p->ny) return ctx->fail(PIMPC_E_ARG, "Q is required without the output form");
    const int count = p->count;
    int64_t snx = 0, snu = 0, sQ = 0, sR = 0, sny = 0, sC = 0, sW = 0;
    for (int i = 0; i < count; ++i) {
        const int nx = p->nx[i], nu = p->nu[i], ny = p->ny ? p->ny[i] : 0;
        if (nx < 1 || nu < 1 || nx > 48 || nu > 16)
            return ctx->fail(PIMPC_E_DIM, "instance %d: nx <= 48, nu <= 16 supported", i);
        if (ny < 0 || ny > 32) return ctx->fail(PIMPC_E_DIM, "instance %d: ny must be in [0, 32]", i);
        snx += nx;
        snu += nu;
        sQ += (int64_t)nx * nx;
        sR += (int64_t)nu * nu;
        sny += ny;
        sC += (int64_t)ny * nx;
        sW += (int64_t)ny * ny;
    }
    if (p->ny && (!p->C || !p->Wy)) return ctx->fail(PIMPC_E_ARG, "the output form needs C and Wy");
    if ((p->C && !finite_arr(p->C, sC)) || (p->Wy && !finite_arr(p->Wy, sW)) ||
        (p->ry && !finite_arr(p->ry, sny)) || !finite_arr(p->R, sR) || (p->ru && !finite_arr(p->ru, snu)) ||
        (p->Q && !finite_arr(p->Q, sQ)) || (p->qbar && !finite_arr(p->qbar, snx + snu)))
        return ctx->fail(PIMPC_E_NONFINITE, "problem data contains NaN or Inf");
    f.Q.assign(sQ, 0.0);
    if (p->Q) std::copy(p->Q, p->Q + sQ, f.Q.begin());
    f.qbar.assign(snx + snu, 0.0);
    if (p->qbar) std::copy(p->qbar, p->qbar + snx + snu, f.qbar.begin());
    f.xmin.assign(p->xmin, p->xmin + snx);
    f.xmax.assign(p->xmax, p->xmax + snx);
    int64_t oq = 0, orr = 0, ox = 0, ou = 0, oy = 0, oc = 0, ow = 0, ob = 0;
    for (int i = 0; i < count; ++i) {
        const int nx = p->nx[i], nu = p->nu[i], ny = p->ny ? p->ny[i] : 0;
        if (ny > 0) {
            const double* C = p->C + oc;
            const double* Wy = p->Wy + ow;
            bool sym = true;
            if (!sym_psd(Wy, ny, &sym))
                return ctx->fail(PIMPC_E_NOT_PSD, "instance %d: Wy is not %s", i, sym ? "PSD" : "symmetric");
            std::vector<double> WC((size_t)ny * nx, 0.0);  // Wy C
            for (int a = 0; a < ny; ++a)
                for (int j = 0; j < nx; ++j)
                    for (int b = 0; b < ny; ++b) WC[(size_t)a * nx + j] += Wy[a * ny + b] * C[(size_t)b * nx + j];
            for (int r = 0; r < nx; ++r)
                for (int c = 0; c < nx; ++c) {
                    double acc = 0.0;
                    for (int a = 0; a < ny; ++a) acc += C[(size_t)a * nx + r] * WC[(size_t)a * nx + c];
                    f.Q[oq + (int64_t)r * nx + c] += acc;
                }
            if (p->ry)
                for (int r = 0; r < nx; ++r) {
                    double acc = 0.0;
                    for (int a = 0; a < ny; ++a) acc += WC[(size_t)a * nx + r] * p->ry[oy + a];
                    f.qbar[ob + r] += acc;  // C' Wy r_y (Wy symmetric)
                }
            if (p->ymin || p->ymax) {
                const int xk = p->xset ? p->xset[i] : PIMPC_SET_BOX;
                for (int a = 0; a < ny; ++a) {
                    const double lo = p->ymin ? p->ymin[oy + a] : -INFINITY;
                    const double hi = p->ymax ? p->ymax[oy + a] : INFINITY;
                    if (std::isnan(lo) || std::isnan(hi) || lo > hi)
                        return ctx->fail(PIMPC_E_ARG, "instance %d: output bound %d needs ymin <= ymax (no NaN)", i, a);
                    if (lo == -INFINITY && hi == INFINITY) continue;
                    int nz = 0, jsel = -1;
                    for (int j = 0; j < nx; ++j)
                        if (C[(size_t)a * nx + j] != 0.0) {
                            ++nz;
                            jsel = j;
                        }
                    if (nz != 1)
                        return ctx->fail(PIMPC_E_UNSUPPORTED,
                                         "instance %d: a bound on output %d, which mixes %d states (a bounded "
                                         "output must select one state)", i, a, nz);
                    if (xk != PIMPC_SET_BOX)
                        return ctx->fail(PIMPC_E_UNSUPPORTED,
                                         "instance %d: output bounds need a box x factor", i);
                    const double cj = C[(size_t)a * nx + jsel];
                    double xl = lo / cj, xh = hi / cj;
                    if (cj < 0.0) std::swap(xl, xh);
                    double& mn = f.xmin[ox + jsel];
                    double& mx = f.xmax[ox + jsel];
                    mn = std::max(mn, xl);
                    mx = std::min(mx, xh);
                    if (!(mn <= mx))
                        return ctx->fail(PIMPC_E_ARG, "instance %d: output bound %d leaves an empty box on x_%d", i,
                                         a, jsel);
                }
            }
        }
        if (p->ru)
            for (int r = 0; r < nu; ++r) {
                double acc = 0.0;
                for (int c = 0; c < nu; ++c) acc += p->R[orr + (int64_t)r * nu + c] * p->ru[ou + c];
                f.qbar[ob + nx + r] += acc;
            }
        oq += (int64_t)nx * nx;
        orr += (int64_t)nu * nu;
        ox += nx;
        ou += nu;
        oy += ny;
        oc += (int64_t)ny * nx;
        ow += (int64_t)ny * ny;
        ob += nx + nu;
    }
    q->Q = f.Q.data();
    q->qbar = f.qbar.data();
    q->xmin = f.xmin.data();
    q->xmax = f.xmax.data();
    q->ny = nullptr;
    q->C = q->Wy = q->ry = q->ymin = q->ymax = q->ru = nullptr;
    return PIMPC_OK;
}

int32_t pimpc_setup(pimpc_ctx* out, const pimpc_problem* prob, const pimpc_options* opts, void* hip_stream) {
    if (!out) {
        g_setup_err = "out pointer is NULL";
        return PIMPC_E_ARG;
    }
    *out = nullptr;
    pimpc_ctx ctx = new (std::nothrow) pimpc_ctx_s();
    if (!ctx) {
        g_setup_err = "host allocation failed";
        return PIMPC_E_NOMEM;
    }
    ctx->stream = (hipStream_t)hip_stream;
    pimpc_problem folded;
    Folded fstore;
    int rc = prob ? fold_outputs(ctx, prob, &folded, fstore) : PIMPC_OK;
    if (rc == PIMPC_OK) rc = setup_impl(ctx, prob ? &folded : nullptr, opts);
    if (rc != PIMPC_OK) {
        g_setup_err = ctx->err;
        destroy_ctx(ctx);
        return rc;
    }
    *out = ctx;
    return PIMPC_OK;
}

int32_t pimpc_linearize(pimpc_ctx ctx, const double* A, const double* B, const double* e, int32_t mem_kind) {
    if (!ctx) return PIMPC_E_ARG;
    if (!A || !B) return ctx->fail(PIMPC_E_ARG, "A and B are required");
    if (mem_kind != PIMPC_MEM_HOST && mem_kind != PIMPC_MEM_DEVICE)
        return ctx->fail(PIMPC_E_ARG, "mem_kind must be PIMPC_MEM_HOST or PIMPC_MEM_DEVICE");
    ctx->tape_id = 0;  // a tape refers to the factors it was recorded with
    if (mem_kind == PIMPC_MEM_DEVICE) {
        // import on the device, ordered on the context's stream after the work
        // that produced A, B, e there; the padded FP64 block is rewritten in
        // place and the host copy of it goes stale
        const hipStream_t s = ctx->stream;
        ctx->h_mats64_valid = false;
        HIPCHK(ctx, launch_fill<int32_t>(ctx->d_nonfinite, 1, 0, s));
        HIPCHK(ctx, launch_stage_import(ctx->d_inst, ctx->count, ctx->d_pack_off, A, B, e, ctx->d_mats64,
                                        ctx->d_nonfinite, s));
        int rc = refactor(ctx, true);  // synchronises the stream
        int32_t nf = 0;
        HIPCHK(ctx, hipMemcpy(&nf, ctx->d_nonfinite, sizeof(int32_t), hipMemcpyDeviceToHost));
        if (nf) return ctx->fail(PIMPC_E_NONFINITE, "stage data contains NaN or Inf");
        return rc;
    }
    int64_t sA = 0, sB = 0, se = 0;
    for (const InstDev& I : ctx->inst) {
        const int64_t S = I.tv ? I.N : 1;
        sA += S * I.nx * I.nx;
        sB += S * I.nx * I.nu;
        se += S * I.nx;
    }
    const double *pA = A, *pB = B, *pe = e;
    if (!finite_arr(pA, sA) || !finite_arr(pB, sB) || (pe && !finite_arr(pe, se)))
        return ctx->fail(PIMPC_E_NONFINITE, "stage data contains NaN or Inf");
    // The weights and bounds of the block stay; only A, B, e are rewritten.
    // The host copy is current unless pimpc_set_params_dev replaced the
    // parameters on the device.
    std::vector<double>& m64v = ctx->h_mats64;
    if (!ctx->h_mats64_valid) {
        m64v.resize(ctx->mat64_elems);
        HIPCHK(ctx, hipMemcpy(m64v.data(), ctx->d_mats64, m64v.size() * sizeof(double), hipMemcpyDeviceToHost));
        ctx->h_mats64_valid = true;
    }
    build_mats64(ctx, pA, pB, pe, nullptr, nullptr, nullptr, m64v, true);
    HIPCHK(ctx, hipMemcpyAsync(ctx->d_mats64, m64v.data(), m64v.size() * sizeof(double), hipMemcpyHostToDevice,
                               ctx->stream));
    int rc = refactor(ctx, true);
    if (rc != PIMPC_OK) return rc;
    return PIMPC_OK;
}

int32_t pimpc_solve(pimpc_ctx ctx, const double* x0, const double* u_prev, double* u0_out, pimpc_info* info) {
    if (!ctx) return PIMPC_E_ARG;
    if (!x0) return ctx->fail(PIMPC_E_ARG, "x0 is required");
    if (!finite_arr(x0, ctx->sum_nx) || (u_prev && !finite_arr(u_prev, ctx->sum_nu)))
        return ctx->fail(PIMPC_E_NONFINITE, "x0 or u_prev contains NaN or Inf");
    const hipStream_t s = ctx->stream;
    // pinned staging (the call ends with a stream synchronisation, so the
    // next call may reuse it)
    char* px = ctx->h_pin;
    char* pu = px + pin_align(ctx->sum_nx * 8);
    char* po = pu + pin_align(ctx->sum_nu * 8);
    InfoDev* pinf = (InfoDev*)(po + pin_align(ctx->sum_nu * 8));
    for (int64_t j = 0; j < ctx->sum_nx; ++j) {
        if (ctx->fp64)
            ((double*)px)[j] = x0[j];
        else
            ((float*)px)[j] = (float)x0[j];
    }
    if (u_prev)
        for (int64_t j = 0; j < ctx->sum_nu; ++j) {
            if (ctx->fp64)
                ((double*)pu)[j] = u_prev[j];
            else
                ((float*)pu)[j] = (float)u_prev[j];
        }
    HIPCHK(ctx, hipMemcpyAsync(ctx->d_x0, px, ctx->sum_nx * ctx->tsize, hipMemcpyHostToDevice, s));
    if (u_prev) HIPCHK(ctx, hipMemcpyAsync(ctx->d_up, pu, ctx->sum_nu * ctx->tsize, hipMemcpyHostToDevice, s));
    const int warm = (ctx->opt.warm_start && ctx->has_state) ? 1 : 0;
    int rc = 0;
    LaunchSet* ls = get_set(ctx, ctx->d_x0, u_prev ? ctx->d_up : nullptr, ctx->d_u0, ctx->d_info, warm, 1, s, &rc);
    if (!ls) return rc;
    rc = run_set(ctx, ls, s, false);
    if (rc != PIMPC_OK) return rc;
    if (ctx->opt.ckpt_every > 0) {
        ctx->tape_id = ++ctx->tape_count;
        ctx->tape_x0 = ctx->d_x0;
        ctx->tape_up = u_prev ? ctx->d_up : nullptr;
    }
    HIPCHK(ctx, hipMemcpyAsync(po, ctx->d_u0, ctx->sum_nu * ctx->tsize, hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipMemcpyAsync(pinf, ctx->d_info, ctx->count * sizeof(InfoDev), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    ctx->has_state = 1;
    if (u0_out)
        for (int64_t j = 0; j < ctx->sum_nu; ++j)
            u0_out[j] = ctx->fp64 ? ((double*)po)[j] : (double)((float*)po)[j];
    const InfoDev* inf = pinf;
    if (info) memcpy(info, inf, ctx->count * sizeof(InfoDev));
    for (int i = 0; i < ctx->count; ++i)
        if (inf[i].status == PIMPC_E_HIP)
            return ctx->fail(PIMPC_E_HIP, "instance %d: a wait between workgroups gave up (the grid was not "
                                          "resident at once)", i);
        else if (inf[i].status == PIMPC_E_NOT_PSD)
            return ctx->fail(PIMPC_E_NOT_PSD, "instance %d: a stage matrix of the last factorisation is not SPD",
                             i);
        else if (inf[i].status != 0)
            return ctx->fail(PIMPC_E_NONFINITE, "instance %d: iterate became non-finite", i);
    return PIMPC_OK;
}

int32_t pimpc_solve_batch(pimpc_ctx ctx, const void* x0_dev, const void* uprev_dev, void* u0_dev,
                          pimpc_info* info_dev, void* hip_stream) {
    if (!ctx) return PIMPC_E_ARG;
    if (!x0_dev || !u0_dev) return ctx->fail(PIMPC_E_ARG, "x0_dev and u0_dev are required");
    const hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    const int warm = (ctx->opt.warm_start && ctx->has_state) ? 1 : 0;
    int rc = 0;
    LaunchSet* ls = get_set(ctx, x0_dev, uprev_dev, u0_dev, info_dev, warm, 0, s, &rc);
    if (!ls) return rc;
    rc = run_set(ctx, ls, s, true);
    if (rc != PIMPC_OK) return rc;
    ctx->has_state = 1;
    if (ctx->opt.ckpt_every > 0) {
        ctx->tape_id = ++ctx->tape_count;
        ctx->tape_x0 = x0_dev;
        ctx->tape_up = uprev_dev;
    }
    return PIMPC_OK;
}

int32_t pimpc_solve_batch_noalloc(pimpc_ctx ctx, const void* x0_dev, const void* uprev_dev, void* u0_dev,
                                  pimpc_info* info_dev, void* hip_stream) {
    if (!ctx) return PIMPC_E_ARG;
    if (!x0_dev || !u0_dev) return ctx->fail(PIMPC_E_ARG, "x0_dev and u0_dev are required");
    int dev = -1;
    HIPCHK(ctx, hipGetDevice(&dev));
    if (dev != ctx->device)
        return ctx->fail(PIMPC_E_STATE, "the context was set up on device %d, device %d is current", ctx->device,
                         dev);
    char* base = (char*)scratch_dev(dev);
    if (!base) return ctx->fail(PIMPC_E_STATE, "the no-alloc scratch of device %d was not set up", dev);
    // layout of this call's scratch: lane arguments | row arguments | bin
    // counters | per-solve part of every row-family instance
    auto up256 = [](size_t x) { return (x + 255) / 256 * 256; };
    const size_t ncls = ctx->runs.size(), nrow = ctx->row_insts.size();
    const size_t o_args = 0;
    const size_t o_rargs = up256(o_args + ncls * sizeof(LaneArgs));
    const size_t o_cnt = up256(o_rargs + nrow * sizeof(RowArgs));
    const size_t o_row = up256(o_cnt + std::max<size_t>(ncls, 1) * sizeof(int32_t));
    const size_t need = o_row + ctx->row_clear_total;
    if (need > (size_t)PIMPC_NOALLOC_SCRATCH_BYTES)
        return ctx->fail(PIMPC_E_DIM, "this context needs %zu bytes of per-solve scratch; the static scratch holds %zu "
                                      "(use pimpc_solve_batch)", need, (size_t)PIMPC_NOALLOC_SCRATCH_BYTES);
    const hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    const int warm = (ctx->opt.warm_start && ctx->has_state) ? 1 : 0;
    const SolveScratch sc{(int32_t*)(base + o_cnt), base + o_row};
    // host staging of the arguments, reserved at setup (no allocation here)
    std::vector<LaneArgs>& args = ctx->na_args;
    std::vector<RowArgs>& rargs = ctx->na_rargs;
    build_args(ctx, x0_dev, uprev_dev, u0_dev, info_dev, warm, 0, sc, args, rargs);
    // the arguments travel as kernel arguments into the scratch, ordered on
    // `s` before the launches that read them
    if (!args.empty()) HIPCHK(ctx, launch_bytes_store(base + o_args, args.data(), args.size() * sizeof(LaneArgs), s));
    if (!rargs.empty())
        HIPCHK(ctx, launch_bytes_store(base + o_rargs, rargs.data(), rargs.size() * sizeof(RowArgs), s));
    const int rc = enqueue_launches(ctx, (const LaneArgs*)(base + o_args), (const RowArgs*)(base + o_rargs), sc, s);
    if (rc != PIMPC_OK) return rc;
    ctx->has_state = 1;
    if (ctx->opt.ckpt_every > 0) {
        ctx->tape_id = ++ctx->tape_count;
        ctx->tape_x0 = x0_dev;
        ctx->tape_up = uprev_dev;
    }
    return PIMPC_OK;
}

int32_t pimpc_set_params_dev(pimpc_ctx ctx, const void* A, const void* B, const void* Qdiag, const void* Rdiag,
                             void* hip_stream) {
    if (!ctx) return PIMPC_E_ARG;
    if (!A || !B || !Qdiag || !Rdiag) return ctx->fail(PIMPC_E_ARG, "A, B, Qdiag, Rdiag are required");
    if (ctx->tv) return ctx->fail(PIMPC_E_STATE, "set_params_dev needs a time-invariant context");
    for (const InstDev& I : ctx->inst)
        if (I.nx != ctx->inst[0].nx || I.nu != ctx->inst[0].nu)
            return ctx->fail(PIMPC_E_STATE, "set_params_dev needs equal nx and nu across instances");
    const hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    ctx->h_mats64_valid = false;  // the device copy changes below
    ctx->tape_id = 0;             // a tape refers to the factors it was recorded with
    if (ctx->fp64)
        HIPCHK(ctx, launch_params<double>(ctx->d_inst, ctx->count, (const double*)A, (const double*)B,
                                          (const double*)Qdiag, (const double*)Rdiag, ctx->d_mats64, s));
    else
        HIPCHK(ctx, launch_params<float>(ctx->d_inst, ctx->count, (const float*)A, (const float*)B,
                                         (const float*)Qdiag, (const float*)Rdiag, ctx->d_mats64, s));
    const hipStream_t saved = ctx->stream;
    ctx->stream = s;
    const int rc = refactor(ctx, false);
    ctx->stream = saved;
    return rc;
}

uint64_t pimpc_tape_id(pimpc_ctx ctx) { return ctx ? ctx->tape_id : 0; }

int32_t pimpc_backward(pimpc_ctx ctx, uint64_t tape_id, const void* dL_du0_dev, void* dx0, void* dQdiag,
                       void* dRdiag, void* dA, void* dB, void* hip_stream) {
    if (!ctx) return PIMPC_E_ARG;
    if (ctx->opt.ckpt_every <= 0 || ctx->tape_id == 0)
        return ctx->fail(PIMPC_E_STATE, "no taped forward is available (needs ckpt_every > 0 and a solve after "
                                        "the last parameter update)");
    if (tape_id != ctx->tape_id)
        return ctx->fail(PIMPC_E_STATE, "tape %llu was overwritten: the current tape is %llu (another taped "
                                        "forward, or a parameter update, came after it)",
                         (unsigned long long)tape_id, (unsigned long long)ctx->tape_id);
    if (!dL_du0_dev) return ctx->fail(PIMPC_E_ARG, "dL_du0_dev is required");
    const hipStream_t s = hip_stream ? (hipStream_t)hip_stream : ctx->stream;
    const int ncls = (int)ctx->bwd_runs.size();
    if (ncls > 0) HIPCHK(ctx, launch_fill<int32_t>(ctx->d_bwd_counters, ncls, 0, s));
    for (int c = 0; c < ncls; ++c) {
        const ClassRun& r = ctx->bwd_runs[c];
        BwdArgs a;
        memset(&a, 0, sizeof(a));
        a.inst = ctx->d_inst;
        a.bins = ctx->d_bwd_bins + r.bin_first;
        a.nbins = r.nbins;
        a.bin_counter = ctx->d_bwd_counters + c;
        a.mats = (const float*)ctx->d_mats;
        a.ckpt = (const float*)ctx->d_ckpt;
        a.tape = ctx->d_tape;
        a.grads = ctx->d_grads;
        a.x0 = (const float*)ctx->tape_x0;
        a.uprev = (const float*)ctx->tape_up;
        a.dLdu0 = (const float*)dL_du0_dev;
        a.rho = ctx->opt.rho;
        a.K = ctx->opt.max_iter;
        a.ckpt_every = ctx->opt.ckpt_every;
        a.full_tape = rec_steps(ctx) ? 1 : 0;
        const int grid = std::max(1, std::min(r.nbins, ctx->num_cus));
        bool handled = false;
        HIPCHK(ctx, launch_backward_class(r.cls, a, grid, s, &handled));
        if (!handled) return ctx->fail(PIMPC_E_UNSUPPORTED, "class %d has no backward kernel", r.cls);
    }
    HIPCHK(ctx, launch_chain(ctx->d_inst, ctx->count, ctx->d_mats64, ctx->d_grads, ctx->opt.rho, (float*)dx0,
                             (float*)dQdiag, (float*)dRdiag, (float*)dA, (float*)dB, s));
    return PIMPC_OK;
}

static int iter_io(pimpc_ctx ctx, int32_t which, double* out, const double* in) {
    if (!ctx) return PIMPC_E_ARG;
    if (which < PIMPC_IT_V || which > PIMPC_IT_XBAR) return ctx->fail(PIMPC_E_ARG, "bad iterate selector %d", which);
    if (in && which > PIMPC_IT_LAMBDA) return ctx->fail(PIMPC_E_ARG, "only v, z, theta, beta, lambda can be set");
    if (!out && !in) return ctx->fail(PIMPC_E_ARG, "buffer is NULL");
    const bool st = which <= PIMPC_IT_LAMBDA;
    const int64_t n = st ? ctx->st_elems : ctx->it_elems;
    std::vector<char> buf(std::max<int64_t>(n, 1) * ctx->tsize);
    void* dsrc = st ? ctx->d_state : ctx->d_iters;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    HIPCHK(ctx, hipMemcpy(buf.data(), dsrc, n * ctx->tsize, hipMemcpyDeviceToHost));
    auto get = [&](int64_t idx) -> double {
        return ctx->fp64 ? ((double*)buf.data())[idx] : (double)((float*)buf.data())[idx];
    };
    auto put = [&](int64_t idx, double v) {
        if (ctx->fp64)
            ((double*)buf.data())[idx] = v;
        else
            ((float*)buf.data())[idx] = (float)v;
    };
    int64_t pos = 0;
    for (int i = 0; i < ctx->count; ++i) {
        const InstDev& I = ctx->inst[i];
        const int N = I.N;
        if (which == PIMPC_IT_DU) {
            for (int k = 0; k < N; ++k)
                for (int r = 0; r < I.nu; ++r) out[pos++] = get(I.it_off + (int64_t)r * N + k);
            continue;
        }
        for (int k = 0; k < N; ++k)
            for (int r = 0; r < I.nb; ++r) {
                const int rp = r < I.nx ? r : I.nxp + (r - I.nx);  // padded row
                int64_t idx;
                if (which == PIMPC_IT_XBAR)
                    idx = I.it_off + (int64_t)(I.nup + rp) * N + k;
                else
                    idx = I.st_off + (int64_t)(which * I.nbp + rp) * N + k;
                if (in)
                    put(idx, in[pos++]);
                else
                    out[pos++] = get(idx);
            }
    }
    if (in) {
        HIPCHK(ctx, hipMemcpy(dsrc, buf.data(), n * ctx->tsize, hipMemcpyHostToDevice));
        ctx->has_state = 1;
    }
    return PIMPC_OK;
}

int32_t pimpc_get_iterates(pimpc_ctx ctx, int32_t which, double* out) { return iter_io(ctx, which, out, nullptr); }

int32_t pimpc_set_iterates(pimpc_ctx ctx, int32_t which, const double* in) {
    if (!in) return ctx ? ctx->fail(PIMPC_E_ARG, "buffer is NULL") : PIMPC_E_ARG;
    return iter_io(ctx, which, nullptr, in);
}

}  // extern "C"
