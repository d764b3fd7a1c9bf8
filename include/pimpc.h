/*
 * pimpc.h -- C ABI of the piMPC solver for MI355X (gfx950).
 *
 * Solves the linear time-varying MPC problem of Section II, eqn. (1), of
 * "piMPC: A Parallel-in-horizon and Construction-free NMPC Solver"
 * (arXiv 2601.14414) with the parallel-in-horizon ADMM iteration of
 * Section IV (eqn. (8) and Algorithm 1):
 *
 *   min  sum_{k<N} 1/2 x_{k+1}' Q x_{k+1} + 1/2 u_k' R u_k - qbar' xbar_{k+1}
 *                  + 1/2 (u_k - u_{k-1})' Wdu (u_k - u_{k-1})
 *   s.t. x_{k+1} = A_k x_k + B_k u_k + e_k,  x_{k+1} in X,  u_k in U,
 *        x_0 = x(t),  u_{-1} = u(t-1)
 *
 * (X, U boxes by default, or a halfspace, hyperplane, second-order cone or l1
 * ball) in the velocity form of Theorem 2 (xbar_k = col(x_k, u_{k-1}), input
 * du_k), with the stage caches J_k, H_k of Algorithm 1 factorised in FP64 on
 * the device and the iteration run in the precision chosen by the caller.
 *
 * The two kernel families and what they support:
 *   - lane family, one lane per stage, when N <= 512 and a compiled class
 *     holds the stage (time-invariant: nx <= 16, nu <= 8; time-varying:
 *     nx <= 4, nu <= 2; FP64 up to nx + nu = 13 after padding): FP32 or FP64
 *     iteration, restart acceleration, non-box sets, and the taped forward /
 *     pimpc_backward for FP32 time-invariant instances with N <= 256;
 *   - row family, one row of a stage per lane, one block of stages per wave
 *     (FP32, nx <= 32, nu <= 16; time-varying data up to nx <= 24, nu <= 12;
 *     restart acceleration; non-box sets at one stage per wave or group; no
 *     tape), as long as the horizon fits one grid whose workgroups are all
 *     resident at once (up to 4 stages per wave; for the 24 + 12 class
 *     N <= 4096 on 256 compute units, N <= 1024 with non-box sets).
 * With options.family = PIMPC_FAMILY_AUTO, a context of one FP32 instance
 * with box sets and no tape runs on the row family whenever a row class
 * holds it (its iteration is several times shorter than one lane walking all
 * rows of its stage); otherwise, and for every instance of a batch, the lane
 * family serves what it holds and the row family the rest.
 * A request outside these returns PIMPC_E_UNSUPPORTED from pimpc_setup.
 *
 * Conventions common to every entry point:
 *   - every call returns an int32 status: PIMPC_OK (0) or a negative error;
 *     on error no output buffer is written and pimpc_last_error() describes
 *     the failure.  Nothing throws or aborts across this boundary;
 *   - matrices are dense, row-major, double precision on the host side;
 *   - a context owns all its device memory; the caller keeps ownership of
 *     every array it passes (inputs are copied before the call returns);
 *   - a context is bound to one HIP stream and is not thread-safe;
 *   - a row-family solve needs every workgroup of its grid resident at once.
 *     A context runs its row-family instances first and one after another;
 *     solves of different contexts that hold row-family instances must not
 *     overlap in time (enqueue them on one stream), and other work that keeps
 *     compute units busy for long delays them.  A wait that cannot complete
 *     gives up after a bounded number of polls (a fraction of a second) and
 *     the solve fails (PIMPC_E_HIP, status of the instance non-zero) instead
 *     of hanging;
 *   - "instance" = one MPC problem; a context holds `count` of them, packed
 *     back to back in the order given (offsets are prefix sums of the sizes).
 */
#ifndef PIMPC_H
#define PIMPC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PIMPC_VERSION 2

/* status codes */
#define PIMPC_OK 0
#define PIMPC_E_ARG (-1)         /* bad scalar argument or NULL required pointer */
#define PIMPC_E_DIM (-2)         /* dimensions out of the supported range */
#define PIMPC_E_NOT_PSD (-3)     /* Q or R not symmetric PSD, or a stage matrix not SPD */
#define PIMPC_E_NONFINITE (-4)   /* NaN/Inf input, or an iterate became non-finite */
#define PIMPC_E_HIP (-5)         /* HIP runtime error */
#define PIMPC_E_NOMEM (-6)       /* device allocation failed */
#define PIMPC_E_STATE (-7)       /* call not valid in the context's state */
#define PIMPC_E_UNSUPPORTED (-8) /* valid request this build does not implement */

/* iteration precision (the stage factorisation is always FP64) */
#define PIMPC_FP64 0
#define PIMPC_FP32 1

/* Constraint set of the x_k or of the u_k factor of Xbar = X x U (the z update
 * of Theorem 1 projects onto it; the proof of Theorem 1 lists these sets).
 * Parameters per instance, w = the factor (nx or nu entries), par = (a, b):
 *   BOX         xmin <= w <= xmax (the problem's bounds; par unused)
 *   HALFSPACE   a'w <= b           (a != 0)
 *   HYPERPLANE  a'w = b            (a != 0)
 *   SOC         ||(w_1..w_{n-1})||_2 <= w_n   (n >= 2; par unused)
 *   L1BALL      ||w||_1 <= r, r = par[n] >= 0 (a unused) */
#define PIMPC_SET_BOX 0
#define PIMPC_SET_HALFSPACE 1
#define PIMPC_SET_HYPERPLANE 2
#define PIMPC_SET_SOC 3
#define PIMPC_SET_L1BALL 4

/* where a pointer lives */
#define PIMPC_MEM_HOST 0
#define PIMPC_MEM_DEVICE 1

/* iterate selectors for pimpc_get_iterates / pimpc_set_iterates */
#define PIMPC_IT_V 0      /* v_k        (copy of Bbar_k du_k)          */
#define PIMPC_IT_Z 1      /* z_{k+1}    (copy of xbar_{k+1}, in the box) */
#define PIMPC_IT_THETA 2  /* theta_k    scaled dual                    */
#define PIMPC_IT_BETA 3   /* beta_k     scaled dual                    */
#define PIMPC_IT_LAMBDA 4 /* lambda_k   scaled dual                    */
#define PIMPC_IT_DU 5     /* du_k of the last step 1 (nu per stage)    */
#define PIMPC_IT_XBAR 6   /* xbar_{k+1} of the last step 1             */

typedef struct pimpc_ctx_s *pimpc_ctx;

/*
 * Problem data, eqn. (1) (Section II) with W_u = R: the state weight Q
 * (C = I, W_y = Q) or the output form below, the velocity-form linear term
 * qbar of Theorem 2 and the input-rate weight W_du of the experiments
 * (Section V).
 *   count          number of instances (1 .. 65535; more: PIMPC_E_DIM)
 *   nx, nu, N      per-instance state/input sizes and horizon (count entries each)
 *   time_varying   0: one (A, B, e) per instance; 1: N stage copies per instance
 *   A, B           row-major nx*nx and nx*nu blocks (times N if time_varying)
 *   e              affine term e_k (nx, times N if time_varying), NULL = 0
 *   Q, R           nx*nx and nu*nu symmetric PSD weights per instance
 *   qbar           (nx+nu) linear cost term per instance, NULL = 0
 *   xmin, xmax     nx per instance; umin, umax nu per instance; +-INFINITY allowed
 *   Wdu            nu*nu symmetric PSD input-rate weight per instance (cost term
 *                  1/2 ||u_k - u_{k-1}||^2_Wdu), NULL = 0.  It changes only the
 *                  du cache: J_k = (Wdu / rho + Bbar_k' Bbar_k)^-1 Bbar_k'.
 *   xset, uset     per-instance PIMPC_SET_* kind of the X and U factors, NULL =
 *                  all boxes.  For a non-box factor the matching xmin/xmax (or
 *                  umin/umax) entries are ignored.  Non-box sets run without
 *                  a tape (the taped forward returns PIMPC_E_UNSUPPORTED).
 *   xset_par       (nx + 1) values per instance: (a, b) or (., r); may be NULL
 *   uset_par       (nu + 1) values per instance, likewise
 * Output form of eqn. (1), all optional (ny == NULL: C = I with W_y = Q and
 * r_y = 0; ru == NULL: r_u = 0).  The tracking cost
 * 1/2 ||C x_{k+1} - r_y||^2_Wy + 1/2 ||u_k - r_u||^2_R is folded into the
 * velocity-form weights at setup (constant terms dropped):
 *   Q <- Q + C' Wy C,  qbar_x <- qbar_x + C' Wy r_y,  qbar_u <- qbar_u + R r_u.
 *   ny             outputs per instance (count entries, each >= 0 and <= 32)
 *   C              ny*nx output matrix per instance (y = C x), row-major
 *   Wy             ny*ny symmetric PSD output weight per instance
 *   ry             ny output reference per instance, NULL = 0
 *   ymin, ymax     ny output bounds per instance, NULL = none; +-INFINITY
 *                  allowed.  A finite bound on output i needs row i of C to
 *                  select one state (one nonzero c_ij): it then tightens the
 *                  box of x_j to [ymin_i, ymax_i] / c_ij, so X stays a box
 *                  (the output constraints of the experiments of Section V
 *                  are of this kind).  A finite bound on a row that mixes
 *                  states returns PIMPC_E_UNSUPPORTED; an empty intersection
 *                  PIMPC_E_ARG.  The x factor must then be a box.
 *   ru             nu input reference per instance (W_u = R), NULL = 0
 * With the output form Q may be NULL (= 0).
 */
typedef struct {
    int32_t count;
    const int32_t *nx;
    const int32_t *nu;
    const int32_t *N;
    int32_t time_varying;
    const double *A;
    const double *B;
    const double *e;
    const double *Q;
    const double *R;
    const double *qbar;
    const double *xmin;
    const double *xmax;
    const double *umin;
    const double *umax;
    const double *Wdu;
    const int32_t *xset;
    const int32_t *uset;
    const double *xset_par;
    const double *uset_par;
    const int32_t *ny;
    const double *C;
    const double *Wy;
    const double *ry;
    const double *ymin;
    const double *ymax;
    const double *ru;
} pimpc_problem;

/*
 * Options (Algorithm 1 inputs).
 *   rho          ADMM penalty (> 0), fixed for the context's life
 *   max_iter     K_max (>= 1)
 *   eps          stop when c^{i+1} <= eps (step 5); <= 0 runs exactly max_iter
 *   check_every  residual cadence (>= 1) when eps > 0
 *   precision    PIMPC_FP32 or PIMPC_FP64 (iteration arithmetic)
 *   accel        0 = plain ADMM; 1 = restart acceleration (steps 6-7)
 *   eta          restart threshold (Algorithm 1 uses 0.999)
 *   warm_start   1 = start from the previous solve's iterate (unshifted)
 *   ckpt_every   > 0: the forward records a tape for pimpc_backward (FP32,
 *                time-invariant, box sets, plain ADMM, eps <= 0).  k >= 2:
 *                the iterate entering every k-th iteration (5 nb floats a
 *                stage), and the backward re-runs each k-step segment from it
 *                into a k-step record buffer; 1: the forward itself writes
 *                the backward's record of every iteration (2 nb + nx + 1
 *                floats a stage and iteration, max_iter of them: 24.8 KB a
 *                stage for nx = 8, nu = 3 and 200 iterations) and the
 *                backward re-runs nothing
 *   schedule     batch schedule: 0 = autotune (measured at setup), k = 1..14
 *                a fixed candidate: bin claiming by atomic counter (1, 2, 5,
 *                6, 7, 9, 11, 12, 14), static striding (3, 13) or one
 *                workgroup per bin (4, 8, 10), on 4 streams (2: 1 stream,
 *                6: 3, 7: 2), class launches whole or split in two (5-8),
 *                grids of all resident workgroups or half (11, 13, 14) or a
 *                quarter (12) of them; when fixed, launches are assigned to
 *                streams by FMA count
 *   family       kernel family: PIMPC_FAMILY_AUTO (choose as described at the
 *                top of this file), PIMPC_FAMILY_LANE or PIMPC_FAMILY_ROW
 *                (PIMPC_E_UNSUPPORTED when that family cannot serve an
 *                instance)
 */
typedef struct {
    double rho;
    int32_t max_iter;
    double eps;
    int32_t check_every;
    int32_t precision;
    int32_t accel;
    double eta;
    int32_t warm_start;
    int32_t ckpt_every;
    int32_t schedule;
    int32_t family;
} pimpc_options;

#define PIMPC_FAMILY_AUTO 0
#define PIMPC_FAMILY_LANE 1
#define PIMPC_FAMILY_ROW 2

/* Per-instance result of a solve (c, r_prim, r_dual of the last residual check). */
typedef struct {
    int32_t iters;
    int32_t restarts;
    double c;       /* c^{i+1} of Algorithm 1 step 4                      */
    double r_prim;  /* ||s^{i+1} - s^i||_inf   (primal residual)         */
    double r_dual;  /* rho ||F'G(q^{i+1}-q^i)||_inf   (dual residual)    */
    int32_t status; /* PIMPC_OK; PIMPC_E_NOT_PSD when a stage matrix of the
                       instance's last factorisation (setup, linearize or
                       set_params_dev) was not SPD: its iterates are then
                       meaningless; PIMPC_E_NONFINITE when an iterate became
                       NaN/Inf; PIMPC_E_HIP when a row-family wait between
                       workgroups gave up                                  */
    int32_t pad;
} pimpc_info;

/* Fill `o` with defaults: rho 1, 200 iterations, eps 0, check_every 1, FP32,
 * plain ADMM, eta 0.999, cold start, no tape, autotuned schedule. */
void pimpc_default_options(pimpc_options *o);

/*
 * Validate the problem on the host (sizes, finiteness, xmin <= xmax, Q and R
 * symmetric PSD, rho > 0), allocate device memory, upload the data and run
 * the FP64 stage factorisation (Algorithm 1 "cache": J_k and H_k, proof of
 * Theorem 2).  `hip_stream` (hipStream_t or NULL for the default stream) is
 * the stream every later call of this context runs on.  On success *out is
 * a new context; on error *out is NULL.
 */
int32_t pimpc_setup(pimpc_ctx *out, const pimpc_problem *prob, const pimpc_options *opts,
                    void *hip_stream);

/*
 * Replace the stage matrices of every instance (same packing as setup's A, B,
 * e; `mem_kind` says whether the pointers are host or device memory, double
 * precision either way) and re-run the FP64 stage factorisation.  Iterates are
 * kept, so the next solve can warm-start: this is the construction-free
 * update of online-linearised / RTI NMPC (Sections I and II).  e may be NULL.
 * Synchronous.  Device pointers are read by a kernel on the context's stream
 * (so they may be produced by earlier work on that stream, with no host round
 * trip); host pointers are validated before anything changes.  Returns
 * PIMPC_E_NONFINITE for NaN/Inf data and PIMPC_E_NOT_PSD when a stage matrix
 * is not SPD; after such a failure of a device import the context holds the
 * rejected data, and its solves report PIMPC_E_NOT_PSD (or non-finite
 * iterates) until a valid linearize.  Invalidates the tape (pimpc_tape_id).
 */
int32_t pimpc_linearize(pimpc_ctx ctx, const double *A, const double *B, const double *e,
                        int32_t mem_kind);

/*
 * Run Algorithm 1 on every instance.  Host pointers, synchronous.
 *   x0      x(t), packed (sum of nx)
 *   u_prev  u(t-1), packed (sum of nu), NULL = 0
 *   u0_out  u_prev + du_0 of the last step 1 (sum of nu); may be NULL
 *   info    count entries; may be NULL
 */
int32_t pimpc_solve(pimpc_ctx ctx, const double *x0, const double *u_prev, double *u0_out,
                    pimpc_info *info);

/*
 * Asynchronous batched solve on `hip_stream` with device pointers whose
 * element type is the context's precision (float for PIMPC_FP32, double for
 * PIMPC_FP64).  Same packing as pimpc_solve.  On a created (non-NULL)
 * stream the launch sequence is captured in a hipGraph on the first call for
 * a given argument set and replayed afterwards; on the NULL stream it is
 * launched directly.  info_dev may be NULL.  The caller synchronises.
 * With opts.ckpt_every > 0 the forward records the tape pimpc_backward uses.
 */
int32_t pimpc_solve_batch(pimpc_ctx ctx, const void *x0_dev, const void *uprev_dev,
                          void *u0_dev, pimpc_info *info_dev, void *hip_stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve as pimpc_solve_batch (same arguments, kernels and results), launched
 * directly on `hip_stream` (never captured into a graph by the library).
 * Every per-call buffer the kernels use -- the kernel arguments, the lane
 * classes' bin counters, the row family's halo mailboxes, abort flag and
 * reduction words -- lives in one static device array of
 * PIMPC_NOALLOC_SCRATCH_BYTES per GPU (held from library load until the
 * process ends) instead of memory the library allocates; the call makes no
 * hipMalloc, hipFree or other allocating call.  What must start at zero is
 * cleared by the call itself (with fill kernels).  Contexts whose per-call
 * scratch exceeds the array (large row-family horizons) get PIMPC_E_DIM;
 * a context used on another device than the one current at its setup gets
 * PIMPC_E_STATE.  All calls on one GPU share the array, so calls that overlap
 * in time on one GPU race (whatever their contexts or streams): order them,
 * e.g. on one stream.
 */
#define PIMPC_NOALLOC_SCRATCH_BYTES (4u << 20)
int32_t pimpc_solve_batch_noalloc(pimpc_ctx ctx, const void *x0_dev, const void *uprev_dev,
                                  void *u0_dev, pimpc_info *info_dev, void *hip_stream);

/*
 * Replace per-instance time-invariant parameters from device memory in the
 * context's precision and re-run the factorisation on the device:
 *   A [count][nx][nx], B [count][nx][nu], Qdiag [count][nx], Rdiag [count][nu]
 * (Q and R become diagonal).  Requires equal nx and nu across instances and a
 * time-invariant context.  Asynchronous on `hip_stream`: a stage matrix that
 * is not SPD (e.g. a negative Qdiag) is not reported here but by every later
 * solve of that instance, as status PIMPC_E_NOT_PSD in its info record (and
 * as the return value of pimpc_solve).  Invalidates the tape.
 */
int32_t pimpc_set_params_dev(pimpc_ctx ctx, const void *A, const void *B, const void *Qdiag,
                             const void *Rdiag, void *hip_stream);

/*
 * Id of the tape the context holds: each taped forward (a solve with
 * opts.ckpt_every > 0) records a new tape with a new id (1, 2, ...); a later
 * taped forward, pimpc_linearize or pimpc_set_params_dev replaces or
 * invalidates it.  0 when there is none (or ctx is NULL).
 */
uint64_t pimpc_tape_id(pimpc_ctx ctx);

/*
 * Reverse mode through the unrolled iterations of the taped forward whose
 * pimpc_tape_id() was `tape_id` (the differentiable layer; the adjoint of
 * Algorithm 1 steps 1-3, not in the paper).  PIMPC_E_STATE when the context
 * has no tape (opts.ckpt_every = 0, no taped solve yet) or when `tape_id` is
 * not the current tape (another taped forward or a parameter update came
 * after it: its gradients can no longer be formed).
 * Given dL/du0 (device, context precision, packed like u0: sum of nu),
 * writes per instance, in instance order, dL/dx0 and dL/dQdiag (packed like
 * x0: sum of nx), dL/dRdiag (sum of nu), dL/dA (one nx x nx block per
 * instance, row-major, sum of nx^2) and dL/dB (one nx x nu block, sum of
 * nx nu): count x nx, count x nx x nx ... when all instances have the same
 * shape.  Any output may be NULL.  The loss sees u0 = du_0 of the K-th step 1, a cold start and
 * u_prev = 0.  Asynchronous on `hip_stream`.
 */
int32_t pimpc_backward(pimpc_ctx ctx, uint64_t tape_id, const void *dL_du0_dev, void *dx0, void *dQdiag,
                       void *dRdiag, void *dA, void *dB, void *hip_stream);

/*
 * Copy an iterate of every instance to the host as double, packed by
 * instance, stage-major: which = PIMPC_IT_V..LAMBDA or PIMPC_IT_XBAR give
 * N*(nx+nu) values per instance, PIMPC_IT_DU gives N*nu.  Synchronous.
 */
int32_t pimpc_get_iterates(pimpc_ctx ctx, int32_t which, double *out);

/* Overwrite one of v, z, theta, beta, lambda (same packing as get) so that
 * the next warm-started solve starts from it.  Synchronous. */
int32_t pimpc_set_iterates(pimpc_ctx ctx, int32_t which, const double *in);

/* Free the context and all its device memory.  NULL is a no-op. */
void pimpc_destroy(pimpc_ctx ctx);

/* Text of the last error of `ctx`, or of the calling thread's last failed
 * pimpc_setup when ctx is NULL.  Never NULL; valid until the next call. */
const char *pimpc_last_error(pimpc_ctx ctx);

/* PIMPC_VERSION of the built library. */
int32_t pimpc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PIMPC_H */
