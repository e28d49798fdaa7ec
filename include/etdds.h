/*
 * etdds: Pade-based dimension-split ETD2RK time stepping (ETD2RK-DS) for
 * u_t - kappa Lap(u) + q u = f(x, t, u) on a 2-D rectangle or 3-D box with
 * homogeneous Dirichlet data (paper Sec. 1), in the Sylvester/spectral form
 * of Sec. 3.3.2, on AMD Instinct MI355X (gfx950).
 *
 * One step (Sec. 3.1, 2-D and 3-D equations; Algorithms 1-2) applies, per
 * direction d, the rational operators Q_l(tau A_d) of the P_{0,2} family
 * (or, with pade = 4, the P_{0,4} family of Sec. 5) to the grid through the
 * reusable eigendecomposition A_d = P_d D_d P_d^T: a dense mode-d product
 * with P_d, a Hadamard scaling by the rational factor of tau*lambda, and the
 * product with P_d back.  The reaction f is evaluated inside the stage
 * kernels.  All arithmetic of a step runs in HIP kernels on the device.
 *
 * Conventions shared by every call:
 *  - n[d] counts interior points; h_d = (hi[d]-lo[d])/(n[d]+1) (Sec. 2.1).
 *  - A field is a contiguous device array ncomp x nz x ny x nx, x fastest
 *    (the vectorisation order of Sec. 2.1), nz = 1 in 2-D.  Its element type
 *    is double for ETD_FP64, ETD_FP64_FP32 and ETD_FP64_BF16X6 and float for
 *    ETD_FP32 and ETD_BF16X6.
 *  - Device memory belongs to the caller: the field and one workspace buffer
 *    of etd_plan_workspace_bytes() bytes (256-byte aligned).  The library
 *    allocates no device memory.  A plan owns host memory only.  Every call
 *    that takes a plan's workspace (advance, adjoint, compare, autotune,
 *    graph capture) requires the one etd_plan_upload last filled for that
 *    plan, else it returns ETD_EWORKSPACE before enqueueing anything.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Device work is enqueued asynchronously on it, in stream order.
 *  - Every call returns an etd_status.  Argument errors are detected on the
 *    host before anything is enqueued and leave all buffers untouched.  HIP
 *    launch errors return ETD_EHIP.  etd_last_error() gives a thread-local
 *    message for the most recent failure.
 *  - Calls on different plans or batches may run on different host threads
 *    at once (the library's per-kernel launch caches are thread-safe); calls
 *    on one plan or batch must not overlap.
 */
#ifndef ETDDS_H
#define ETDDS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    ETD_OK = 0,
    ETD_EINVAL = -1,        /* invalid argument */
    ETD_EUNSUPPORTED = -2,  /* valid problem the library cannot run (size limits) */
    ETD_EWORKSPACE = -3,    /* workspace missing, misaligned or too small */
    ETD_EHIP = -4,          /* HIP runtime error */
    ETD_ENONFINITE = -5     /* etd_compare found NaN or Inf in the field */
} etd_status;

typedef enum {
    ETD_FP64 = 0,   /* FP64 state, FP64 MFMA mode products */
    ETD_FP32 = 1,   /* FP32 state, FP32 MFMA mode products */
    ETD_BF16X6 = 2, /* FP32 state; mode products as six BF16 MFMA terms
                       (hi/mid/lo splits of both operands), FP32 accumulation */
    ETD_FP64_FP32 = 3,   /* FP64 state, diagonals and epilogues; FP32 MFMA mode
                            products (P held in FP32, the other operand rounded
                            to FP32 as it is read), FP32 accumulation */
    ETD_FP64_BF16X6 = 4  /* FP64 state, diagonals and epilogues; split-BF16
                            mode products as in ETD_BF16X6 (the other operand
                            rounded to FP32, then split) */
} etd_precision;

typedef enum {
    ETD_RXN_NONE = 0,        /* f = 0 */
    ETD_RXN_LINEAR = 1,      /* f = c u                                  p0 = c */
    ETD_RXN_FISHER = 2,      /* f = a u (1-u)                            p0 = a */
    ETD_RXN_ALLEN_CAHN = 3,  /* f = u - u^3 */
    ETD_RXN_AC_MMS = 4,      /* f = u(1-u^2) + psi(x,t), psi chosen so that
                                e^{-lam t} prod_d sin(pi (x_d-lo_d)/L_d) solves
                                the equation (Example 5.1); p0 = lam, p1 != 0
                                uses the discrete Laplacian eigenvalue */
    ETD_RXN_SATURATING = 5,  /* f = rho u/(1-u) (Example 5.2)           p0 = rho */
    ETD_RXN_FHN_CUBIC = 6,   /* fu = u(1-u)(u-a) - v, fv = eps(u - g v)  p = a, eps, g */
    ETD_RXN_FHN_CLASSIC = 7  /* fu = u - u^3/3 - v, fv = eps(u - alpha v)
                                (Example 5.3)                            p = eps, alpha */
} etd_reaction;

typedef struct {
    int dim;               /* 2 or 3 */
    int n[3];              /* interior points in x, y, z (n[2] ignored in 2-D) */
    double lo[3], hi[3];   /* box (hi > lo) */
    int ncomp;             /* 1, or 2 for the FitzHugh-Nagumo reactions */
    double kappa[2];       /* diffusivity per component, >= 0 */
    double q;              /* potential >= 0, q/dim per direction (Sec. 2.1) */
    double tau;            /* time step > 0; T = nsteps*tau (Sec. 2.2) */
    int rxn;               /* etd_reaction */
    double rxn_param[8];
    int pade;              /* 2: P_{0,2} family (Sec. 3.1); 4: P_{0,4} family (Sec. 5);
                              0: exact exponentials, Q_1..Q_3 = e^{-z}, phi_1, phi_2
                              (the fully discrete scheme of Sec. 2.2) */
    int precision;         /* etd_precision */
} etd_problem;

typedef struct etd_plan etd_plan;

/* Build a plan on the host (Sec. 3.4, steps 1-2 of Algorithms 1-2): the
 * closed-form eigenpairs of every A_d and the rational factors of tau*lambda,
 * computed in FP64.  *out receives a new plan (free with etd_plan_destroy).
 * ETD_EINVAL on a malformed problem; ETD_EUNSUPPORTED when a padded grid
 * direction exceeds 1024 points or the stage tiles exceed the on-chip limits
 * (FP64 tiles of one component hold extents up to 576). */
etd_status etd_plan_create(const etd_problem* prob, etd_plan** out);

/* Bytes of device workspace the plan needs: eigenvector tables, rational
 * factors and the stage buffers (five padded fields) and reduction scratch. */
etd_status etd_plan_workspace_bytes(const etd_plan* plan, size_t* bytes);

/* Copy the plan's tables into the workspace (asynchronous on `stream`; the
 * plan's host tables stay valid until destroy).  Must precede etd_advance
 * with the same workspace.  ETD_EWORKSPACE if bytes is too small or the
 * pointer is not 256-byte aligned. */
etd_status etd_plan_upload(const etd_plan* plan, void* workspace_dev, size_t bytes, void* stream);

/* Advance the field u_dev (device, layout above, updated in place) by nsteps
 * steps from time t0 (the time argument of f).  nsteps = 0 is a no-op.
 * Asynchronous on `stream`.  ETD_EWORKSPACE unless workspace_dev is the
 * workspace the plan was last uploaded to (etd_plan_upload records it; a
 * later upload of another plan to the same memory takes it over). */
etd_status etd_advance(const etd_plan* plan, void* u_dev, double t0, int nsteps,
                       void* workspace_dev, void* stream);

/* Validation reductions over the interior (all components), the ingredients
 * of Sec. 5's error measures (the max-norm E(N) over grid points and
 * components, and the relative 2-norm error out[0]/out[1]): out[0] =
 * ||a - b||_2, out[1] = ||b||_2, out[2] = max |a - b|, out[3] = number of
 * non-finite entries of a.  a and b are fields of the plan's layout and
 * element type (device).  Entries where a is not finite are left out of
 * out[0] and out[2] (and counted in out[3]); out[1] takes every entry of b.
 * Accumulates in FP64 in a fixed order (repeatable).  Synchronises `stream`
 * to return the result.  Returns ETD_ENONFINITE (with out filled) when a
 * holds NaN or Inf; ETD_EWORKSPACE as etd_advance. */
etd_status etd_compare(const etd_plan* plan, const void* a_dev, const void* b_dev, double out[4],
                       void* workspace_dev, void* stream);

/* etd_compare for callers that cannot allocate device memory or hand over a
 * workspace (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation).  Computes the same four values as etd_compare, with
 * the same kernels in the same order (bit-identical results), but:
 *  - it needs no workspace and no etd_plan_upload: the per-workgroup partial
 *    sums go to a fixed array inside the library's device code (1024 x 4
 *    doubles, 32 KB per GPU, held until the process ends).  The reduction
 *    strides over the field, so fields of any size fit and no size is refused;
 *  - out_dev is a device array of 4 doubles that receives out[0..3]; nothing
 *    is copied to the host and `stream` is not synchronised, so the call can
 *    be captured into a graph; non-finite entries are reported in out_dev[3]
 *    only (the return value is ETD_OK once the work is enqueued).
 * Every call on one GPU uses that GPU's one array and overwrites all of it
 * before reading it: calls that overlap on one GPU (other streams or host
 * threads) race and must be serialised by the caller.  ETD_EINVAL on NULL
 * arguments; ETD_EHIP on a launch error. */
etd_status etd_compare_noalloc(const etd_plan* plan, const void* a_dev, const void* b_dev, double* out_dev,
                               void* stream);

/* The problem the plan was created from (Sec. 1: dimension, grid, box,
 * coefficients, time step, source and precision), copied to *out; lets a
 * caller check a field's size and element type against the plan. */
etd_status etd_plan_problem(const etd_plan* plan, etd_problem* out);

/* Host copies of the plan's FP64 tables, for inspection and tests (no device
 * involvement).  which: 0 = eigenvalues lambda_j of A_d (component comp),
 * 1 = eigenvector matrix P_d (n_d x n_d, row-major), 2/3/4 = the rational
 * factors Q_1, Q_2, Q_3 (R_1..R_3, or e^{-z}, phi_1, phi_2) at tau*lambda_j, 5/6/7 = the
 * increments Q_1 - 1, Q_2 - 1, Q_3 - 1/2 the kernels apply.  count is the capacity
 * of out in doubles; ETD_EINVAL if too small. */
etd_status etd_plan_table(const etd_plan* plan, int which, int d, int comp, double* out, size_t count);

/* Adjoint of etd_advance (reverse mode), for the gradient of a scalar loss
 * L(U_N), U_N the field after nsteps steps from u0_dev at time t0.  Given
 * ubar_final_dev = dL/dU_N (device, field layout), writes dL/du0 to ubar0_dev
 * and, on the host, grad[c] = dL/dkappa_c for c < ncomp and grad[ncomp] =
 * dL/dq.  Each stage's transpose is applied in reverse order (the step of
 * Sec. 3.1 with symmetric, commuting directional operators; the reaction
 * enters through its pointwise Jacobian); parameter derivatives use
 * dQ_l(tau lambda)/dlambda and dlambda/dkappa, dlambda/dq.  Forward states
 * come from checkpoints every K steps held in the adjoint workspace (256-byte
 * aligned, caller-owned, adjoint_bytes long); each segment of K steps is
 * replayed once, keeping every step's stage fields, so the forward work is
 * (nsteps - K) + nsteps steps.  etd_adjoint takes the longest K whose layout
 * fits adjoint_bytes: etd_adjoint_workspace_bytes is the smallest workspace
 * (K = ceil(sqrt(nsteps))), etd_adjoint_workspace_bytes_segment the size for
 * a given K between that and nsteps (ETD_EINVAL outside), and K = nsteps (one
 * forward pass; about six fields per step in 3-D, four in 2-D) is the
 * fastest.  The plan's workspace is used as scratch.  Synchronises `stream`.  Gradients
 * are summed in FP64 in a fixed order.  ETD_EUNSUPPORTED when the adjoint's
 * tiles exceed the on-chip limits: they hold four fields of one component,
 * so padded extents up to 288 with an FP64 state and 576 with an FP32 one
 * (and the forward x tile of all components must fit, as the replayed steps
 * keep W). */
etd_status etd_adjoint_workspace_bytes(const etd_plan* plan, int nsteps, size_t* bytes);
etd_status etd_adjoint_workspace_bytes_segment(const etd_plan* plan, int nsteps, int segment, size_t* bytes);
etd_status etd_adjoint(const etd_plan* plan, const void* u0_dev, double t0, int nsteps, const void* ubar_final_dev,
                       void* ubar0_dev, double* grad, void* workspace_dev, void* adjoint_workspace_dev,
                       size_t adjoint_bytes, void* stream);

/* Stage timing (diagnostics).  While enabled, etd_advance records a HIP event
 * on its stream before and after every stage kernel.  etd_timing_read waits
 * for the last recorded event and returns, per stage kind (0 = first outer
 * stage: z in 3-D, y in 2-D, with f(t_n, U) fused; 1 = middle outer stage, y
 * in 3-D; 2 = fused x stage), the summed milliseconds and the number of
 * launches since the previous read or enable, then resets the counters.
 * Enabling or disabling also resets them.  Not thread-safe per plan. */
etd_status etd_timing_enable(etd_plan* plan, int enable);
etd_status etd_timing_read(etd_plan* plan, double ms[3], long long counts[3]);

/* Tile shapes of the stage kernels (how the mode products of Sec. 3.4 are
 * blocked on the device; they never change a result, only its speed).  Per
 * direction d (0 = x, 1 = y, 2 = z), tiles[2d] = 16-row blocks of each product
 * per wave and tiles[2d+1] = 16-column (outer stages) or 16-line (x stage)
 * blocks per workgroup; zeros for directions beyond dim.  Rows per wave are
 * 1, 2 or 4, and 8 for FP32-state precisions: with one block, or, in the x
 * direction of one-component systems whose lines are too long for a
 * two-array tile of two blocks (from 640 padded points on), with two blocks
 * in a tile that holds one array; a tile has NP / (16 rows) waves, at most 16.
 * etd_plan_tiles reports the shapes in use.  etd_plan_set_tiles selects them
 * ((0, 0) restores the built-in default of a direction); ETD_EUNSUPPORTED if a
 * shape is not valid there (wave count, LDS, line count), leaving the plan
 * unchanged.  etd_plan_autotune times every valid shape of every stage on the
 * uploaded workspace (its stage buffers are scratch) with HIP events on
 * `stream`, keeps the fastest, and synchronises.  Two-component systems whose
 * joint tile exceeds the LDS keep their one split shape. */
etd_status etd_plan_tiles(const etd_plan* plan, int tiles[6]);
etd_status etd_plan_set_tiles(etd_plan* plan, const int tiles[6]);
etd_status etd_plan_autotune(etd_plan* plan, void* workspace_dev, void* stream);

/* How etd_advance launches the stages of Algorithm 2 (speed only: shapes and
 * schedules give identical results, except that the manufactured Allen-Cahn
 * source's time factor e^{-lambda t} is formed on the device by the resident
 * schedule and on the host otherwise, which may differ in the last bit).
 *  - ETD_SCHEDULE_STAGES: one launch per stage and step (two-dimensional grids
 *    with at least 128 blocks of 64 y rows x 16 x columns run every mode
 *    product as a launch of its own).
 *  - ETD_SCHEDULE_RESIDENT: all steps of the call in ONE cooperative launch
 *    whose workgroups run the stages' tiles in turn, with a grid-wide barrier
 *    between stages.  Applies to grids whose directions share one padded
 *    extent of at most 128 points.  etd_advance returns ETD_EUNSUPPORTED on a
 *    stream that is capturing a graph; stage timing records nothing for it.
 *    A cooperative launch costs tens of microseconds of host time, and on
 *    small grids per-stage launches of one-block tiles are as fast, so it is
 *    never chosen by AUTO.
 *  - ETD_SCHEDULE_AUTO (default): STAGES.
 * etd_plan_set_schedule: ETD_EINVAL for an unknown value, ETD_EUNSUPPORTED for
 * RESIDENT on a plan it does not apply to (the plan is then unchanged).
 * etd_plan_schedule: the schedule (STAGES or RESIDENT) that etd_advance takes
 * on a stream that is not capturing.  Tile shapes set with etd_plan_set_tiles
 * apply to the STAGES schedule only. */
typedef enum { ETD_SCHEDULE_AUTO = 0, ETD_SCHEDULE_STAGES = 1, ETD_SCHEDULE_RESIDENT = 2 } etd_schedule;
etd_status etd_plan_set_schedule(etd_plan* plan, int schedule);
etd_status etd_plan_schedule(const etd_plan* plan, int* schedule);

/* Batches: `count` (1..4096) independent problems advanced together.  They
 * must share dim, ncomp and precision; extents, box, coefficients, time step,
 * reaction and Pade order are per instance.  Instances of one padded shape
 * form a group whose every stage runs as one persistent launch over all of
 * its instances' tiles (a descriptor table in the workspace gives each
 * instance's buffers and tables); groups run on streams of their own,
 * created by the first upload, forked from and joined back to `stream`.
 * Instances of equal extent share one eigenvector table; an instance that
 * finds every direction's table in an earlier instance holds no copy.
 *  - create: ETD_EINVAL as etd_plan_create (message names the instance) or
 *    when instances differ in dim/ncomp/precision; ETD_EUNSUPPORTED for a
 *    two-component instance whose joint tile exceeds the LDS.
 *  - upload: tables and descriptors into one caller-owned workspace of
 *    etd_batch_workspace_bytes bytes (256-byte aligned); synchronises
 *    `stream`.  Descriptors hold device addresses, so advance, autotune and
 *    capture take exactly the uploaded workspace (else ETD_EWORKSPACE).
 *  - advance: u_dev[i] (a host array of count device pointers) is instance
 *    i's field, updated in place; each instance's time is t0 + k tau_i.
 *  - autotune: as etd_plan_autotune, per group (synchronises).
 *  - tiles: the shapes of instance i's group; groups: number of groups.
 * Calls on one batch must not overlap. */
typedef struct etd_batch etd_batch;
etd_status etd_batch_create(const etd_problem* probs, int count, etd_batch** out);
etd_status etd_batch_workspace_bytes(const etd_batch* batch, size_t* bytes);
etd_status etd_batch_upload(etd_batch* batch, void* workspace_dev, size_t bytes, void* stream);
etd_status etd_batch_advance(etd_batch* batch, void* const* u_dev, double t0, int nsteps, void* workspace_dev,
                             void* stream);
etd_status etd_batch_autotune(etd_batch* batch, void* workspace_dev, void* stream);
etd_status etd_batch_tiles(const etd_batch* batch, int instance, int tiles[6]);
etd_status etd_batch_groups(const etd_batch* batch, int* groups);
etd_status etd_batch_destroy(etd_batch* batch);

/* HIP graphs: the device work of one etd_advance (or etd_batch_advance) call
 * captured from `stream` (which must not be the null stream) into an
 * executable graph, bound to the given field pointers, workspace, t0 and
 * nsteps.  Nothing runs during capture.  etd_graph_launch replays that work
 * on any stream: each replay advances the fields by nsteps steps again, with
 * the captured times (so time-dependent sources see t0 .. t0 + nsteps tau on
 * every replay).  The captured work contains kernels only (no memset or copy
 * nodes).  A plan graph keeps the tile shapes it was captured with.  A batch
 * graph reads the batch's descriptors at replay, so after etd_batch_autotune,
 * a new etd_batch_upload or etd_batch_destroy it refuses to launch
 * (ETD_EINVAL; capture again).  Graphs own host memory only. */
typedef struct etd_graph etd_graph;
etd_status etd_graph_capture(const etd_plan* plan, void* u_dev, double t0, int nsteps, void* workspace_dev,
                             void* stream, etd_graph** out);
etd_status etd_batch_graph_capture(etd_batch* batch, void* const* u_dev, double t0, int nsteps,
                                   void* workspace_dev, void* stream, etd_graph** out);
etd_status etd_graph_launch(etd_graph* graph, void* stream);
etd_status etd_graph_destroy(etd_graph* graph);

/* Free the plan (host memory and any timing events). */
etd_status etd_plan_destroy(etd_plan* plan);

const char* etd_status_string(etd_status s);
const char* etd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
