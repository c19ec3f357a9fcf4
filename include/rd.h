/*
 * rd.h -- C ABI of librd, the MI355X (gfx950) Radau5 reaction-step library.
 *
 * Operation.  The reaction substep R_dt of the Strang splitting scheme
 * U_{n+1} = R_{Δt/2} D_{Δt} R_{Δt/2} U_n (Descombes et al., §2.1): every cell
 * (leaf of the adapted grid) integrates its own stiff system du/dt = f(u) over
 * [0, dt] with Radau5 (paper §1, footnote: implicit fifth-order Runge-Kutta,
 * A- and L-stable, adaptive time step), i.e. the 3-stage Radau IIA method with a
 * simplified Newton iteration on the stage equations, solved through one real
 * and one complex m x m linear system, an embedded error estimate, and
 * step-size control (Hairer & Wanner, Solving ODEs II, §IV.8).  Cells are
 * independent (paper §2.1: as many independent problems as grid nodes); the
 * number of sub-steps and Newton iterations differs from cell to cell (paper
 * Appendix A), which is why the default schedule is a persistent kernel whose
 * lanes claim new cells as soon as theirs finish.
 *
 * Layout.  Structure of arrays (paper §3.2, one contiguous array per unknown):
 * states[i * n_cells + c] is species i of cell c, float64.  The update is in
 * place: on return (or completion, for async calls) states holds u(dt).
 * Optional stats: int32, [RD_NSTATS][n_cells], rows
 *   0 status, 1 nstep (step attempts), 2 naccept, 3 nreject (error-test
 *   rejections and Newton failures), 4 nfev (f evaluations), 5 njac,
 *   6 ndec (factorizations of the iteration matrices), 7 nsol (linear solves),
 *   8 nnewt (Newton iterations).
 * nfev is the paper's per-node complexity measure (Appendix A).
 *
 * Ownership.  states and stats are DEVICE pointers owned by the caller (for
 * instance torch tensors); the library never frees them and they must stay
 * valid and untouched until the call completes.  rd_model.params is a HOST
 * pointer, read during the call only.  The library owns its workspace (claim
 * counters, model-parameter blocks, captured graphs), allocated lazily per
 * device and released at process exit.
 *
 * Errors.  >= 0: the number of cells whose per-cell status is nonzero (those
 * cells keep their last accepted state; the others are unaffected).  Per-cell
 * status: 1 MAXSTEPS, 2 H_TOO_SMALL, 3 SINGULAR (five singular factorizations
 * in a row), 4 NONFINITE, 5 NEWTON_FAIL (fixed-step mode only).
 * < 0: nothing was done: RD_EINVAL, RD_ENOMEM, RD_EDEVICE (a HIP error; text in
 * rd_last_error()), RD_ETOOBIG (request larger than a session's budget),
 * RD_ECLOSED (session destroyed), RD_ENOTFOUND (unknown request id).
 * n_cells == 0 is valid and does nothing.
 */
#ifndef RD_H
#define RD_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RD_OREGONATOR = 1, /* m = 3, params {eps, mu, f, q}: BZ model (paper §1, II):
                          a' = (-q a - a b + f c)/mu, b' = (q a - a b + b(1-b))/eps,
                          c' = b - c                                              */
    RD_KINETICS = 2,   /* m in {1..16}, params {K[m*m], G[m*m]} row-major:
                          f_i = sum_j K_ij u_j - u_i sum_k G_ik u_k              */
    RD_NAGUMO = 3,     /* m = 1, params {k}: f = k u^2 (1 - u) (paper §1, I)      */
    RD_LINEAR = 4,     /* m in {1..16}, params {K[m*m]}: f = K u (tests)         */
    RD_ROBERTSON = 5,  /* m = 3, params {k1, k2, k3}: Robertson kinetics (tests)  */
    RD_BYTECODE = 6    /* m in {1..16}: f supplied at run time as a register
                          program (below); its Jacobian is always taken by finite
                          differences                                             */
};

/*
 * Bytecode model.  params = [L, C, c_0 .. c_{C-1}, then L instructions of 4
 * doubles (op, d, a, b)], all integer-valued except the constants, over 64
 * FP64 registers r[0..64): r[0..m) hold u (read only), r[m..m+C) the
 * constants, the rest are temporaries.  Ops:
 *   1 ADD r[d] = r[a] + r[b]    2 SUB r[d] = r[a] - r[b]   3 MUL r[d] = r[a] * r[b]
 *   4 DIV r[d] = r[a] / r[b]    5 NEG r[d] = -r[a]         6 EXP r[d] = exp(r[a])
 *   7 LOG r[d] = log(r[a])      8 POW r[d] = r[a] ^ r[b]   9 OUT f_d = r[a]
 * Valid when 1 <= L <= 4096, m + C <= 64, d >= m + C for ops 1-8, every
 * register is written before it is read, and OUT writes each f_0 .. f_{m-1}
 * exactly once; anything else is RD_EINVAL.  Evaluation follows the program
 * order exactly (no reassociation, no contraction), so a program reproduces
 * a hand-written f operation for operation.
 */
enum { RD_BC_ADD = 1, RD_BC_SUB, RD_BC_MUL, RD_BC_DIV, RD_BC_NEG, RD_BC_EXP, RD_BC_LOG,
       RD_BC_POW, RD_BC_OUT };
#define RD_BC_REGS 64

enum { RD_JAC_ANALYTIC = 0, RD_JAC_FD = 1 };   /* jacobian */

enum { RD_FP64 = 0, RD_MIXED = 1 };            /* precision */
enum { RD_PERSISTENT = 0, RD_ONE_LAUNCH = 1 };  /* schedule  */

enum { RD_OK = 0, RD_MAXSTEPS = 1, RD_H_TOO_SMALL = 2, RD_SINGULAR = 3,
       RD_NONFINITE = 4, RD_NEWTON_FAIL = 5 };

enum { RD_EINVAL = -1, RD_ENOMEM = -2, RD_EDEVICE = -3, RD_ETOOBIG = -4,
       RD_ECLOSED = -5, RD_ENOTFOUND = -6 };

#define RD_NSTATS 9
#define RD_MAX_M 16

typedef struct {
    int32_t kind;          /* RD_OREGONATOR ... */
    int32_t m;             /* species per cell; must match the kind */
    const double* params;  /* HOST pointer, n_params doubles */
    int64_t n_params;
} rd_model;

typedef struct {
    int32_t precision;     /* RD_FP64 (default) or RD_MIXED: iteration-matrix LU
                              factors and triangular solves in FP32; f, residuals,
                              stage update, error estimate, control in FP64      */
    int32_t schedule;      /* RD_PERSISTENT (default) or RD_ONE_LAUNCH           */
    int32_t tol_transform; /* 1 (default): local tolerances rtol' = 0.1 rtol^(2/3),
                              atol' = rtol' atol / rtol; 0: use rtol, atol as given */
    int32_t max_steps;     /* step attempts per cell (default 100000)            */
    int32_t newton_max;    /* Newton iterations per attempt (default 7)          */
    int32_t fixed_steps;   /* 0 (default): adaptive; N > 0: N equal steps, no error
                              control (tests)                                      */
    double h0;             /* first trial step, 0 (default) means dt             */
    double h_min;          /* 0 (default) means 1e-14 dt                          */
    int32_t variant;       /* kernel variant: 0 = tuned default, else an id from
                              rd_variant_count/rd_variant_name                     */
    int32_t use_graph;     /* 1: capture the launch sequence of this shape in a
                              hipGraph on first use and replay it afterwards       */
    int32_t order;         /* claim order of the persistent schedule: 1 (default)
                              longest first, by a per-cell cost estimate (bucketed
                              scaled initial rate |f(u0)| dt / sc); 0 cell order  */
    int32_t jacobian;      /* RD_JAC_ANALYTIC (default) or RD_JAC_FD: forward
                              differences, column j = (f(u + d_j e_j) - f(u)) / d_j,
                              d_j = sqrt(uround max(1e-5, |u_j|)), m more f
                              evaluations per Jacobian (counted in nfev); every
                              model except RD_LINEAR with m > 4.  RD_BYTECODE
                              always uses RD_JAC_FD.                               */
    double* h_cells;       /* null (default), or DEVICE [n_cells] float64: per-cell
                              step size, in and out (warm start across split
                              steps).  In: a value > 0 is that cell's first trial
                              step (in place of h0, capped at dt).  Out: the step
                              size the controller held before it shortened the final
                              step to end at dt; dt/N in fixed-step mode; for a
                              failed cell the step size of its last attempt (0 if
                              none).  Not accepted by sessions.                     */
    int32_t session_streams; /* sessions only (rd_session_create): concurrent launch
                              streams, 0 (default) = 4, at most 64; ignored by the
                              direct entry points                                   */
} rd_options;

/* Fill *opts with the defaults above. */
void rd_default_options(rd_options* opts);

/*
 * Synchronous reaction step with default options on the current device's
 * null stream.  See the file comment for layout, ownership and errors.
 */
int64_t rd_reaction_step(double* states, int64_t n_cells, int32_t m, double dt,
                         double rtol, double atol, const rd_model* model);

/*
 * Full form.  opts nullable (defaults); stats nullable (DEVICE, [9][n_cells]
 * int32); hip_stream nullable (= null stream) is a hipStream_t.  async = 0:
 * returns after completion with the failed-cell count.  async = 1: returns 0
 * once the work is enqueued; completion is observed through the stream, and
 * failures through stats.
 */
int64_t rd_reaction_step_ex(double* states, int64_t n_cells, int32_t m,
                            double dt, double rtol, double atol,
                            const rd_model* model, const rd_options* opts,
                            int32_t* stats, void* hip_stream, int32_t async);

/*
 * For callers that cannot allocate memory (code under stream capture, tight
 * serving loops, harnesses that forbid allocation): rd_reaction_step_ex
 * without any device or pinned-host allocation, on any call including the
 * first.  Its scratch (the kernel's two counters, the model's parameter
 * block, the claim-order scratch of the persistent schedule) is a fixed
 * device array of rd_noalloc_scratch_bytes() bytes (about 21 MB) that every
 * device the library runs on holds until the process ends; requests of more
 * than RD_NOALLOC_MAX_CELLS cells are refused with RD_ETOOBIG.  All calls on
 * one device share that device's array, so calls that overlap on one device
 * (other streams, other threads) race: the caller orders them.  The model
 * parameters are copied asynchronously from a per-device host copy of the
 * block that the next call on the device overwrites.  opts->use_graph and
 * opts->h_cells must be unset (RD_EINVAL).  Arguments, layout, results and
 * the other errors as rd_reaction_step_ex; same kernels, bitwise the same
 * results.
 */
#define RD_NOALLOC_MAX_CELLS 4194304
int64_t rd_reaction_step_noalloc(double* states, int64_t n_cells, int32_t m,
                                 double dt, double rtol, double atol,
                                 const rd_model* model, const rd_options* opts,
                                 int32_t* stats, void* hip_stream, int32_t async);
size_t rd_noalloc_scratch_bytes(void);

/* ------------------------------------------------------------------------ */
/* The steps around the reaction step: diffusion and the Strang step on a     */
/* uniform grid (Descombes et al., §2.1: U_{n+1} = R_{dt/2} D_dt R_{dt/2} U_n).  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t dim;          /* 2 or 3                                               */
    int32_t nx, ny, nz;   /* cells per direction (nz = 1 when dim = 2); cell
                             c = x + nx (y + ny z) of the states array          */
    double h;             /* grid spacing, the same in every direction           */
    const double* diff;   /* HOST, m diffusion coefficients eps_i >= 0            */
} rd_grid;

/*
 * Diffusion step D_dt: dU/dt = A_eps U on the cell-centred grid, A_eps = eps_i
 * times the centred 5-point (2D) / 7-point (3D) Laplacian with homogeneous
 * Neumann boundaries (paper §2 and §1), advanced over dt by one step of the
 * explicit stabilised second-order Runge-Kutta-Chebyshev method RKC (damping
 * 2/13; Sommeijer, Shampine & Verwer 1997).  The paper's ROCK4 is of the same
 * family but needs tabulated coefficients; RKC's follow in closed form.
 * stages: 0 chooses s = 1 + floor(sqrt(1 + 1.54 dt rho)) (at least 2) from the
 * Gershgorin bound rho = 4 dim max(eps) / h^2; > 0 forces that count (>= 2).
 * states: DEVICE [m][nx*ny*nz], updated in place.  The library keeps four
 * state-sized work vectors per (device, stream).  Synchronous on hip_stream
 * (null = null stream).  Returns the number of stages used, or RD_EINVAL /
 * RD_ENOMEM / RD_EDEVICE.
 */
int64_t rd_diffusion_step(double* states, int32_t m, const rd_grid* grid, double dt,
                          int32_t stages, void* hip_stream);

/*
 * Strang step: R_{dt/2} (rd_reaction_step_ex with opts), then D_dt, then
 * R_{dt/2}, in place, synchronous on hip_stream.  stats nullable: DEVICE
 * [2][RD_NSTATS][n] int32, the counters of the first and second reaction half.
 * opts->h_cells must be null.  Returns the sum of the failed-cell counts of
 * the two reaction halves, or a negative error.  With opts->use_graph and a
 * non-null stream, the whole split step (both reaction halves with their
 * claim-order passes, the diffusion stages, the failure-count copies) is
 * recorded once as one hipGraph per (stream, states, stats, model constants,
 * options, grid, coefficients, dt) and replayed on later calls with the same
 * arguments; the graph keeps its own counters and pinned result words, so
 * replays of one graph must not overlap (the stream orders them).
 */
int64_t rd_strang_step(double* states, int32_t m, const rd_grid* grid, double dt, double rtol,
                       double atol, const rd_model* model, const rd_options* opts,
                       int32_t* stats, void* hip_stream);

/* ------------------------------------------------------------------------ */
/* Multiresolution leaf sets (Descombes et al., §2.2 after Cohen et al. 2003;  */
/* node keys §3.1) on the dyadic tree of [0,1]^d, d = 2, 3.                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t dim;          /* 2 or 3                                               */
    int32_t levels;       /* J >= 1, the finest level: 2^J cells per direction;
                             dim * J <= 30                                        */
    double eps;           /* threshold eps >= 0; level thresholds
                             eps_j = 2^((dim/2)(j - J)) eps                        */
    const double* scale;  /* HOST, m per-species detail scales s_i > 0, or null
                             (all 1)                                              */
    int32_t refine;       /* 0: compression only (a node has children when one of
                             them is significant); 1: also refine every node below
                             the finest level whose own detail is significant
                             (§2.2; children with predicted values)               */
} rd_mra_params;

/*
 * Leaf set of the graded tree built from a field on the finest level: node
 * values by projection (average of the 2^dim children); details d = u -
 * prediction, the prediction being the third-order centred interpolation
 * (l = 1) applied as a tensor product one direction at a time, with even
 * reflection at the domain edge; a node gets children when one of them has
 * (1/m) sum_i (d_i / s_i)^2 >= eps_j^2 (and, with params->refine, when its
 * own detail does); grading: a node with children makes the parents of its
 * 3^dim neighbours get children (finest to coarsest).
 * fine: DEVICE [m][2^(dim J)] float64, x fastest (cell x + N (y + N z)).
 * Output in Morton order of the leaves: keys DEVICE [n_leaves] uint64 (the
 * level-j Morton index, bits of x, y[, z] interleaved with x most significant,
 * left-aligned in bits 63..16; the level in bits 15..12; bits 11..0 zero) and
 * values DEVICE [m][n_leaves] (cell averages, packed with stride n_leaves),
 * written only when n_leaves <= capacity (values must hold m * capacity
 * doubles).  level_counts: HOST [J + 1] or null, leaves per level (when
 * written).  Synchronous.  Returns n_leaves, or RD_EINVAL / RD_ENOMEM /
 * RD_EDEVICE.  Workspace (the whole pyramid) is kept per (device, stream).
 */
int64_t rd_mra_leaves(const double* fine, int32_t m, const rd_mra_params* params,
                      uint64_t* keys, double* values, int64_t capacity,
                      int64_t* level_counts, void* hip_stream);

/*
 * Inverse: the finest-level field from a leaf set (keys, values as written by
 * rd_mra_leaves): tree nodes valued by projection of the leaves, every node
 * outside the tree predicted level by level from the coarser one.  fine:
 * DEVICE [m][2^(dim J)] output, x fastest.  Keys that do not name a node of
 * the tree are ignored.  Synchronous.  Returns 0 or a negative error.
 */
int64_t rd_mra_reconstruct(const uint64_t* keys, const double* values, int64_t n_leaves,
                           int32_t m, const rd_mra_params* params, double* fine,
                           void* hip_stream);

/*
 * Adaptation of a leaf set to its current values, for instance after a
 * reaction step (refinement and coarsening, §3.1; thresholds §2.2): the
 * levels of its reconstruction (tree nodes by projection of the leaves, the
 * other nodes predicted, so their details are zero), then the details, flags
 * (params->refine as in rd_mra_leaves), grading and leaves of rd_mra_leaves.
 * New leaves carry predicted values; nodes whose children are no longer
 * significant become leaves holding their projected values.  keys, values:
 * the input leaf set (DEVICE, as written by rd_mra_leaves; keys that do not
 * name a node are ignored).  out_keys, out_values, capacity, level_counts and
 * the return value as in rd_mra_leaves; the outputs must not overlap the
 * inputs.  Synchronous.
 */
int64_t rd_mra_adapt(const uint64_t* keys, const double* values, int64_t n_leaves, int32_t m,
                     const rd_mra_params* params, uint64_t* out_keys, double* out_values,
                     int64_t capacity, int64_t* level_counts, void* hip_stream);

/* ------------------------------------------------------------------------ */
/* Serving: a session admits reaction-step requests into an HBM arena of a    */
/* fixed byte budget.  Admitted requests are copied into the arena, batched   */
/* with whatever else was admitted at the same time, and run by persistent    */
/* kernels on a pool of streams, so work of requests that arrive while others */
/* run overlaps on the device.  Results are copied back into the caller's     */
/* states (and stats) when the request completes.                             */
/* ------------------------------------------------------------------------ */
typedef struct rd_session rd_session;

typedef struct {
    int32_t done;          /* 1 when complete                                    */
    int32_t status;        /* 0, or a negative call-level error                  */
    int64_t n_failed;      /* cells with nonzero per-cell status                 */
    int64_t n_cells;
    uint64_t t_submit_ns;  /* CLOCK_MONOTONIC timestamps                         */
    uint64_t t_admit_ns;   /* admitted into the arena, copies and kernel queued  */
    uint64_t t_done_ns;    /* completion observed by the session                 */
    int64_t batch_id;      /* scheduler pass that admitted the request            */
    double kernel_start_ms;/* device time of the request's reaction-step kernel,  */
    double kernel_end_ms;  /* ms since the session was created (-1 if unknown)    */
    int32_t stream;        /* index of the session stream it ran on               */
    int32_t deferred;      /* scheduler passes in which it did not fit the arena  */
} rd_request_info;

/*
 * Create a session on `device` (HIP ordinal) whose arena holds at most
 * hbm_budget_bytes of device memory (allocated here, once).  defaults
 * nullable: the options every request of the session runs with
 * (defaults->session_streams sets the number of launch streams; h_cells must
 * be null).  Returns 0 or RD_EINVAL / RD_ENOMEM / RD_EDEVICE.
 */
int32_t rd_session_create(rd_session** out, int32_t device,
                          size_t hbm_budget_bytes, const rd_options* defaults);

/*
 * Queue a request (non-blocking).  states/stats are DEVICE pointers owned by
 * the caller and must stay valid and untouched until the request is done;
 * stats nullable.  The model parameters are copied.  The session reads the
 * states only after all work enqueued on the device's null stream before
 * this call has completed (an event recorded here); rd_submit_ex takes the
 * stream whose work the read must follow (null = the null stream).
 * RD_ETOOBIG if the request can never fit the budget; RD_ECLOSED once the
 * session is being destroyed.  *req_id receives an id for rd_poll / rd_wait.
 */
int32_t rd_submit(rd_session* s, double* states, int64_t n_cells, int32_t m,
                  double dt, double rtol, double atol, const rd_model* model,
                  int32_t* stats, uint64_t* req_id);
int32_t rd_submit_ex(rd_session* s, double* states, int64_t n_cells, int32_t m,
                     double dt, double rtol, double atol, const rd_model* model,
                     int32_t* stats, void* producer_stream, uint64_t* req_id);

/* 0 done (info filled; the request is then forgotten), 1 pending, < 0 error:
 * the request's own error (message in rd_last_error) or RD_ENOTFOUND.  info
 * nullable.  Results are in the caller's states once done is reported. */
int32_t rd_poll(rd_session* s, uint64_t req_id, rd_request_info* info);

/* Block until done; 0 or < 0 as rd_poll.  info nullable.  Several threads may
 * wait for, or poll, the same id: each is told the outcome once it is done,
 * later calls get RD_ENOTFOUND. */
int32_t rd_wait(rd_session* s, uint64_t req_id, rd_request_info* info);

/* Bytes of the arena a request of this size occupies: its states, its
 * counters when with_stats, and for 8192 cells or more the claim-order
 * scratch of its persistent launch (4 bytes per cell plus a byte per cell
 * and a few KiB). */
size_t rd_request_bytes(int64_t n_cells, int32_t m, int32_t with_stats);

/* Drain outstanding requests, free the arena and streams. */
int32_t rd_session_destroy(rd_session* s);

/* ------------------------------------------------------------------------ */
/* Introspection                                                              */
/* ------------------------------------------------------------------------ */

/* Last error message of the calling thread ("" if none). */
const char* rd_last_error(void);

/* Number of kernel variants for (model kind, m, precision, schedule), and the
 * name of variant v (1-based); NULL when out of range.  Kinetics and linear
 * models share one variant set for m = 5..8 (8-column kernels) and one for
 * m = 9..16 (16-column kernels); a default set for one m of a set applies to
 * the whole set. */
int32_t rd_variant_count(int32_t kind, int32_t m, int32_t precision,
                         int32_t schedule);
const char* rd_variant_name(int32_t kind, int32_t m, int32_t precision,
                            int32_t schedule, int32_t variant);

/* Lanes of a wave that integrate one cell in variant v (1-based; 0 = the
 * default): 1 for the one-lane kernels (64 cells per wave), 16 for the
 * 16-lane-group kernels (4 cells per wave; also offered for the kinetics and
 * linear models with m <= 4).  RD_EINVAL when there is no such variant. */
int32_t rd_variant_lanes(int32_t kind, int32_t m, int32_t precision, int32_t schedule,
                         int32_t variant);

/* Make variant v (1-based) the default for (kind, m, precision, schedule):
 * the autotuner's result.  0 or RD_EINVAL. */
int32_t rd_set_default_variant(int32_t kind, int32_t m, int32_t precision,
                               int32_t schedule, int32_t variant);

/* Device properties the launch sizing uses: compute units and the persistent
 * grid (workgroups) chosen for (kind, m, precision, variant); < 0 on error. */
int32_t rd_persistent_grid(int32_t kind, int32_t m, int32_t precision,
                           int32_t variant, int64_t n_cells);

/*
 * Time the last call's main kernel: returns the duration in milliseconds of
 * the most recent rd_reaction_step_ex launch on this thread, measured with HIP
 * events recorded on the launch stream around the kernel (not the counter
 * reset), or a negative value if unavailable (async calls must have completed).
 */
double rd_last_kernel_ms(void);

#ifdef __cplusplus
}
#endif
#endif
