/*
 * rdo.h -- C ABI of the CPU FP64 Radau5 oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU reaction
 * step; the product path never links, loads or calls it.  It shares no source
 * with the GPU library: its structs below are its own, laid out independently.
 *
 * What it computes: the reaction substep R_dt of the Strang splitting scheme
 * (Descombes et al., §2.1): every cell c integrates du/dt = f(u) over [0, dt]
 * on its own, with Radau5, i.e. the 3-stage Radau IIA collocation method with
 * simplified Newton iterations, an embedded error estimate and step-size
 * control (paper §1, footnote naming Radau5; Hairer & Wanner, Solving ODEs II,
 * §IV.5 and §IV.8).  Unknowns are stored one contiguous array per species
 * (paper §3.2): states[i*n + c] is species i of cell c.
 *
 * All pointers are HOST pointers.  The caller owns every buffer; params are
 * read during the call only.
 */
#ifndef RDO_H
#define RDO_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* model kinds */
enum {
    RDO_OREGONATOR = 1, /* m=3, params {eps, mu, f, q}                         */
    RDO_KINETICS   = 2, /* any m, params {K[m*m] row-major, G[m*m] row-major}  */
    RDO_NAGUMO     = 3, /* m=1, params {k}                                      */
    RDO_LINEAR     = 4, /* any m, params {K[m*m] row-major}: f(u) = K u          */
    RDO_ROBERTSON  = 5, /* m=3, params {k1, k2, k3}                             */
    RDO_BYTECODE   = 6  /* m=1..16, f given as a register program, see below     */
};

/*
 * Bytecode model (a user-supplied f without compiled code).  params =
 *   [L, C, c_0 .. c_{C-1}, then L instructions of 4 doubles (op, d, a, b)]
 * over 64 FP64 registers r[0..64): r[0..m) hold u (read only), r[m..m+C) the
 * constants, the rest are temporaries.  Ops:
 *   1 ADD r[d] = r[a] + r[b]    2 SUB r[d] = r[a] - r[b]   3 MUL r[d] = r[a] * r[b]
 *   4 DIV r[d] = r[a] / r[b]    5 NEG r[d] = -r[a]         6 EXP r[d] = exp(r[a])
 *   7 LOG r[d] = log(r[a])      8 POW r[d] = r[a] ^ r[b]   9 OUT f_d = r[a]
 * A program is valid when every field is an integer in range, d >= m+C for
 * ops 1-8, every register is written before it is read, and OUT writes each
 * of f_0 .. f_{m-1} exactly once.  Its Jacobian is always taken by finite
 * differences.
 */
#define RDO_BC_REGS 64
enum { RDO_BC_ADD = 1, RDO_BC_SUB, RDO_BC_MUL, RDO_BC_DIV, RDO_BC_NEG, RDO_BC_EXP,
       RDO_BC_LOG, RDO_BC_POW, RDO_BC_OUT };

typedef struct {
    int32_t kind;
    int32_t m;
    const double* params;
    int64_t n_params;
} rdo_model;

typedef struct {
    int32_t tol_transform; /* 1: rtol' = 0.1 rtol^(2/3), atol' = rtol' atol/rtol   */
    int32_t max_steps;     /* step attempts per cell before status MAXSTEPS          */
    int32_t newton_max;    /* kmax, Newton iterations per step attempt               */
    int32_t fixed_steps;   /* 0: adaptive; N>0: N equal steps, no error control      */
    double  h0;            /* first trial step; 0 means dt                           */
    double  h_min;         /* 0 means 1e-14 * dt                                     */
    int32_t jacobian;      /* 0 analytic (bytecode: always 1); 1 forward differences:
                              column j = (f(u + d_j e_j) - f(u)) / d_j with
                              d_j = sqrt(uround * max(1e-5, |u_j|)), m extra f
                              evaluations per Jacobian (counted in nfev)           */
    int32_t pad_;
    double* h_cells;       /* null, or [n]: per-cell step size in and out.  In: a
                              value > 0 replaces h0 for that cell.  Out: the step
                              size the controller held before it shortened the final
                              step to end at dt (fixed-step mode: dt / N; a failed
                              cell: the last step size tried)                      */
} rdo_options;

/* per-cell status codes */
enum { RDO_OK = 0, RDO_MAXSTEPS = 1, RDO_H_TOO_SMALL = 2, RDO_SINGULAR = 3,
       RDO_NONFINITE = 4, RDO_NEWTON_FAIL = 5 /* fixed-step mode only */ };

/* call-level error codes */
enum { RDO_EINVAL = -1 };

/* number of int32 rows of the optional stats array, laid out [RDO_NSTATS][n] */
#define RDO_NSTATS 9
/* rows: 0 status, 1 nstep, 2 naccept, 3 nreject, 4 nfev, 5 njac, 6 ndec,
 *       7 nsol, 8 nnewt                                                      */

/*
 * Advance every cell over [0, dt] in place.
 *   states   [m][n] float64, overwritten with u(dt) (failed cells keep their
 *            last accepted state)
 *   opts     nullable -> defaults {1, 100000, 7, 0, 0, 0, 0, 0, null}
 *   stats    nullable, [RDO_NSTATS][n] int32
 *   nthreads 0 -> all hardware threads
 * Returns the number of cells with a nonzero status, or RDO_EINVAL (nothing
 * done) for n<0, m<1, m != model->m, bad params, dt<=0 or non-finite,
 * rtol<=0, atol<0, or a null states/model pointer with n>0.
 */
int64_t rdo_reaction_step(double* states, int64_t n, int32_t m, double dt,
                          double rtol, double atol, const rdo_model* model,
                          const rdo_options* opts, int32_t* stats,
                          int32_t nthreads);

/*
 * One Radau IIA step of size h from y0 (test hook): exact Jacobian at y0,
 * zero Newton start, Newton iterated until the convergence test of the
 * adaptive code passes (at most newton_max iterations).
 *   y1       out, m values
 *   err      out [2]: first and second pass of the error estimate (RMS norm)
 *   info     out [2]: Newton iterations used, 1 if Newton failed else 0
 * Returns 0, or RDO_EINVAL.
 */
int32_t rdo_single_step(const double* y0, int32_t m, double h, double rtol,
                        double atol, int32_t tol_transform, int32_t newton_max,
                        const rdo_model* model, double* y1, double* err,
                        int32_t* info);

/* Newton start values (test hook): the stage increments zold[3][m] of the
 * last accepted step of size h_old define the collocation cubic q(s), s in
 * units of h_old from the end of that step: q(-1) = -z3, q(c_i - 1) = z_i - z3
 * (i = 1, 2), q(0) = 0.  Writes z[i*m + r] = q(c_i h / h_old) for the next
 * step of size h (Hairer & Wanner §IV.8, starting values).  0 or RDO_EINVAL. */
int32_t rdo_start_values(const double* zold, int32_t m, double h, double h_old,
                         double* z);

/* Model hook (tests): f(y) into f[m] and the Jacobian into J[m*m]
 * (row-major, J[i*m+j] = d f_i / d y_j); either output may be null. */
int32_t rdo_model_eval(const rdo_model* model, const double* y, double* f,
                       double* J);

/* Method constants as the oracle uses them: c[3], A[9] row-major,
 * gamma_hat, d[3] (16 doubles). */
void rdo_constants(double* out);

#ifdef __cplusplus
}
#endif
#endif
