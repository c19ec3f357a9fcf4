/*
 * rd_cell_small.h -- Radau5 for one cell held by one lane (m <= 4).
 *
 * Method (Hairer & Wanner, Solving ODEs II, §IV.8; paper §1 footnote on
 * Radau5 and Appendix A): 3-stage Radau IIA; the stage increments Z solve
 * Z = h (A (x) I) F(y0 + Z) by simplified Newton.  Multiplying the Newton
 * system by (h A)^{-1} (x) I and changing variables W = (T^{-1} (x) I) Z, where
 * T^{-1} A^{-1} T = diag(gamma) (+) [[alpha, -beta], [beta, alpha]], splits it
 * into one real m x m system with E1 = (gamma/h) I - J and one complex m x m
 * system with E2 = ((alpha + i beta)/h) I - J.  The embedded error estimate
 * is filtered through E1; step sizes follow the classical controller with the
 * predictive (Gustafsson) correction.  Every decision is the one the FP64 CPU
 * oracle takes; only the arithmetic is arranged for registers (reciprocals
 * instead of divisions, division-free forms of the Newton tests), so results
 * agree with the oracle to rounding.
 *
 * Register budget: the Newton iterate is kept in transformed form W only
 * (Z = T W is formed on the fly), and the two arrays touched once per step --
 * the Jacobian and the stage increments of the last accepted step -- live in
 * LDS, one column of a [rows][BLOCK] array per lane (conflict-free).
 *
 * The cell advances as a state machine (START -> NEWTON* -> START ...) so a
 * lane takes one Newton iteration per pass of the scheduling loop whatever its
 * wave-mates are doing.
 *
 * LT is the type of the LU factors and triangular solves: double for the FP64
 * path, float for the mixed path (f, residuals, W, error estimate and control
 * stay double, and every FP32 solve is refined once against the FP64
 * iteration matrix, so the mixed path takes the FP64 path's decisions).
 */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rd_constants.h"
#include "rd_fastmath.h"
#include "rd_launch.h"
#include "rd_models.h"

namespace rd {

enum : int { ST_OK = 0, ST_MAXSTEPS = 1, ST_HSMALL = 2, ST_SINGULAR = 3,
             ST_NONFINITE = 4, ST_NEWTON = 5 };
enum : int { PH_IDLE = 0, PH_START = 1, PH_NEWTON = 2, PH_END = 3 };
enum : int { NW_CONTINUE = 0, NW_CONVERGED = 1, NW_FAILED = 2 };

/* flag bits */
enum : unsigned { F_FIRST = 1u, F_REJECT = 2u, F_JSTALE = 4u, F_JATY0 = 8u, F_LUOK = 16u,
                  F_OLD = 32u, F_ACC = 64u, F_LAST = 128u, F_KEEPJ = 256u };

constexpr double UROUND = 2.220446049250313e-16;

__device__ __forceinline__ bool finite_d(double x) { return __builtin_isfinite(x); }

__device__ __forceinline__ float fabs_t(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double fabs_t(double x) { return __builtin_fabs(x); }

/* ---------------- small dense LU with partial pivoting ------------------ */
/* Factor a in place (unit-lower L below the diagonal, reciprocal of U's
 * diagonal on the diagonal).  Row swaps are selects so every index stays a
 * compile-time constant.  The pivot rows are returned packed, 2 bits per
 * elimination step.  Returns false on an exactly-zero pivot. */
template <int M, typename T>
__device__ __forceinline__ bool lu_real(T (&a)[M][M], unsigned& piv) {
    bool ok = true;
    piv = 0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        int p = k;
        T best = fabs_t(a[k][k]);
#pragma unroll
        for (int i = k + 1; i < M; ++i) {
            const T v = fabs_t(a[i][k]);
            const bool gt = v > best;
            best = gt ? v : best;
            p = gt ? i : p;
        }
        piv |= (unsigned)p << (2 * k);
        if (__ballot(p != k) != 0ull) {
#pragma unroll
            for (int i = k + 1; i < M; ++i) {
                const bool s = (p == i);
#pragma unroll
                for (int j = 0; j < M; ++j) {
                    const T ak = a[k][j], ai = a[i][j];
                    a[k][j] = s ? ai : ak;
                    a[i][j] = s ? ak : ai;
                }
            }
        }
        ok = ok && (a[k][k] != T(0));
        const T inv = rcp(a[k][k]);
        a[k][k] = inv;
#pragma unroll
        for (int i = k + 1; i < M; ++i) {
            const T l = a[i][k] * inv;
            a[i][k] = l;
#pragma unroll
            for (int j = k + 1; j < M; ++j) a[i][j] -= l * a[k][j];
        }
    }
    return ok;
}

/* packed pivot word of the identity permutation: step k chose row k */
template <int M>
__device__ __forceinline__ constexpr unsigned piv_identity() {
    unsigned v = 0;
    for (int k = 0; k < M; ++k) v |= (unsigned)k << (2 * k);
    return v;
}

template <int M, typename T>
__device__ __forceinline__ void lu_solve_real(const T (&a)[M][M], unsigned piv, T (&b)[M]) {
    /* row interchanges are rare for these iteration matrices: the selects run
     * only when some lane of the wave actually pivoted */
    if (__ballot(piv != piv_identity<M>()) != 0ull) {
#pragma unroll
        for (int k = 0; k < M - 1; ++k) {
            const int p = (piv >> (2 * k)) & 3;
#pragma unroll
            for (int i = k + 1; i < M; ++i) {
                const bool s = (p == i);
                const T bk = b[k], bi = b[i];
                b[k] = s ? bi : bk;
                b[i] = s ? bk : bi;
            }
        }
    }
#pragma unroll
    for (int i = 1; i < M; ++i)
#pragma unroll
        for (int j = 0; j < i; ++j) b[i] -= a[i][j] * b[j];
#pragma unroll
    for (int i = M - 1; i >= 0; --i) {
        T s = b[i];
#pragma unroll
        for (int j = i + 1; j < M; ++j) s -= a[i][j] * b[j];
        b[i] = s * a[i][i];
    }
}

/* Complex version, real and imaginary parts in separate arrays. */
template <int M, typename T>
__device__ __forceinline__ bool lu_cplx(T (&ar)[M][M], T (&ai)[M][M], unsigned& piv) {
    bool ok = true;
    piv = 0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        int p = k;
        T best = ar[k][k] * ar[k][k] + ai[k][k] * ai[k][k];
#pragma unroll
        for (int i = k + 1; i < M; ++i) {
            const T v = ar[i][k] * ar[i][k] + ai[i][k] * ai[i][k];
            const bool gt = v > best;
            best = gt ? v : best;
            p = gt ? i : p;
        }
        piv |= (unsigned)p << (2 * k);
        if (__ballot(p != k) != 0ull)
#pragma unroll
        for (int i = k + 1; i < M; ++i) {
            const bool s = (p == i);
#pragma unroll
            for (int j = 0; j < M; ++j) {
                T x = ar[k][j], y = ar[i][j];
                ar[k][j] = s ? y : x;
                ar[i][j] = s ? x : y;
                x = ai[k][j];
                y = ai[i][j];
                ai[k][j] = s ? y : x;
                ai[i][j] = s ? x : y;
            }
        }
        const T pr = ar[k][k], pi = ai[k][k];
        ok = ok && !(pr == T(0) && pi == T(0));
        /* 1/(pr + i pi) = (pr - i pi) / (pr^2 + pi^2); scaled first where the
         * square leaves the reciprocal's safe range */
        const T nn = pr * pr + pi * pi;
        const T rn = rcp_nr(nn);
        T ir = pr * rn, ii = -pi * rn;
        if (!rcp_nr_ok(nn)) {
            const auto z = slow_crcp(pr, pi);
            ir = z.x;
            ii = z.y;
        }
        ar[k][k] = ir;
        ai[k][k] = ii;
#pragma unroll
        for (int i = k + 1; i < M; ++i) {
            const T xr = ar[i][k], xi = ai[i][k];
            const T lr = xr * ir - xi * ii, li = xr * ii + xi * ir;
            ar[i][k] = lr;
            ai[i][k] = li;
#pragma unroll
            for (int j = k + 1; j < M; ++j) {
                const T ur = ar[k][j], ui = ai[k][j];
                ar[i][j] -= lr * ur - li * ui;
                ai[i][j] -= lr * ui + li * ur;
            }
        }
    }
    return ok;
}

template <int M, typename T>
__device__ __forceinline__ void lu_solve_cplx(const T (&ar)[M][M], const T (&ai)[M][M],
                                              unsigned piv, T (&br)[M], T (&bi)[M]) {
    if (__ballot(piv != piv_identity<M>()) != 0ull) {
#pragma unroll
        for (int k = 0; k < M - 1; ++k) {
            const int p = (piv >> (2 * k)) & 3;
#pragma unroll
            for (int i = k + 1; i < M; ++i) {
                const bool s = (p == i);
                T x = br[k], y = br[i];
                br[k] = s ? y : x;
                br[i] = s ? x : y;
                x = bi[k];
                y = bi[i];
                bi[k] = s ? y : x;
                bi[i] = s ? x : y;
            }
        }
    }
#pragma unroll
    for (int i = 1; i < M; ++i)
#pragma unroll
        for (int j = 0; j < i; ++j) {
            const T lr = ar[i][j], li = ai[i][j];
            br[i] -= lr * br[j] - li * bi[j];
            bi[i] -= lr * bi[j] + li * br[j];
        }
#pragma unroll
    for (int i = M - 1; i >= 0; --i) {
        T sr = br[i], si = bi[i];
#pragma unroll
        for (int j = i + 1; j < M; ++j) {
            const T ur = ar[i][j], ui = ai[i][j];
            sr -= ur * br[j] - ui * bi[j];
            si -= ur * bi[j] + ui * br[j];
        }
        const T dr = ar[i][i], di = ai[i][i];
        br[i] = sr * dr - si * di;
        bi[i] = sr * di + si * dr;
    }
}

/* Per-lane LDS slots with row stride STRIDE: a [ROWS][BLOCK] array read by
 * lane column (STRIDE = BLOCK, base &arr[0][tid]: consecutive lanes hit
 * consecutive words), or a [BLOCK][ROWS'] array read by lane row (STRIDE = 1,
 * base &arr[tid][0], ROWS' odd). */
template <int STRIDE, typename V = double>
struct LdsCol {
    V* base;
    __device__ __forceinline__ V& operator[](int row) const { return base[row * STRIDE]; }
};

/* Rows of the per-lane LDS column: Jacobian (M*M), Z of the last accepted
 * step (3*M), then the step-control scalars read once per step (previous
 * step size, 1/h and err^(1/4) of the last accepted step, the warm-start
 * step size); and the integer rows of the counters that change once per
 * step or less.  Keeping this cold state out of registers lets the engine
 * run three waves per SIMD with fewer spills. */
template <int M>
struct SmallLds {
    static constexpr int J0 = 0;
    static constexpr int Z0 = M * M;
    static constexpr int HOLD = M * M + 3 * M, IHACC = HOLD + 1, QACC = HOLD + 2, HPRE = HOLD + 3;
    static constexpr int ROWS = HPRE + 1;
    static constexpr int NSTEP = 0, NACCEPT = 1, NREJECT = 2, NJAC = 3, NDEC = 4;
    static constexpr int IROWS = 5;
    /* odd row counts of the lane-row layout */
    static constexpr int ROWS_AOS = ROWS | 1, IROWS_AOS = IROWS | 1;
};

/* ---------------- the per-cell engine ----------------------------------- */
/* BLOCK: the row stride of the cell's LDS slots (LdsCol) */
template <class Model, typename LT, int BLOCK>
struct SmallCell {
    static constexpr int M = Model::M;
    using L = SmallLds<M>;
    /* FP32 factors: every solve is refined once against the FP64 matrices */
    static constexpr bool kRefine = sizeof(LT) < sizeof(double);

    /* state */
    double y[M], f0[M], isc[M];
    double w[3][M];
    LT e1[M][M], e2r[M][M], e2i[M][M];
    double t, h, ih, eta, inprev;
    unsigned p1, p2, flags;
    int phase, status, k, nsing, outcome;
    /* counters (paper Appendix A: f evaluations per node); the ones that
     * change once per step or less live in LDS (SmallLds) */
    int nfev, nsol, nnewt;
    LdsCol<BLOCK> lds;
    LdsCol<BLOCK, int> ilds;

    __device__ __forceinline__ bool has(unsigned f) const { return (flags & f) != 0u; }
    __device__ __forceinline__ void set(unsigned f, bool v) { flags = v ? (flags | f) : (flags & ~f); }

    __device__ __forceinline__ void load(const Model& md, const StepParams& P,
                                         const double* __restrict__ states, int64_t n,
                                         int64_t c, const double* __restrict__ hcell) {
#pragma unroll
        for (int r = 0; r < M; ++r) y[r] = states[(int64_t)r * n + c];
        ilds[L::NSTEP] = ilds[L::NACCEPT] = ilds[L::NREJECT] = 0;
        ilds[L::NJAC] = ilds[L::NDEC] = 0;
        nsol = nnewt = 0;
        nfev = 1;
        md.rhs(y, f0);
        status = ST_OK;
        bool fin = true;
#pragma unroll
        for (int r = 0; r < M; ++r) fin = fin && finite_d(y[r]) && finite_d(f0[r]);
        t = 0.0;
        /* first trial step: the cell's warm-start value when one is given */
        const double hw = hcell ? hcell[c] : 0.0;
        h = P.fixed_steps > 0 ? P.dt / P.fixed_steps
                              : fmin(hw > 0.0 ? hw : (P.h0 > 0.0 ? P.h0 : P.dt), P.dt);
        lds[L::HPRE] = fin ? h : 0.0;
        lds[L::HOLD] = lds[L::IHACC] = lds[L::QACC] = inprev = 0.0;
        eta = 1.0;
        k = 0;
        nsing = 0;
        flags = F_FIRST | F_JSTALE;
        phase = fin ? PH_START : PH_IDLE;
        if (!fin) status = ST_NONFINITE;
    }

    __device__ __forceinline__ void store(double* __restrict__ states, int32_t* __restrict__ stats,
                                          int64_t n, int64_t c, double* __restrict__ hcell) const {
#pragma unroll
        for (int r = 0; r < M; ++r) states[(int64_t)r * n + c] = y[r];
        if (hcell) hcell[c] = lds[L::HPRE];
        if (stats) {
            stats[0 * n + c] = status;
            stats[1 * n + c] = ilds[L::NSTEP];
            stats[2 * n + c] = ilds[L::NACCEPT];
            stats[3 * n + c] = ilds[L::NREJECT];
            stats[4 * n + c] = nfev;
            stats[5 * n + c] = ilds[L::NJAC];
            stats[6 * n + c] = ilds[L::NDEC];
            stats[7 * n + c] = nsol;
            stats[8 * n + c] = nnewt;
        }
    }

    /* E1 = (gamma/h) I - J, E2 = ((alpha + i beta)/h) I - J, both factored. */
    __device__ __forceinline__ bool factor() {
        const double g = radau::GAMMA * ih, ar = radau::ALPHA * ih, bi = radau::BETA * ih;
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const double mj = -lds[L::J0 + i * M + j];
                e1[i][j] = (LT)(i == j ? g + mj : mj);
                e2r[i][j] = (LT)(i == j ? ar + mj : mj);
                e2i[i][j] = (LT)(i == j ? bi : 0.0);
            }
        const bool ok1 = lu_real<M, LT>(e1, p1);
        const bool ok2 = lu_cplx<M, LT>(e2r, e2i, p2);
        return ok1 && ok2;
    }

    /* Start of a step attempt.  Leaves phase = PH_NEWTON when Newton can
     * start, PH_START to retry (singular matrix, h halved), PH_IDLE when the
     * cell stops with a status. */
    template <bool FIXED>
    __device__ __forceinline__ void start(const Model& md, const StepParams& P) {
        if (!FIXED) {
            lds[L::HPRE] = h;
            if (ilds[L::NSTEP] >= P.max_steps) { status = ST_MAXSTEPS; phase = PH_IDLE; return; }
            if (h < P.h_min) { status = ST_HSMALL; phase = PH_IDLE; return; }
            const bool last = t + 1.0001 * h >= P.dt;
            if (last) {
                const double hl = P.dt - t;
                if (hl != h) flags &= ~F_LUOK;
                h = hl;
            }
            set(F_LAST, last);
        }
        ih = rcp(h);
#pragma unroll
        for (int r = 0; r < M; ++r) isc[r] = rcp(P.atol + P.rtol * __builtin_fabs(y[r]));
        if (FIXED || has(F_JSTALE)) {
            double J[M][M];
            if (fd_jac_of<Model>::value) {
                fd_jacobian(md, y, f0, J);
                nfev += M;
            } else {
                md.jac(y, J);
            }
#pragma unroll
            for (int i = 0; i < M; ++i)
#pragma unroll
                for (int j = 0; j < M; ++j) lds[L::J0 + i * M + j] = J[i][j];
            ++ilds[L::NJAC];
            flags = (flags & ~(F_JSTALE | F_LUOK)) | F_JATY0;
        }
        RD_PH_BEGIN(ph_f)
        if (FIXED || !has(F_LUOK)) {
            ++ilds[L::NDEC];
            if (!factor()) {
                if (FIXED || ++nsing >= 5) { status = ST_SINGULAR; phase = PH_IDLE; return; }
                h *= 0.5;
                phase = PH_START;
                return;
            }
            nsing = 0;
            flags |= F_LUOK;
        }
        RD_PH_END(ph_f, PHASE_FACTOR);
        /* Newton start: zero, or the collocation cubic of the last accepted
         * step continued to the new stage points (nodes s = -1, c1-1, c2-1, 0
         * in units of h_old; values -z3, z1 - z3, z2 - z3, 0), then W = T^-1 Z. */
        if (has(F_OLD)) {
            const double r = h * rcp(lds[L::HOLD]);
            const double s1 = -1.0, s2 = radau::C1 - 1.0, s3 = radau::C2 - 1.0;
            const double cs[3] = {radau::C1 * r, radau::C2 * r, r};
            double Lw[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double s = cs[i];
                const double d1 = s - s1, d2 = s - s2, d3 = s - s3, d4 = s;
                Lw[i][0] = d2 * d3 * d4 * radau::LAG_INV0;
                Lw[i][1] = d1 * d3 * d4 * radau::LAG_INV1;
                Lw[i][2] = d1 * d2 * d4 * radau::LAG_INV2;
            }
#pragma unroll
            for (int q = 0; q < M; ++q) {
                const double z1o = lds[L::Z0 + q], z2o = lds[L::Z0 + M + q], z3o = lds[L::Z0 + 2 * M + q];
                const double v0 = -z3o, v1 = z1o - z3o, v2 = z2o - z3o;
                const double a = Lw[0][0] * v0 + Lw[0][1] * v1 + Lw[0][2] * v2;
                const double b = Lw[1][0] * v0 + Lw[1][1] * v1 + Lw[1][2] * v2;
                const double c = Lw[2][0] * v0 + Lw[2][1] * v1 + Lw[2][2] * v2;
                w[0][q] = radau::TI11 * a + radau::TI12 * b + radau::TI13 * c;
                w[1][q] = radau::TI21 * a + radau::TI22 * b + radau::TI23 * c;
                w[2][q] = radau::TI31 * a + radau::TI32 * b + radau::TI33 * c;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int q = 0; q < M; ++q) w[i][q] = 0.0;
        }
        k = 0;
        inprev = 0.0;
        phase = PH_NEWTON;
    }

    /* One simplified-Newton iteration in transformed variables. */
    __device__ __forceinline__ int newton(const Model& md, const StepParams& P) {
        ++k;
        ++nnewt;
        /* G = T^-1 F(y0 + Z), Z = T W, one stage at a time */
        double G[3][M];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double ys[M], F[M];
#pragma unroll
            for (int q = 0; q < M; ++q) {
                const double zi = i == 0 ? radau::T11 * w[0][q] + radau::T12 * w[1][q] + radau::T13 * w[2][q]
                                : i == 1 ? radau::T21 * w[0][q] + radau::T22 * w[1][q] + radau::T23 * w[2][q]
                                         : w[0][q] + w[1][q]; /* row 3 of T is (1, 1, 0) */
                ys[q] = y[q] + zi;
            }
            md.rhs(ys, F);
            const double t1 = i == 0 ? radau::TI11 : i == 1 ? radau::TI12 : radau::TI13;
            const double t2 = i == 0 ? radau::TI21 : i == 1 ? radau::TI22 : radau::TI23;
            const double t3 = i == 0 ? radau::TI31 : i == 1 ? radau::TI32 : radau::TI33;
#pragma unroll
            for (int q = 0; q < M; ++q) {
                if (i == 0) {
                    G[0][q] = t1 * F[q];
                    G[1][q] = t2 * F[q];
                    G[2][q] = t3 * F[q];
                } else {
                    G[0][q] += t1 * F[q];
                    G[1][q] += t2 * F[q];
                    G[2][q] += t3 * F[q];
                }
            }
        }
        nfev += 3;
        const double g = radau::GAMMA * ih, al = radau::ALPHA * ih, be = radau::BETA * ih;
        /* right-hand sides of the real and the complex system */
        double b1[M], b2[M], b3[M];
        LT r1[M], r2[M], r3[M];
#pragma unroll
        for (int q = 0; q < M; ++q) {
            b1[q] = G[0][q] - g * w[0][q];
            b2[q] = G[1][q] - al * w[1][q] + be * w[2][q];
            b3[q] = G[2][q] - be * w[1][q] - al * w[2][q];
            r1[q] = (LT)b1[q];
            r2[q] = (LT)b2[q];
            r3[q] = (LT)b3[q];
        }
        lu_solve_real<M, LT>(e1, p1, r1);
        lu_solve_cplx<M, LT>(e2r, e2i, p2, r2, r3);
        double x1[M], x2[M], x3[M];
#pragma unroll
        for (int q = 0; q < M; ++q) {
            x1[q] = (double)r1[q];
            x2[q] = (double)r2[q];
            x3[q] = (double)r3[q];
        }
        if constexpr (kRefine) refine_newton(b1, b2, b3, x1, x2, x3);
        ++nsol;
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < M; ++q) {
            const double d1 = x1[q], d2 = x2[q], d3 = x3[q];
            w[0][q] += d1;
            w[1][q] += d2;
            w[2][q] += d3;
            const double dz1 = radau::T11 * d1 + radau::T12 * d2 + radau::T13 * d3;
            const double dz2 = radau::T21 * d1 + radau::T22 * d2 + radau::T23 * d3;
            const double dz3 = d1 + d2;
            const double s1 = dz1 * isc[q], s2 = dz2 * isc[q], s3 = dz3 * isc[q];
            acc += s1 * s1 + s2 * s2 + s3 * s3;
        }
        const double nk = sqrt_f(acc * (1.0 / (3 * M)));
        if (!finite_d(nk)) return NW_FAILED;
        const double tol = P.newton_tol;
        if (k >= 2) {
            /* theta = n_k / n_{k-1}; diverging if theta >= 0.99; eta =
             * theta / (1 - theta); too slow if theta^(kmax-k) / (1 - theta)
             * n_k > tol, tested as theta^(kmax-k) n_k > tol (1 - theta) since
             * 1 - theta > 0.01 here */
            const double th = nk * inprev;
            if (th >= 0.99) return NW_FAILED;
            const double om = 1.0 - th;
            eta = th * rcp_nr(om);
            double tp = 1.0;
            for (int j = 0; j < P.kmax - k; ++j) tp *= th;
            if (tp * nk > tol * om) return NW_FAILED;
            set(F_KEEPJ, th <= 1e-3);
        } else {
            set(F_KEEPJ, true);
        }
        if (eta * nk <= tol) return NW_CONVERGED;
        /* nk > 0 here (nk == 0 converges above) */
        inprev = rcp(nk);
        return k >= P.kmax ? NW_FAILED : NW_CONTINUE;
    }

    /* Mixed precision: one step of iterative refinement of the FP32-factored
     * solves, with the residual of the FP64 systems E1 = (gamma/h) I - J and
     * E2 = ((alpha + i beta)/h) I - J (J from the LDS column, the same J the
     * factors were rounded from): x += LU32^{-1} (b - E x).  The solve error
     * drops from about cond * 2^-24 to its square, so the Newton iterates are
     * those of the FP64 iteration to rounding and the same control decisions
     * follow. */
    __device__ __forceinline__ void refine_newton(const double (&b1)[M], const double (&b2)[M],
                                                  const double (&b3)[M], double (&x1)[M],
                                                  double (&x2)[M], double (&x3)[M]) {
        const double g = radau::GAMMA * ih, al = radau::ALPHA * ih, be = radau::BETA * ih;
        LT c1[M], c2[M], c3[M];
#pragma unroll
        for (int i = 0; i < M; ++i) {
            double j1 = 0.0, j2 = 0.0, j3 = 0.0;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const double a = lds[L::J0 + i * M + j];
                j1 += a * x1[j];
                j2 += a * x2[j];
                j3 += a * x3[j];
            }
            c1[i] = (LT)(b1[i] - g * x1[i] + j1);
            c2[i] = (LT)(b2[i] - al * x2[i] + be * x3[i] + j2);
            c3[i] = (LT)(b3[i] - be * x2[i] - al * x3[i] + j3);
        }
        lu_solve_real<M, LT>(e1, p1, c1);
        lu_solve_cplx<M, LT>(e2r, e2i, p2, c2, c3);
#pragma unroll
        for (int q = 0; q < M; ++q) {
            x1[q] += (double)c1[q];
            x2[q] += (double)c2[q];
            x3[q] += (double)c3[q];
        }
    }

    /* e = E1^{-1} [fb + (d1 z1 + d2 z2 + d3 z3)/h]; returns RMS(e/sc). */
    __device__ __forceinline__ double estimate(const double (&fb)[M], double (&e)[M]) {
        /* d.Z = (d^T T) W */
        constexpr double DW1 = radau::D1 * radau::T11 + radau::D2 * radau::T21 + radau::D3;
        constexpr double DW2 = radau::D1 * radau::T12 + radau::D2 * radau::T22 + radau::D3;
        constexpr double DW3 = radau::D1 * radau::T13 + radau::D2 * radau::T23;
        double b[M];
        LT v[M];
#pragma unroll
        for (int q = 0; q < M; ++q) {
            b[q] = fb[q] + (DW1 * w[0][q] + DW2 * w[1][q] + DW3 * w[2][q]) * ih;
            v[q] = (LT)b[q];
        }
        lu_solve_real<M, LT>(e1, p1, v);
#pragma unroll
        for (int q = 0; q < M; ++q) e[q] = (double)v[q];
        if constexpr (kRefine) {
            /* one refinement step against E1 in FP64, as in refine_newton */
            const double g = radau::GAMMA * ih;
            LT c[M];
#pragma unroll
            for (int i = 0; i < M; ++i) {
                double jx = 0.0;
#pragma unroll
                for (int j = 0; j < M; ++j) jx += lds[L::J0 + i * M + j] * e[j];
                c[i] = (LT)(b[i] - g * e[i] + jx);
            }
            lu_solve_real<M, LT>(e1, p1, c);
#pragma unroll
            for (int q = 0; q < M; ++q) e[q] += (double)c[q];
        }
        ++nsol;
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < M; ++q) {
            const double s = e[q] * isc[q];
            acc += s * s;
        }
        return sqrt_f(acc * (1.0 / M));
    }

    /* After the Newton loop ends: error test, step-size control, accept or
     * reject.  Leaves phase = PH_START for the next attempt or PH_IDLE. */
    template <bool FIXED>
    __device__ __forceinline__ void finish(const Model& md, const StepParams& P, int outcome) {
        if (FIXED) {
            if (outcome == NW_FAILED) { status = ST_NEWTON; phase = PH_IDLE; return; }
            ++ilds[L::NSTEP];
            ++ilds[L::NACCEPT];
            accept_state(md);
            bool fin = true;
#pragma unroll
            for (int q = 0; q < M; ++q) fin = fin && finite_d(y[q]);
            if (!fin) { status = ST_NONFINITE; phase = PH_IDLE; return; }
            lds[L::HOLD] = h;
            eta = pow08(fmax(eta, UROUND));
            phase = (ilds[L::NACCEPT] >= P.fixed_steps) ? PH_IDLE : PH_START;
            return;
        }
        if (outcome == NW_FAILED) {
            ++ilds[L::NSTEP];
            ++ilds[L::NREJECT];
            h *= 0.5;
            flags = (flags | F_REJECT) & ~F_LUOK;
            if (!has(F_JATY0)) flags |= F_JSTALE;
            phase = PH_START;
            return;
        }
        double e[M];
        double err = estimate(f0, e);
        if (err >= 1.0 && (flags & (F_FIRST | F_REJECT))) {
            double ye[M], fe[M];
#pragma unroll
            for (int q = 0; q < M; ++q) ye[q] = y[q] + e[q];
            md.rhs(ye, fe);
            ++nfev;
            err = estimate(fe, e);
        }
        if (!finite_d(err)) { status = ST_NONFINITE; phase = PH_IDLE; return; }
        ++ilds[L::NSTEP];
        const double fac = k <= kMaxFacTable
                               ? P.fac[k]
                               : 0.9 * (2.0 * P.kmax + 1.0) / (2.0 * P.kmax + (double)k);
        /* s = err^(-1/4); the classical factor is fac / err^(1/4) = fac s */
        const double s = rroot4(err == 0.0 ? 1.0 : err);
        const double ratio = (err == 0.0) ? 8.0 : fmin(8.0, fmax(0.2, fac * s));
        double h_new = h * ratio;
        if (err < 1.0) {
            if (has(F_ACC)) {
                /* predictive: fac (h / h_acc) err_acc^(1/4) / err^(1/2) */
                const double r2 = (err == 0.0)
                    ? 8.0
                    : fmin(8.0, fmax(0.2, fac * (h * lds[L::IHACC]) * lds[L::QACC] * (s * s)));
                h_new = fmin(h_new, h * r2);
            }
            double zs[3][M];
            double y1[M], f1[M];
#pragma unroll
            for (int q = 0; q < M; ++q) {
                zs[0][q] = radau::T11 * w[0][q] + radau::T12 * w[1][q] + radau::T13 * w[2][q];
                zs[1][q] = radau::T21 * w[0][q] + radau::T22 * w[1][q] + radau::T23 * w[2][q];
                zs[2][q] = w[0][q] + w[1][q];
                y1[q] = y[q] + zs[2][q];
            }
            md.rhs(y1, f1);
            ++nfev;
            bool fin = true;
#pragma unroll
            for (int q = 0; q < M; ++q) fin = fin && finite_d(y1[q]) && finite_d(f1[q]);
            if (!fin) { status = ST_NONFINITE; phase = PH_IDLE; return; }
            lds[L::IHACC] = ih;
            /* max(err, 1e-2)^(1/4); (1e-2)^(1/4) = sqrt(0.1) */
            lds[L::QACC] = err >= 1e-2 ? rcp_nr(s) : 0.31622776601683794;
#pragma unroll
            for (int q = 0; q < M; ++q) {
                y[q] = y1[q];
                f0[q] = f1[q];
                lds[L::Z0 + q] = zs[0][q];
                lds[L::Z0 + M + q] = zs[1][q];
                lds[L::Z0 + 2 * M + q] = zs[2][q];
            }
            t = has(F_LAST) ? P.dt : t + h;
            lds[L::HOLD] = h;
            eta = pow08(fmax(eta, UROUND));
            ++ilds[L::NACCEPT];
            if (has(F_REJECT)) h_new = fmin(h_new, h);
            const bool keep_j = has(F_KEEPJ);
            flags = (flags & ~(F_FIRST | F_REJECT | F_JATY0 | F_JSTALE)) | F_OLD | F_ACC |
                    (keep_j ? 0u : F_JSTALE);
            if (keep_j) {
                /* h_new / h in [1, 1.2] */
                if (h_new >= h && h_new <= 1.2 * h) h_new = h;
            }
            const double hn = fmin(h_new, P.dt - t);
            if (hn != h) flags &= ~F_LUOK;
            h = hn;
            phase = (t < P.dt) ? PH_START : PH_IDLE;
        } else {
            ++ilds[L::NREJECT];
            const double hn = has(F_FIRST) ? 0.1 * h : h_new;
            if (hn != h) flags &= ~F_LUOK;
            h = hn;
            flags |= F_REJECT;
            phase = PH_START;
        }
    }

    /* fixed-step accept: y += z3, f0 = f(y), keep Z for the next start */
    __device__ __forceinline__ void accept_state(const Model& md) {
#pragma unroll
        for (int q = 0; q < M; ++q) {
            const double z1 = radau::T11 * w[0][q] + radau::T12 * w[1][q] + radau::T13 * w[2][q];
            const double z2 = radau::T21 * w[0][q] + radau::T22 * w[1][q] + radau::T23 * w[2][q];
            const double z3 = w[0][q] + w[1][q];
            y[q] += z3;
            lds[L::Z0 + q] = z1;
            lds[L::Z0 + M + q] = z2;
            lds[L::Z0 + 2 * M + q] = z3;
        }
        md.rhs(y, f0);
        ++nfev;
        flags |= F_OLD;
    }
};

}  // namespace rd
