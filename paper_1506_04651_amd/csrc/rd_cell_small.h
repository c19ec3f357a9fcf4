/*
 * rd_cell_small.h -- Radau5 for one cell held entirely by one lane (m <= 4).
 *
 * Method (Hairer & Wanner, Solving ODEs II, §IV.8; paper §1 footnote on
 * Radau5 and Appendix A): 3-stage Radau IIA; the stage increments Z solve
 * Z = h (A (x) I) F(y0 + Z) by simplified Newton.  Multiplying the Newton
 * system by (h A)^{-1} (x) I and changing variables W = (T^{-1} (x) I) Z, where
 * T^{-1} A^{-1} T = diag(gamma) (+) [[alpha, -beta], [beta, alpha]], splits it
 * into one real m x m system with E1 = (gamma/h) I - J and one complex m x m
 * system with E2 = ((alpha + i beta)/h) I - J.  The embedded error estimate
 * is filtered through E1; step sizes follow the classical controller with the
 * predictive (Gustafsson) correction.  Every decision below is the same as in
 * the FP64 CPU oracle's reading of the method; only the linear algebra is
 * arranged for registers.
 *
 * The cell advances as a small state machine (START -> NEWTON* -> START ...)
 * so that a lane can take one Newton iteration per pass of the scheduling loop
 * regardless of what the other lanes of its wave are doing.
 *
 * LT is the type of the LU factors and triangular solves: double for the FP64
 * path, float for the mixed path (residuals, stage values, error estimate and
 * control stay double).
 */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rd_constants.h"
#include "rd_launch.h"
#include "rd_models.h"

namespace rd {

enum : int { ST_OK = 0, ST_MAXSTEPS = 1, ST_HSMALL = 2, ST_SINGULAR = 3,
             ST_NONFINITE = 4, ST_NEWTON = 5 };
enum : int { PH_IDLE = 0, PH_START = 1, PH_NEWTON = 2 };
enum : int { NW_CONTINUE = 0, NW_CONVERGED = 1, NW_FAILED = 2 };

constexpr double UROUND = 2.220446049250313e-16;

__device__ __forceinline__ bool finite_d(double x) { return __builtin_isfinite(x); }

/* ---------------- small dense LU with partial pivoting ------------------ */
/* Factor a in place (unit-lower L below the diagonal, reciprocal of U's
 * diagonal on the diagonal).  Row swaps are done with selects so every index
 * stays a compile-time constant (registers, no scratch).  Returns false on an
 * exactly-zero pivot. */
template <int M, typename T>
__device__ __forceinline__ bool lu_real(T (&a)[M][M], int (&piv)[M]) {
    bool ok = true;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        int p = k;
        T best = __builtin_fabs(a[k][k]);
#pragma unroll
        for (int i = k + 1; i < M; ++i) {
            const T v = __builtin_fabs(a[i][k]);
            const bool gt = v > best;
            best = gt ? v : best;
            p = gt ? i : p;
        }
        piv[k] = p;
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
        ok = ok && (a[k][k] != T(0));
        const T inv = T(1) / a[k][k];
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

template <int M, typename T>
__device__ __forceinline__ void lu_solve_real(const T (&a)[M][M], const int (&piv)[M],
                                              T (&b)[M]) {
#pragma unroll
    for (int k = 0; k < M; ++k) {
#pragma unroll
        for (int i = k + 1; i < M; ++i) {
            const bool s = (piv[k] == i);
            const T bk = b[k], bi = b[i];
            b[k] = s ? bi : bk;
            b[i] = s ? bk : bi;
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
__device__ __forceinline__ bool lu_cplx(T (&ar)[M][M], T (&ai)[M][M], int (&piv)[M]) {
    bool ok = true;
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
        piv[k] = p;
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
        const T rn = T(1) / (pr * pr + pi * pi);
        const T ir = pr * rn, ii = -pi * rn; /* 1/(pr + i pi) */
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
                                              const int (&piv)[M], T (&br)[M], T (&bi)[M]) {
#pragma unroll
    for (int k = 0; k < M; ++k) {
#pragma unroll
        for (int i = k + 1; i < M; ++i) {
            const bool s = (piv[k] == i);
            T x = br[k], y = br[i];
            br[k] = s ? y : x;
            br[i] = s ? x : y;
            x = bi[k];
            y = bi[i];
            bi[k] = s ? y : x;
            bi[i] = s ? x : y;
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

/* ---------------- the per-cell engine ----------------------------------- */
template <class Model, typename LT>
struct SmallCell {
    static constexpr int M = Model::M;

    /* state */
    double y[M], f0[M], isc[M];
    double z[3][M], w[3][M], zold[3][M];
    double J[M][M];
    LT e1[M][M], e2r[M][M], e2i[M][M];
    int p1[M], p2[M];
    double t, h, h_lu, h_old, h_acc, err_acc, eta, theta, nprev;
    int phase, status, k, nsing;
    bool first, reject, j_stale, j_at_y0, have_lu, have_old, have_acc, last;
    /* counters (paper Appendix A: f evaluations per node) */
    int nstep, naccept, nreject, nfev, njac, ndec, nsol, nnewt;

    __device__ __forceinline__ void load(const Model& md, const StepParams& P,
                                         const double* __restrict__ states, int64_t n,
                                         int64_t c) {
#pragma unroll
        for (int r = 0; r < M; ++r) y[r] = states[(int64_t)r * n + c];
        nstep = naccept = nreject = njac = ndec = nsol = nnewt = 0;
        nfev = 1;
        md.rhs(y, f0);
        status = ST_OK;
        bool fin = true;
#pragma unroll
        for (int r = 0; r < M; ++r) fin = fin && finite_d(y[r]) && finite_d(f0[r]);
        t = 0.0;
        h = P.fixed_steps > 0 ? P.dt / P.fixed_steps : fmin(P.h0 > 0.0 ? P.h0 : P.dt, P.dt);
        h_lu = h_old = h_acc = err_acc = theta = nprev = 0.0;
        eta = 1.0;
        k = 0;
        nsing = 0;
        first = true;
        reject = false;
        j_stale = true;
        j_at_y0 = false;
        have_lu = have_old = have_acc = last = false;
        if (!fin) {
            status = ST_NONFINITE;
            phase = PH_IDLE;
        } else {
            phase = PH_START;
        }
    }

    __device__ __forceinline__ void store(double* __restrict__ states, int32_t* __restrict__ stats,
                                          int64_t n, int64_t c) const {
#pragma unroll
        for (int r = 0; r < M; ++r) states[(int64_t)r * n + c] = y[r];
        if (stats) {
            stats[0 * n + c] = status;
            stats[1 * n + c] = nstep;
            stats[2 * n + c] = naccept;
            stats[3 * n + c] = nreject;
            stats[4 * n + c] = nfev;
            stats[5 * n + c] = njac;
            stats[6 * n + c] = ndec;
            stats[7 * n + c] = nsol;
            stats[8 * n + c] = nnewt;
        }
    }

    /* E1 = (gamma/h) I - J, E2 = ((alpha + i beta)/h) I - J, both factored. */
    __device__ __forceinline__ bool factor() {
        const double ih = 1.0 / h;
        const double g = radau::GAMMA * ih, ar = radau::ALPHA * ih, bi = radau::BETA * ih;
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const double mj = -J[i][j];
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
            if (nstep >= P.max_steps) { status = ST_MAXSTEPS; phase = PH_IDLE; return; }
            if (h < P.h_min) { status = ST_HSMALL; phase = PH_IDLE; return; }
            last = false;
            if (t + 1.0001 * h >= P.dt) { h = P.dt - t; last = true; }
        }
#pragma unroll
        for (int r = 0; r < M; ++r) isc[r] = 1.0 / (P.atol + P.rtol * __builtin_fabs(y[r]));
        if (FIXED || j_stale) {
            md.jac(y, J);
            ++njac;
            j_stale = false;
            j_at_y0 = true;
            have_lu = false;
        }
        if (FIXED || !have_lu || h != h_lu) {
            ++ndec;
            if (!factor()) {
                have_lu = false;
                if (FIXED || ++nsing >= 5) { status = ST_SINGULAR; phase = PH_IDLE; return; }
                h *= 0.5;
                phase = PH_START;
                return;
            }
            nsing = 0;
            have_lu = true;
            h_lu = h;
        }
        /* Newton start: zero, or the collocation cubic of the last accepted
         * step continued to the new stage points (nodes s = -1, c1-1, c2-1, 0
         * in units of h_old; values -z3, z1 - z3, z2 - z3, 0). */
        if (have_old) {
            const double r = h / h_old;
            const double s1 = -1.0, s2 = radau::C1 - 1.0, s3 = radau::C2 - 1.0;
            const double cs[3] = {radau::C1 * r, radau::C2 * r, r};
            double L[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double s = cs[i];
                const double d1 = s - s1, d2 = s - s2, d3 = s - s3, d4 = s; /* s - 0 */
                L[i][0] = d2 * d3 * d4 * radau::LAG_INV0;
                L[i][1] = d1 * d3 * d4 * radau::LAG_INV1;
                L[i][2] = d1 * d2 * d4 * radau::LAG_INV2;
            }
#pragma unroll
            for (int q = 0; q < M; ++q) {
                const double v0 = -zold[2][q];
                const double v1 = zold[0][q] - zold[2][q];
                const double v2 = zold[1][q] - zold[2][q];
#pragma unroll
                for (int i = 0; i < 3; ++i) z[i][q] = L[i][0] * v0 + L[i][1] * v1 + L[i][2] * v2;
            }
        } else {
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int q = 0; q < M; ++q) z[i][q] = 0.0;
        }
#pragma unroll
        for (int q = 0; q < M; ++q) {
            const double a = z[0][q], b = z[1][q], c = z[2][q];
            w[0][q] = radau::TI11 * a + radau::TI12 * b + radau::TI13 * c;
            w[1][q] = radau::TI21 * a + radau::TI22 * b + radau::TI23 * c;
            w[2][q] = radau::TI31 * a + radau::TI32 * b + radau::TI33 * c;
        }
        k = 0;
        nprev = 0.0;
        phase = PH_NEWTON;
    }

    /* One simplified-Newton iteration in transformed variables. */
    __device__ __forceinline__ int newton(const Model& md, const StepParams& P) {
        ++k;
        ++nnewt;
        double F[3][M];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double ys[M];
#pragma unroll
            for (int q = 0; q < M; ++q) ys[q] = y[q] + z[i][q];
            md.rhs(ys, F[i]);
        }
        nfev += 3;
        const double ih = 1.0 / h;
        const double g = radau::GAMMA * ih, al = radau::ALPHA * ih, be = radau::BETA * ih;
        LT r1[M], r2[M], r3[M];
#pragma unroll
        for (int q = 0; q < M; ++q) {
            const double a = F[0][q], b = F[1][q], c = F[2][q];
            const double g1 = radau::TI11 * a + radau::TI12 * b + radau::TI13 * c;
            const double g2 = radau::TI21 * a + radau::TI22 * b + radau::TI23 * c;
            const double g3 = radau::TI31 * a + radau::TI32 * b + radau::TI33 * c;
            r1[q] = (LT)(g1 - g * w[0][q]);
            r2[q] = (LT)(g2 - al * w[1][q] + be * w[2][q]);
            r3[q] = (LT)(g3 - be * w[1][q] - al * w[2][q]);
        }
        lu_solve_real<M, LT>(e1, p1, r1);
        lu_solve_cplx<M, LT>(e2r, e2i, p2, r2, r3);
        ++nsol;
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < M; ++q) {
            const double d1 = (double)r1[q], d2 = (double)r2[q], d3 = (double)r3[q];
            w[0][q] += d1;
            w[1][q] += d2;
            w[2][q] += d3;
            const double dz1 = radau::T11 * d1 + radau::T12 * d2 + radau::T13 * d3;
            const double dz2 = radau::T21 * d1 + radau::T22 * d2 + radau::T23 * d3;
            const double dz3 = d1 + d2; /* row 3 of T is (1, 1, 0) */
            z[0][q] += dz1;
            z[1][q] += dz2;
            z[2][q] += dz3;
            const double s1 = dz1 * isc[q], s2 = dz2 * isc[q], s3 = dz3 * isc[q];
            acc += s1 * s1 + s2 * s2 + s3 * s3;
        }
        const double nk = __builtin_sqrt(acc * (1.0 / (3 * M)));
        if (!finite_d(nk)) return NW_FAILED;
        if (k >= 2) {
            const double th = nk / nprev;
            theta = th;
            if (th >= 0.99) return NW_FAILED;
            eta = th / (1.0 - th);
            double tp = 1.0;
            for (int j = 0; j < P.kmax - k; ++j) tp *= th;
            if (tp / (1.0 - th) * nk > P.newton_tol) return NW_FAILED;
        }
        if (eta * nk <= P.newton_tol) return NW_CONVERGED;
        nprev = nk;
        return k >= P.kmax ? NW_FAILED : NW_CONTINUE;
    }

    /* e = E1^{-1} [fb + (d1 z1 + d2 z2 + d3 z3)/h]; returns RMS(e/sc). */
    __device__ __forceinline__ double estimate(const double (&fb)[M], double (&e)[M]) {
        const double ih = 1.0 / h;
        LT v[M];
#pragma unroll
        for (int q = 0; q < M; ++q)
            v[q] = (LT)(fb[q] + (radau::D1 * z[0][q] + radau::D2 * z[1][q] + radau::D3 * z[2][q]) * ih);
        lu_solve_real<M, LT>(e1, p1, v);
        ++nsol;
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < M; ++q) {
            e[q] = (double)v[q];
            const double s = e[q] * isc[q];
            acc += s * s;
        }
        return __builtin_sqrt(acc * (1.0 / M));
    }

    /* After the Newton loop ends: error test, step-size control, accept or
     * reject.  Leaves phase = PH_START for the next attempt or PH_IDLE. */
    template <bool FIXED>
    __device__ __forceinline__ void finish(const Model& md, const StepParams& P, int outcome) {
        if (FIXED) {
            if (outcome == NW_FAILED) { status = ST_NEWTON; phase = PH_IDLE; return; }
            ++nstep;
            ++naccept;
#pragma unroll
            for (int q = 0; q < M; ++q) y[q] += z[2][q];
            md.rhs(y, f0);
            ++nfev;
            bool fin = true;
#pragma unroll
            for (int q = 0; q < M; ++q) fin = fin && finite_d(y[q]);
            if (!fin) { status = ST_NONFINITE; phase = PH_IDLE; return; }
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int q = 0; q < M; ++q) zold[i][q] = z[i][q];
            have_old = true;
            h_old = h;
            eta = pow(fmax(eta, UROUND), 0.8);
            phase = (naccept >= P.fixed_steps) ? PH_IDLE : PH_START;
            return;
        }
        if (outcome == NW_FAILED) {
            ++nstep;
            ++nreject;
            h *= 0.5;
            reject = true;
            if (!j_at_y0) j_stale = true;
            phase = PH_START;
            return;
        }
        double e[M];
        double err = estimate(f0, e);
        if (err >= 1.0 && (first || reject)) {
            double ye[M], fe[M];
#pragma unroll
            for (int q = 0; q < M; ++q) ye[q] = y[q] + e[q];
            md.rhs(ye, fe);
            ++nfev;
            err = estimate(fe, e);
        }
        if (!finite_d(err)) { status = ST_NONFINITE; phase = PH_IDLE; return; }
        ++nstep;
        const double kmx = (double)P.kmax;
        const double fac = 0.9 * (2.0 * kmx + 1.0) / (2.0 * kmx + (double)k);
        const double ratio =
            (err == 0.0) ? 8.0 : fmin(8.0, fmax(0.2, fac / __builtin_sqrt(__builtin_sqrt(err))));
        double h_new = h * ratio;
        if (err < 1.0) {
            if (have_acc) {
                const double r2 = (err == 0.0)
                    ? 8.0
                    : fmin(8.0, fmax(0.2, fac * (h / h_acc) * __builtin_sqrt(__builtin_sqrt(err_acc)) /
                                              __builtin_sqrt(err)));
                h_new = fmin(h_new, h * r2);
            }
            double y1[M], f1[M];
#pragma unroll
            for (int q = 0; q < M; ++q) y1[q] = y[q] + z[2][q];
            md.rhs(y1, f1);
            ++nfev;
            bool fin = true;
#pragma unroll
            for (int q = 0; q < M; ++q) fin = fin && finite_d(y1[q]) && finite_d(f1[q]);
            if (!fin) { status = ST_NONFINITE; phase = PH_IDLE; return; }
            have_acc = true;
            h_acc = h;
            err_acc = fmax(err, 1e-2);
#pragma unroll
            for (int q = 0; q < M; ++q) { y[q] = y1[q]; f0[q] = f1[q]; }
            t = last ? P.dt : t + h;
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int q = 0; q < M; ++q) zold[i][q] = z[i][q];
            h_old = h;
            have_old = true;
            eta = pow(fmax(eta, UROUND), 0.8);
            ++naccept;
            if (reject) h_new = fmin(h_new, h);
            first = false;
            reject = false;
            j_stale = !(k == 1 || theta <= 1e-3);
            j_at_y0 = false;
            if (!j_stale) {
                const double qq = h_new / h;
                if (qq >= 1.0 && qq <= 1.2) h_new = h;
            }
            h = fmin(h_new, P.dt - t);
            phase = (t < P.dt) ? PH_START : PH_IDLE;
        } else {
            ++nreject;
            h = first ? 0.1 * h : h_new;
            reject = true;
            phase = PH_START;
        }
    }
};

}  // namespace rd
