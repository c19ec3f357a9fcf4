/*
 * rd_cell_group.h -- Radau5 for one cell held by a 16-lane group (m <= 16).
 *
 * Same method and the same decisions as the one-lane engine (rd_cell_small.h):
 * 3-stage Radau IIA, simplified Newton on the transformed stage system with
 * E1 = (gamma/h) I - J and E2 = ((alpha + i beta)/h) I - J, the error estimate
 * filtered through E1, classical + predictive step control (Hairer & Wanner,
 * §IV.8; paper §1 footnote and Appendix A).  Here lane q of the group owns
 * component q of every vector and row q of every matrix:
 *
 *  - f(u): u_j reaches every lane of the group by DPP row broadcast; the
 *    model's rows (shared by all cells) are read from LDS.
 *  - E1 and E2 are inverted explicitly, by Gauss-Jordan elimination with
 *    partial pivoting across lanes: at column k the group finds the largest
 *    |a_ik| (i > k) by a DPP butterfly max over an ordering key of the
 *    magnitude (pivot within a factor 1 + 2^-20 of the largest in FP64, exact
 *    in FP32); rows are exchanged between lanes only when that beats the
 *    diagonal (the exchange is skipped for the whole wave when no group needs
 *    it), and the pivot row is broadcast by DPP to all other lanes, which
 *    eliminate column k from their rows.  The simplified Newton iteration
 *    solves with the same two matrices several times per factorization, and
 *    with the inverse each solve is one matrix-vector product (m broadcast
 *    steps with every lane busy) instead of a forward and a backward
 *    substitution in which the lanes outside the triangle idle.  The inverse
 *    only changes how the Newton increments are rounded, not the iteration
 *    they belong to.
 *  - norms: butterfly sums, bitwise identical in all lanes, so every lane of
 *    the group takes the same control decisions; the per-cell scalars (t, h,
 *    flags, counters) are replicated in the 16 lanes.
 *
 * Lanes q >= M (when m < 16) hold zero rows and zero vectors and never take
 * part in pivoting, so they do not change any result.
 */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rd_constants.h"
#include "rd_group.h"
#include "rd_group_fused.h"
#include "rd_launch.h"
#include "rd_cell_small.h" /* status / phase / flag enums, UROUND, finite_d */

namespace rd {

__device__ __forceinline__ float absv(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double absv(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ float fmaf_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
/* v (wave-uniform, kept in a scalar register), opaque to the optimizer at
 * this point: comparisons derived from it are formed where they are used
 * instead of being hoisted out of the kernel's loop as lane masks (which
 * would be kept in, and spilled from, scalar registers) */
__device__ __forceinline__ int opaque_uniform(int v) {
    __asm__ volatile("" : "+s"(v));
    return v;
}
__device__ __forceinline__ double fmaf_t(double a, double b, double c) { return __builtin_fma(a, b, c); }

/* LDS table of the model, zero padded to 16 x 16: row q holds K[q][0..16)
 * then G[q][0..16); the stride is padded so the 16 rows fall in different
 * banks. */
struct GroupTable {
    static constexpr int STRIDE = 2 * kGroup + 2;
    static constexpr int DOUBLES = kGroup * STRIDE;
    /* the two padding columns of every row hold 1/m and 1/(3m) */
    static constexpr int INVM = 2 * kGroup, INV3M = 2 * kGroup + 1;
};

/* f_i = sum_j K_ij u_j - u_i sum_k G_ik u_k; J_ij = K_ij - u_i G_ij - d_ij (G u)_i */
struct GroupKinetics {
    static constexpr bool HAS_G = true;
};
/* f = K u; J = K */
struct GroupLinear {
    static constexpr bool HAS_G = false;
};
/* an analytic model run with the forward-difference Jacobian instead */
template <class Base>
struct GroupFd : Base {
    static constexpr bool FD_JAC = true;
};
/* f given at run time as a register program (format in the public header),
 * Jacobian by forward differences */
struct GroupBytecode {
    static constexpr bool HAS_G = false;
    static constexpr bool FD_JAC = true;
    static constexpr bool BYTECODE = true;
};
template <class Model, class = void>
struct bytecode_of { static constexpr bool value = false; };
template <class Model>
struct bytecode_of<Model, decltype((void)Model::BYTECODE)> { static constexpr bool value = Model::BYTECODE; };

/* FUSE: broadcasts fused into the multiply-adds (rd_group_fused.h); same
 * operations in the same order as the plain loops.  NC: matrix columns held
 * per lane, 16, or 8 for m <= 8 (lanes 8..15 of the group then hold zero
 * rows, as lanes m..15 do in either form; halving the columns halves the
 * matrices' registers and the elimination work). */
/* COLD: the per-cell values touched once per step or less (Z of the last
 * accepted step, the step-control scalars, the Jacobian point) live in LDS
 * slots instead of registers, which leaves more registers to the hot loop */
template <class Model, typename LT, bool FUSE = false, int NC = kGroup, bool COLD = false>
struct GroupCell {
    static_assert(NC == 8 || NC == kGroup, "8 or 16 columns");
    static constexpr int M = NC; /* loops run over NC columns; rows and columns >= m are zero */
    static constexpr bool HAS_G = Model::HAS_G;
    static constexpr bool kFused = FUSE;
    /* Jacobian by forward differences, rows kept in LDS (jl, stride jstride) */
    static constexpr bool FDJ = fd_jac_of<Model>::value;
    /* f from the register program at prog */
    static constexpr bool BC = bytecode_of<Model>::value;
    /* FP32 inverses: every solve is refined once against the FP64 matrices */
    static constexpr bool kRefine = sizeof(LT) < sizeof(double);
    int m;           /* species (run time, 1..16) */

    /* lane-q components */
    double y, f0, isc, w1, w2, w3;
    /* cold values: Z of the last accepted step, lane q's component of the
     * Jacobian point and (G u)_q there, the step-control scalars, the
     * Newton rate estimates (eta, 1/norm of the last increment) and the time
     * reached in the substep */
    enum : int { C_Z1 = 0, C_Z2, C_Z3, C_UJ, C_GJ, C_HOLD, C_IHACC, C_QACC, C_HPRE, C_ETA, C_INPREV, C_T, C_N };
    double creg[C_N];
    double* cl; /* COLD: slot i at cl[i * jstride] (LDS) */
    __device__ __forceinline__ double& cv(int i) {
        if constexpr (COLD) return cl[i * jstride];
        else return creg[i];
    }
    __device__ __forceinline__ double cv(int i) const {
        if constexpr (COLD) return cl[i * jstride];
        else return creg[i];
    }
    /* the counters, updated once per step or less: the step count is the
     * sum of accepted and rejected steps, and a step's Newton iterations
     * (k of them: 3 k f evaluations, k solves) are added when it ends;
     * COLD: in further LDS slots, the low word of slot C_N + i */
    enum : int { K_NACC = 0, K_NREJ, K_NJAC, K_NDEC, K_NFEV, K_NSOL, K_NNEWT, K_N };
    static constexpr int COLD_SLOTS = C_N + K_N; /* LDS slots per lane (COLD) */
    int kreg[K_N];
    __device__ __forceinline__ int& kc(int i) {
        if constexpr (COLD) return *reinterpret_cast<int*>(cl + (C_N + i) * jstride);
        else return kreg[i];
    }
    __device__ __forceinline__ int kc(int i) const {
        if constexpr (COLD) return *reinterpret_cast<const int*>(cl + (C_N + i) * jstride);
        else return kreg[i];
    }
    LT e1[M], e2r[M], e2i[M]; /* rows of the Gauss-Jordan inverses (see gj_real) */
    LT d1, d2r, d2i;          /* reciprocal pivots */
    int org1, org2;
    const double* kg; /* LDS row q: K at kg[0..16), G at kg[16..32) */
    double* jl;       /* FDJ: row q of J at jl[j * jstride], j < 16 (LDS) */
    int jstride;
    const double* prog; /* BC: the register program (device) */
    int q;
    bool act;         /* q < m */
    /* per-cell scalars, replicated across the group (the step-control ones
     * that change once per step are cold values, cv) */
    double h, ih;
    unsigned flags;
    int phase, status, k, nsing, outcome;

    __device__ __forceinline__ bool has(unsigned f) const { return (flags & f) != 0u; }
    __device__ __forceinline__ void set(unsigned f, bool v) { flags = v ? (flags | f) : (flags & ~f); }

    /* lin = (K u)_q and loss = (G u)_q; every lane of the group must be active */
    __device__ __forceinline__ void rows(double u, double& lin, double& loss) const {
        lin = 0.0;
        loss = 0.0;
        if constexpr (kFused) {
            if constexpr (HAS_G) {
                fused_row4<0>(u, kg, kg + kGroup, lin, loss);
                fused_row4<4>(u, kg, kg + kGroup, lin, loss);
                if constexpr (NC == 16) {
                    fused_row4<8>(u, kg, kg + kGroup, lin, loss);
                    fused_row4<12>(u, kg, kg + kGroup, lin, loss);
                }
            } else {
                fused_row4<0>(u, kg, lin);
                fused_row4<4>(u, kg, lin);
                if constexpr (NC == 16) {
                    fused_row4<8>(u, kg, lin);
                    fused_row4<12>(u, kg, lin);
                }
            }
        } else {
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const double uj = bcast_dyn(u, j);
                lin += kg[j] * uj;
                if (HAS_G) loss += kg[kGroup + j] * uj;
            }
        }
    }

    /* f_q(u) of the register program: every lane of the group gathers u,
     * runs the whole program (wave-uniform control flow and register
     * indices; the register file is a per-lane array) and keeps output q.
     * Operation by operation in program order, without contraction across
     * instructions. */
    __device__ __forceinline__ double rhs_program(double u) const {
        const long long* w = reinterpret_cast<const long long*>(prog);
        const int L = (int)w[0], C = (int)w[1];
        double r[kBcRegs];
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const double uj = bcast_dyn(u, j);
            if (j < m) r[j] = uj;
        }
        for (int c = 0; c < C; ++c) r[m + c] = prog[2 + c];
        const long long* ins = w + 2 + C;
        double out = 0.0;
        for (int k = 0; k < L; ++k) {
            const unsigned x = (unsigned)ins[k];
            const int op = (int)(x & 0xffu), d = (int)((x >> 8) & 0xffu);
            const int a = (int)((x >> 16) & 0xffu), b = (int)(x >> 24);
            const double va = r[a], vb = r[b];
            double v;
            switch (op) {
            case BC_ADD: v = va + vb; break;
            case BC_SUB: v = va - vb; break;
            case BC_MUL: v = va * vb; break;
            case BC_DIV: v = va / vb; break;
            case BC_NEG: v = -va; break;
            case BC_EXP: v = exp(va); break;
            case BC_LOG: v = log(va); break;
            case BC_POW: v = pow(va, vb); break;
            default: v = va; break; /* BC_OUT */
            }
            if (op == BC_OUT) {
                if (d == q) out = v;
            } else {
                r[d] = v;
            }
        }
        return out;
    }

    /* The rows of the model for the forward-difference Jacobian: each
     * product and sum rounded on its own, in column order from +0, so that
     * f, and the differences of f that make up the Jacobian, round like the
     * plain sums of the definition (a rounding difference in f is amplified
     * by 1/d_j ~ 1e8 in a difference quotient). */
    __device__ __forceinline__ double rhs_plain(double u, double& gu) const {
#pragma clang fp contract(off)
        double lin = 0.0, loss = 0.0;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const double uj = bcast_dyn(u, j);
            if (j < m) {
                lin += kg[j] * uj;
                if (HAS_G) loss += kg[kGroup + j] * uj;
            }
        }
        gu = loss;
        return HAS_G ? lin - u * loss : lin;
    }

    /* f_q(u) and (G u)_q; every lane of the group must be active */
    __device__ __forceinline__ double rhs(double u, double& gu) const {
        if constexpr (BC) {
            gu = 0.0;
            return rhs_program(u);
        } else if constexpr (FDJ) {
            return rhs_plain(u, gu);
        } else {
            double lin, loss;
            rows(u, lin, loss);
            gu = loss;
            return HAS_G ? lin - u * loss : lin;
        }
    }

    /* f_q at the three stage arguments of a Newton iteration; for the fused
     * kinetics rows in one pass over the model rows (each LDS row entry read
     * once), which gives the bits of three rhs calls */
    __device__ __forceinline__ void rhs3(double u1, double u2, double u3, double& F1, double& F2,
                                         double& F3) const {
        if constexpr (kFused && HAS_G && !BC && !FDJ) {
            double lin[3] = {0.0, 0.0, 0.0}, loss[3] = {0.0, 0.0, 0.0};
            fused_row4x3<0>(u1, u2, u3, kg, kg + kGroup, lin, loss);
            fused_row4x3<4>(u1, u2, u3, kg, kg + kGroup, lin, loss);
            if constexpr (NC == 16) {
                fused_row4x3<8>(u1, u2, u3, kg, kg + kGroup, lin, loss);
                fused_row4x3<12>(u1, u2, u3, kg, kg + kGroup, lin, loss);
            }
            F1 = lin[0] - u1 * loss[0];
            F2 = lin[1] - u2 * loss[1];
            F3 = lin[2] - u3 * loss[2];
        } else {
            double gu;
            F1 = rhs(u1, gu);
            F2 = rhs(u2, gu);
            F3 = rhs(u3, gu);
        }
    }

    /* (J x)_q with the current Jacobian: from the LDS rows (forward
     * differences), else (K x)_q - uJ (G x)_q - gJ x_q at the stored point */
    __device__ __forceinline__ double jmul(double x) const {
        if constexpr (FDJ) {
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const double xj = bcast_dyn(x, j);
                if (j < m) acc += jl[j * jstride] * xj;
            }
            return acc;
        } else {
            double lin, loss;
            rows(x, lin, loss);
            return HAS_G ? lin - cv(C_UJ) * loss - cv(C_GJ) * x : lin;
        }
    }

    /* jmul at three arguments; for the fused kinetics rows in one pass over
     * the model rows, with the bits of three jmul calls */
    __device__ __forceinline__ void jmul3(double x1, double x2, double x3, double& j1, double& j2,
                                          double& j3) const {
        if constexpr (kFused && HAS_G && !BC && !FDJ) {
            double lin[3] = {0.0, 0.0, 0.0}, loss[3] = {0.0, 0.0, 0.0};
            fused_row4x3<0>(x1, x2, x3, kg, kg + kGroup, lin, loss);
            fused_row4x3<4>(x1, x2, x3, kg, kg + kGroup, lin, loss);
            if constexpr (NC == 16) {
                fused_row4x3<8>(x1, x2, x3, kg, kg + kGroup, lin, loss);
                fused_row4x3<12>(x1, x2, x3, kg, kg + kGroup, lin, loss);
            }
            const double uj = cv(C_UJ), gj = cv(C_GJ);
            j1 = lin[0] - uj * loss[0] - gj * x1;
            j2 = lin[1] - uj * loss[1] - gj * x2;
            j3 = lin[2] - uj * loss[2] - gj * x3;
        } else {
            j1 = jmul(x1);
            j2 = jmul(x2);
            j3 = jmul(x3);
        }
    }

    /* Forward-difference Jacobian at y with f0 = f(y): column j =
     * (f(y + d_j e_j) - f(y)) / d_j, d_j = sqrt(u_r max(1e-5, |y_j|)); lane q
     * stores J_qj in its LDS row (zero rows for q >= m); m f evaluations. */
    __device__ __forceinline__ void fd_jacobian() {
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const double yj = bcast_dyn(y, j);
            if (j < m) {
                const double dj = __builtin_sqrt(2.220446049250313e-16 * fmax(1e-5, __builtin_fabs(yj)));
                double gu;
                const double fp = rhs(q == j ? y + dj : y, gu);
                jl[j * jstride] = act ? (fp - f0) / dj : 0.0;
            }
        }
        kc(K_NFEV) += m;
    }

    __device__ __forceinline__ void load(const StepParams& P, const double* __restrict__ states,
                                         int64_t n, int64_t c, const double* __restrict__ hcell) {
        y = act ? states[(int64_t)q * n + c] : 0.0;
        kc(K_NACC) = kc(K_NREJ) = kc(K_NJAC) = kc(K_NDEC) = 0;
        kc(K_NSOL) = kc(K_NNEWT) = 0;
        kc(K_NFEV) = 1;
        double gu;
        f0 = rhs(y, gu);
        status = ST_OK;
        const bool fin = grp_bits(finite_d(y) && finite_d(f0)) == 0xFFFFu;
        cv(C_T) = 0.0;
        const double hw = hcell ? hcell[c] : 0.0;
        h = P.fixed_steps > 0 ? P.dt / P.fixed_steps
                              : fmin(hw > 0.0 ? hw : (P.h0 > 0.0 ? P.h0 : P.dt), P.dt);
        cv(C_HPRE) = fin ? h : 0.0;
        cv(C_HOLD) = cv(C_IHACC) = cv(C_QACC) = cv(C_INPREV) = 0.0;
        cv(C_ETA) = 1.0;
        k = 0;
        nsing = 0;
        flags = F_FIRST | F_JSTALE;
        w1 = 0.0;
        w2 = 0.0;
        w3 = 0.0;
        cv(C_Z1) = 0.0;
        cv(C_Z2) = 0.0;
        cv(C_Z3) = 0.0;
        phase = fin ? PH_START : PH_IDLE;
        if (!fin) status = ST_NONFINITE;
    }

    __device__ __forceinline__ void store(double* __restrict__ states, int32_t* __restrict__ stats,
                                          int64_t n, int64_t c, double* __restrict__ hcell) const {
        if (act) states[(int64_t)q * n + c] = y;
        if (hcell && q == 0) hcell[c] = cv(C_HPRE);
        if (stats && q == 0) {
            stats[0 * n + c] = status;
            stats[1 * n + c] = kc(K_NACC) + kc(K_NREJ);
            stats[2 * n + c] = kc(K_NACC);
            stats[3 * n + c] = kc(K_NREJ);
            stats[4 * n + c] = kc(K_NFEV);
            stats[5 * n + c] = kc(K_NJAC);
            stats[6 * n + c] = kc(K_NDEC);
            stats[7 * n + c] = kc(K_NSOL);
            stats[8 * n + c] = kc(K_NNEWT);
        }
    }

    /* J_qj at the stored Jacobian point (uJ, gJ = (G u)_q at that point), or
     * from the LDS row of the forward-difference Jacobian */
    __device__ __forceinline__ double jac(int j, int qv, bool av) const {
        if constexpr (FDJ) return (av && j < m) ? jl[j * jstride] : 0.0;
        double v = kg[j];
        if (HAS_G) {
            v -= cv(C_UJ) * kg[kGroup + j];
            if (j == qv) v -= cv(C_GJ);
        }
        return av ? v : 0.0;
    }
    __device__ __forceinline__ double jac(int j) const { return jac(j, q, act); }

    /* ---- inverse of E1 (real) by Gauss-Jordan with partial pivoting ----
     * Step kk: the pivot row (after the exchange, lane kk) is left unscaled;
     * every other lane q subtracts f_q = a_q,kk / p_kk times it from its own
     * row (f = 0 in the pivot lane, so the update runs in all lanes without a
     * select) and stores -f_q in column kk, the pivot lane stores 1 there and
     * keeps d = 1 / p_kk.  At the end lane q holds row q of R with
     * (P E)^{-1} = diag(d) R, P the row exchanges (org: source row of lane q).
     * The pivots, and so the singularity test, are those of the LU
     * factorization with the same pivoting.
     * SAFE: reciprocal pivots by rcp (library division outside its fast
     * range); returns false for a zero pivot.  Otherwise by rcp_nr alone,
     * and false as soon as a pivot lies outside rcp_nr's range (the caller
     * then repeats the inversion with SAFE; inside the range both give the
     * same bits). */
    template <bool SAFE>
    __device__ __forceinline__ bool gj_real(LT (&a)[M], LT& d, int& org) {
        bool ok = true;
        const int q = grp_lane_here();
        const int m = opaque_uniform(this->m);
        const bool act = q < m;
        org = q;
        d = LT(0);
#pragma unroll
        for (int kk = 0; kk < M; ++kk) {
            if (kk < m) {
                const bool below = act && q > kk;
                const unsigned key = below ? mag_key(absv(a[kk])) : 0u;
                LT akk = bcast_dyn(a[kk], kk);
                const unsigned kd = mag_key(absv(akk));
                /* an exchange is needed in a group iff one of its lanes
                 * below the diagonal holds a larger key than the diagonal;
                 * the group maximum is formed only then (rarely) */
                if (__ballot(key > kd) != 0ull) {
                    const unsigned kmax = grp_max_u(key);
                    const bool need = kmax > kd;
                    const unsigned cand = grp_bits(below && key == kmax);
                    const int p = (need && cand) ? __ffs(cand) - 1 : kk;
                    const int src = (q == kk) ? p : (q == p ? kk : q);
#pragma unroll
                    for (int j = 0; j < M; ++j) a[j] = grp_shfl(a[j], src);
                    org = grp_shfl(org, src);
                    akk = bcast_dyn(a[kk], kk);
                }
                LT inv;
                if constexpr (SAFE) {
                    ok = ok && (akk != LT(0));
                    inv = rcp(akk);
                } else {
                    ok = ok && rcp_nr_ok(akk);
                    inv = rcp_nr(akk);
                }
                const bool piv = q == kk;
                const LT f = piv ? LT(0) : a[kk] * inv;
                if constexpr (kFused) {
                    fused_gj_real<NC>(a, f, kk);
                } else {
#pragma unroll
                    for (int j = 0; j < M; ++j)
                        if (j != kk) a[j] = fmaf_t(-f, bcast_dyn(a[j], kk), a[j]);
                }
                a[kk] = piv ? LT(1) : -f;
                d = piv ? inv : d;
            }
        }
        return ok;
    }

    /* ---- inverse of E2 (complex), same scheme in complex arithmetic ---- */
    template <bool SAFE>
    __device__ __forceinline__ bool gj_cplx(LT (&ar)[M], LT (&ai)[M], LT& dr, LT& di, int& org) {
        bool ok = true;
        const int q = grp_lane_here();
        const int m = opaque_uniform(this->m);
        const bool act = q < m;
        org = q;
        dr = di = LT(0);
#pragma unroll
        for (int kk = 0; kk < M; ++kk) {
            if (kk < m) {
                const bool below = act && q > kk;
                const unsigned key = below ? mag_key(ar[kk] * ar[kk] + ai[kk] * ai[kk]) : 0u;
                LT pr = bcast_dyn(ar[kk], kk), pi = bcast_dyn(ai[kk], kk);
                const unsigned kd = mag_key(pr * pr + pi * pi);
                if (__ballot(key > kd) != 0ull) {
                    const unsigned kmax = grp_max_u(key);
                    const bool need = kmax > kd;
                    const unsigned cand = grp_bits(below && key == kmax);
                    const int p = (need && cand) ? __ffs(cand) - 1 : kk;
                    const int src = (q == kk) ? p : (q == p ? kk : q);
#pragma unroll
                    for (int j = 0; j < M; ++j) {
                        ar[j] = grp_shfl(ar[j], src);
                        ai[j] = grp_shfl(ai[j], src);
                    }
                    org = grp_shfl(org, src);
                    pr = bcast_dyn(ar[kk], kk);
                    pi = bcast_dyn(ai[kk], kk);
                }
                /* 1 / (pr + i pi) = (pr - i pi) / (pr^2 + pi^2) */
                const LT nn = pr * pr + pi * pi;
                LT ir, ii;
                if constexpr (SAFE) {
                    ok = ok && !(pr == LT(0) && pi == LT(0));
                    if (rcp_nr_ok(nn)) {
                        const LT rn = rcp_nr(nn);
                        ir = pr * rn;
                        ii = -pi * rn;
                    } else {
                        const auto z = slow_crcp(pr, pi);
                        ir = z.x;
                        ii = z.y;
                    }
                } else {
                    ok = ok && rcp_nr_ok(nn);
                    const LT rn = rcp_nr(nn);
                    ir = pr * rn;
                    ii = -pi * rn;
                }
                const bool piv = q == kk;
                const LT xr = ar[kk], xi = ai[kk];
                const LT fr = piv ? LT(0) : xr * ir - xi * ii;
                const LT fi = piv ? LT(0) : xr * ii + xi * ir;
                if constexpr (kFused) {
                    fused_gj_cplx<NC>(ar, ai, fr, fi, kk);
                } else {
#pragma unroll
                    for (int j = 0; j < M; ++j) {
                        if (j != kk) {
                            const LT ur = bcast_dyn(ar[j], kk), ui = bcast_dyn(ai[j], kk);
                            ar[j] = fmaf_t(-fr, ur, fmaf_t(fi, ui, ar[j]));
                            ai[j] = fmaf_t(-fr, ui, fmaf_t(-fi, ur, ai[j]));
                        }
                    }
                }
                ar[kk] = piv ? LT(1) : -fr;
                ai[kk] = piv ? LT(0) : -fi;
                dr = piv ? ir : dr;
                di = piv ? ii : di;
            }
        }
        return ok;
    }

    /* x = E1^{-1} b = diag(d) R (P b); lane q holds b_q on entry, x_q on return */
    __device__ __forceinline__ LT solve_real(LT b) const {
        /* the lane's row index from the lane id (cheaper than keeping q live) */
        if (__ballot(org1 != grp_lane_here()) != 0ull) b = grp_shfl(b, org1);
        if constexpr (kFused) {
            if (m == M) {
                if constexpr (NC == 16) return fused_mv16(e1, b) * d1;
                else return fused_mv8(e1, b) * d1;
            }
        }
        LT acc = LT(0);
#pragma unroll
        for (int j = 0; j < M; ++j)
            if (j < m) acc = fmaf_t(e1[j], bcast_dyn(b, j), acc);
        return acc * d1;
    }

    __device__ __forceinline__ void solve_cplx(LT& br, LT& bi) const {
        if (__ballot(org2 != grp_lane_here()) != 0ull) {
            br = grp_shfl(br, org2);
            bi = grp_shfl(bi, org2);
        }
        LT sr = LT(0), si = LT(0);
        bool done = false;
        if constexpr (kFused) {
            if (m == M) {
                if constexpr (NC == 16) fused_cmv16(e2r, e2i, br, bi, sr, si);
                else fused_cmv8(e2r, e2i, br, bi, sr, si);
                done = true;
            }
        }
        if (!done) {
#pragma unroll
            for (int j = 0; j < M; ++j) {
                if (j < m) {
                    const LT ur = bcast_dyn(br, j), ui = bcast_dyn(bi, j);
                    sr = fmaf_t(e2r[j], ur, fmaf_t(-e2i[j], ui, sr));
                    si = fmaf_t(e2r[j], ui, fmaf_t(e2i[j], ur, si));
                }
            }
        }
        br = sr * d2r - si * d2i;
        bi = sr * d2i + si * d2r;
    }

    /* rows q of E1 = (gamma/h) I - J and E2 = ((alpha + i beta)/h) I - J */
    __device__ __forceinline__ void form_e() {
        const double g = radau::GAMMA * ih, ar = radau::ALPHA * ih, bi = radau::BETA * ih;
        const int qv = grp_lane_here();
        const bool av = qv < m;
#pragma unroll
        for (int j = 0; j < M; ++j) {
            const double mj = -jac(j, qv, av);
            const bool d = av && j == qv;
            e1[j] = (LT)(d ? g + mj : mj);
            e2r[j] = (LT)(d ? ar + mj : mj);
            e2i[j] = (LT)(d ? bi : 0.0);
        }
    }

    /* Both inverses; false if E1 or E2 is singular.  A group whose pivots
     * leave the fast reciprocal's range (rare: near-singular or badly scaled
     * matrices) inverts again with the safe reciprocal, so every group ends
     * with the bits of the safe inversion. */
    __device__ __forceinline__ bool factor() {
        form_e();
        bool ok1 = gj_real<false>(e1, d1, org1);
        bool ok2 = gj_cplx<false>(e2r, e2i, d2r, d2i, org2);
        const bool redo = !(ok1 && ok2); /* group-uniform */
        if (__ballot(redo) != 0ull) {
            if (redo) {
                form_e();
                ok1 = gj_real<true>(e1, d1, org1);
                ok2 = gj_cplx<true>(e2r, e2i, d2r, d2i, org2);
            }
        }
        return ok1 && ok2;
    }

    template <bool FIXED>
    __device__ __forceinline__ void start(const StepParams& P) {
        if (!FIXED) {
            cv(C_HPRE) = h;
            if (kc(K_NACC) + kc(K_NREJ) >= P.max_steps) { status = ST_MAXSTEPS; phase = PH_IDLE; return; }
            if (h < P.h_min) { status = ST_HSMALL; phase = PH_IDLE; return; }
            const bool last = cv(C_T) + 1.0001 * h >= P.dt;
            if (last) {
                const double hl = P.dt - cv(C_T);
                if (hl != h) flags &= ~F_LUOK;
                h = hl;
            }
            set(F_LAST, last);
        }
        ih = rcp(h);
        isc = act ? rcp(P.atol + P.rtol * __builtin_fabs(y)) : 0.0;
        if (FIXED || has(F_JSTALE)) {
            if constexpr (FDJ) {
                fd_jacobian();
            } else {
                double gu;
                (void)rhs(y, gu);
                cv(C_UJ) = y;
                cv(C_GJ) = gu;
            }
            ++kc(K_NJAC);
            flags = (flags & ~(F_JSTALE | F_LUOK)) | F_JATY0;
        }
        RD_PH_BEGIN(ph_f)
        if (FIXED || !has(F_LUOK)) {
            ++kc(K_NDEC);
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
        /* start values (zero on the cell's first step); every branch ends in
         * the same single assignment of w1, w2, w3 */
        double za = 0.0, zb = 0.0, zc = 0.0;
        if (has(F_OLD)) {
            const double r = h * rcp(cv(C_HOLD));
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
            const double v0 = -cv(C_Z3), v1 = cv(C_Z1) - cv(C_Z3), v2 = cv(C_Z2) - cv(C_Z3);
            za = Lw[0][0] * v0 + Lw[0][1] * v1 + Lw[0][2] * v2;
            zb = Lw[1][0] * v0 + Lw[1][1] * v1 + Lw[1][2] * v2;
            zc = Lw[2][0] * v0 + Lw[2][1] * v1 + Lw[2][2] * v2;
        }
        w1 = radau::TI11 * za + radau::TI12 * zb + radau::TI13 * zc;
        w2 = radau::TI21 * za + radau::TI22 * zb + radau::TI23 * zc;
        w3 = radau::TI31 * za + radau::TI32 * zb + radau::TI33 * zc;
        k = 0;
        cv(C_INPREV) = 0.0;
        phase = PH_NEWTON;
    }

    __device__ __forceinline__ int newton(const StepParams& P) {
        ++k;
        double G1, G2, G3, Fs1, Fs2, Fs3;
        {
            const double z1 = radau::T11 * w1 + radau::T12 * w2 + radau::T13 * w3;
            const double z2 = radau::T21 * w1 + radau::T22 * w2 + radau::T23 * w3;
            const double z3 = w1 + w2;
            rhs3(y + z1, y + z2, y + z3, Fs1, Fs2, Fs3);
        }
        G1 = radau::TI11 * Fs1;
        G2 = radau::TI21 * Fs1;
        G3 = radau::TI31 * Fs1;
        G1 += radau::TI12 * Fs2;
        G2 += radau::TI22 * Fs2;
        G3 += radau::TI32 * Fs2;
        G1 += radau::TI13 * Fs3;
        G2 += radau::TI23 * Fs3;
        G3 += radau::TI33 * Fs3;
        const double g = radau::GAMMA * ih, al = radau::ALPHA * ih, be = radau::BETA * ih;
        const double b1 = G1 - g * w1, b2 = G2 - al * w2 + be * w3, b3 = G3 - be * w2 - al * w3;
        const LT r1 = solve_real((LT)b1);
        LT r2 = (LT)b2, r3 = (LT)b3;
        solve_cplx(r2, r3);
        double d1 = (double)r1, d2 = (double)r2, d3 = (double)r3;
        if constexpr (kRefine) {
            /* one step of iterative refinement against the FP64 matrices
             * E1 = g I - J, E2 = (al + i be) I - J: x += E32^{-1} (b - E x) */
            double j1, j2, j3;
            jmul3(d1, d2, d3, j1, j2, j3);
            const LT c1 = solve_real((LT)(b1 - g * d1 + j1));
            LT c2 = (LT)(b2 - al * d2 + be * d3 + j2), c3 = (LT)(b3 - be * d2 - al * d3 + j3);
            solve_cplx(c2, c3);
            d1 += (double)c1;
            d2 += (double)c2;
            d3 += (double)c3;
        }
        w1 += d1;
        w2 += d2;
        w3 += d3;
        const double dz1 = radau::T11 * d1 + radau::T12 * d2 + radau::T13 * d3;
        const double dz2 = radau::T21 * d1 + radau::T22 * d2 + radau::T23 * d3;
        const double dz3 = d1 + d2;
        const double s1 = dz1 * isc, s2 = dz2 * isc, s3 = dz3 * isc;
        const double acc = grp_sum(s1 * s1 + s2 * s2 + s3 * s3);
        const double nk = sqrt_f(acc * kg[GroupTable::INV3M]);
        if (!finite_d(nk)) return NW_FAILED;
        const double tol = P.newton_tol;
        if (k >= 2) {
            const double th = nk * cv(C_INPREV);
            if (th >= 0.99) return NW_FAILED;
            const double om = 1.0 - th;
            cv(C_ETA) = th * rcp_nr(om);
            double tp = 1.0;
            for (int j = 0; j < P.kmax - k; ++j) tp *= th;
            if (tp * nk > tol * om) return NW_FAILED;
            set(F_KEEPJ, th <= 1e-3);
        } else {
            set(F_KEEPJ, true);
        }
        if (cv(C_ETA) * nk <= tol) return NW_CONVERGED;
        cv(C_INPREV) = rcp(nk); /* nk > 0: nk == 0 converges above */
        return k >= P.kmax ? NW_FAILED : NW_CONTINUE;
    }

    __device__ __forceinline__ double estimate(double fb, double& e) {
        constexpr double DW1 = radau::D1 * radau::T11 + radau::D2 * radau::T21 + radau::D3;
        constexpr double DW2 = radau::D1 * radau::T12 + radau::D2 * radau::T22 + radau::D3;
        constexpr double DW3 = radau::D1 * radau::T13 + radau::D2 * radau::T23;
        const double b = fb + (DW1 * w1 + DW2 * w2 + DW3 * w3) * ih;
        const LT v = solve_real((LT)b);
        ++kc(K_NSOL);
        e = (double)v;
        if constexpr (kRefine) {
            const LT c = solve_real((LT)(b - (radau::GAMMA * ih) * e + jmul(e)));
            e += (double)c;
        }
        const double s = e * isc;
        return sqrt_f(grp_sum(s * s) * kg[GroupTable::INVM]);
    }

    template <bool FIXED>
    __device__ __forceinline__ void finish(const StepParams& P, int oc) {
        kc(K_NNEWT) += k;
        kc(K_NSOL) += k;
        kc(K_NFEV) += 3 * k;
        if (FIXED) {
            if (oc == NW_FAILED) { status = ST_NEWTON; phase = PH_IDLE; return; }
            ++kc(K_NACC);
            cv(C_Z1) = radau::T11 * w1 + radau::T12 * w2 + radau::T13 * w3;
            cv(C_Z2) = radau::T21 * w1 + radau::T22 * w2 + radau::T23 * w3;
            cv(C_Z3) = w1 + w2;
            y += cv(C_Z3);
            double gu;
            f0 = rhs(y, gu);
            ++kc(K_NFEV);
            flags |= F_OLD;
            if (grp_bits(finite_d(y)) != 0xFFFFu) { status = ST_NONFINITE; phase = PH_IDLE; return; }
            cv(C_HOLD) = h;
            cv(C_ETA) = pow08(fmax(cv(C_ETA), UROUND));
            phase = (kc(K_NACC) >= P.fixed_steps) ? PH_IDLE : PH_START;
            return;
        }
        if (oc == NW_FAILED) {
            ++kc(K_NREJ);
            h *= 0.5;
            flags = (flags | F_REJECT) & ~F_LUOK;
            if (!has(F_JATY0)) flags |= F_JSTALE;
            phase = PH_START;
            return;
        }
        double e;
        double err = estimate(f0, e);
        if (err >= 1.0 && (flags & (F_FIRST | F_REJECT))) {
            double gu;
            const double fe = rhs(y + e, gu);
            ++kc(K_NFEV);
            err = estimate(fe, e);
        }
        if (!finite_d(err)) { status = ST_NONFINITE; phase = PH_IDLE; return; }
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
                    : fmin(8.0, fmax(0.2, fac * (h * cv(C_IHACC)) * cv(C_QACC) * (s * s)));
                h_new = fmin(h_new, h * r2);
            }
            const double zz1 = radau::T11 * w1 + radau::T12 * w2 + radau::T13 * w3;
            const double zz2 = radau::T21 * w1 + radau::T22 * w2 + radau::T23 * w3;
            const double zz3 = w1 + w2;
            const double y1 = y + zz3;
            double gu;
            const double f1 = rhs(y1, gu);
            ++kc(K_NFEV);
            if (grp_bits(finite_d(y1) && finite_d(f1)) != 0xFFFFu) {
                status = ST_NONFINITE;
                phase = PH_IDLE;
                return;
            }
            cv(C_IHACC) = ih;
            /* max(err, 1e-2)^(1/4); (1e-2)^(1/4) = sqrt(0.1) */
            cv(C_QACC) = err >= 1e-2 ? rcp_nr(s) : 0.31622776601683794;
            y = y1;
            f0 = f1;
            cv(C_Z1) = zz1;
            cv(C_Z2) = zz2;
            cv(C_Z3) = zz3;
            const double t = has(F_LAST) ? P.dt : cv(C_T) + h;
            cv(C_T) = t;
            cv(C_HOLD) = h;
            cv(C_ETA) = pow08(fmax(cv(C_ETA), UROUND));
            ++kc(K_NACC);
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
            ++kc(K_NREJ);
            const double hn = has(F_FIRST) ? 0.1 * h : h_new;
            if (hn != h) flags &= ~F_LUOK;
            h = hn;
            flags |= F_REJECT;
            phase = PH_START;
        }
    }
};

}  // namespace rd
