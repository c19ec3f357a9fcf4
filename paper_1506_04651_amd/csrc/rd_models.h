/*
 * rd_models.h -- right-hand sides f(u) and analytic Jacobians for the GPU
 * kernels.  Parameter blocks arrive pre-processed by the host (reciprocals
 * of the time scales instead of the time scales), laid out as stated per model.
 */
#pragma once
#include <hip/hip_runtime.h>

namespace rd {

/* BZ / Oregonator, paper §1 model II (variables a = u1, b = u2, c = u3):
 *   a' = (f c - q a - a b)/mu,  b' = (q a - a b + b (1 - b))/eps,  c' = b - c.
 * Device block: {q, f, 1/mu, 1/eps}. */
struct Oregonator {
    static constexpr int M = 3;
    static constexpr int N_DEV_PARAMS = 4;
    double q, f, imu, ieps;
    __device__ __forceinline__ explicit Oregonator(const double* __restrict__ p)
        : q(p[0]), f(p[1]), imu(p[2]), ieps(p[3]) {}
    __device__ __forceinline__ void rhs(const double (&y)[3], double (&o)[3]) const {
        const double a = y[0], b = y[1], c = y[2];
        o[0] = (f * c - q * a - a * b) * imu;
        o[1] = (q * a - a * b + b * (1.0 - b)) * ieps;
        o[2] = b - c;
    }
    __device__ __forceinline__ void jac(const double (&y)[3], double (&J)[3][3]) const {
        const double a = y[0], b = y[1];
        J[0][0] = -(q + b) * imu; J[0][1] = -a * imu;                    J[0][2] = f * imu;
        J[1][0] = (q - b) * ieps; J[1][1] = (1.0 - a - 2.0 * b) * ieps;  J[1][2] = 0.0;
        J[2][0] = 0.0;            J[2][1] = 1.0;                         J[2][2] = -1.0;
    }
};

/* Robertson kinetics (a classic stiff test with sum(u) conserved):
 *   u1' = -k1 u1 + k2 u2 u3, u2' = k1 u1 - k2 u2 u3 - k3 u2^2, u3' = k3 u2^2.
 * Device block: {k1, k2, k3}. */
struct Robertson {
    static constexpr int M = 3;
    static constexpr int N_DEV_PARAMS = 3;
    double k1, k2, k3;
    __device__ __forceinline__ explicit Robertson(const double* __restrict__ p)
        : k1(p[0]), k2(p[1]), k3(p[2]) {}
    __device__ __forceinline__ void rhs(const double (&y)[3], double (&o)[3]) const {
        const double r2 = k2 * y[1] * y[2];
        const double r3 = k3 * y[1] * y[1];
        o[0] = -k1 * y[0] + r2;
        o[1] = k1 * y[0] - r2 - r3;
        o[2] = r3;
    }
    __device__ __forceinline__ void jac(const double (&y)[3], double (&J)[3][3]) const {
        J[0][0] = -k1; J[0][1] = k2 * y[2];                     J[0][2] = k2 * y[1];
        J[1][0] = k1;  J[1][1] = -k2 * y[2] - 2.0 * k3 * y[1];  J[1][2] = -k2 * y[1];
        J[2][0] = 0.0; J[2][1] = 2.0 * k3 * y[1];               J[2][2] = 0.0;
    }
};

/* NAGUMO, paper §1 model I: f = k u^2 (1 - u).  Device block: {k}. */
struct Nagumo {
    static constexpr int M = 1;
    static constexpr int N_DEV_PARAMS = 1;
    double k;
    __device__ __forceinline__ explicit Nagumo(const double* __restrict__ p) : k(p[0]) {}
    __device__ __forceinline__ void rhs(const double (&y)[1], double (&o)[1]) const {
        o[0] = k * y[0] * y[0] * (1.0 - y[0]);
    }
    __device__ __forceinline__ void jac(const double (&y)[1], double (&J)[1][1]) const {
        J[0][0] = k * y[0] * (2.0 - 3.0 * y[0]);
    }
};

/* f = K u (tests).  Device block: K[M*M] row-major. */
template <int M_>
struct Linear {
    static constexpr int M = M_;
    static constexpr int N_DEV_PARAMS = M_ * M_;
    const double* __restrict__ K;
    __device__ __forceinline__ explicit Linear(const double* __restrict__ p) : K(p) {}
    __device__ __forceinline__ void rhs(const double (&y)[M], double (&o)[M]) const {
#pragma unroll
        for (int i = 0; i < M; ++i) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < M; ++j) s += K[i * M + j] * y[j];
            o[i] = s;
        }
    }
    __device__ __forceinline__ void jac(const double (&)[M], double (&J)[M][M]) const {
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int j = 0; j < M; ++j) J[i][j] = K[i * M + j];
    }
};

/* Mass-action style kinetics: f_i = sum_j K_ij u_j - u_i sum_k G_ik u_k,
 * J = K - diag(G u) - diag(u) G.  Device block: K[M*M], G[M*M] row-major. */
template <int M_>
struct Kinetics {
    static constexpr int M = M_;
    static constexpr int N_DEV_PARAMS = 2 * M_ * M_;
    const double* __restrict__ K;
    const double* __restrict__ G;
    __device__ __forceinline__ explicit Kinetics(const double* __restrict__ p)
        : K(p), G(p + M_ * M_) {}
    __device__ __forceinline__ void rhs(const double (&y)[M], double (&o)[M]) const {
#pragma unroll
        for (int i = 0; i < M; ++i) {
            double lin = 0.0, loss = 0.0;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                lin += K[i * M + j] * y[j];
                loss += G[i * M + j] * y[j];
            }
            o[i] = lin - y[i] * loss;
        }
    }
    __device__ __forceinline__ void jac(const double (&y)[M], double (&J)[M][M]) const {
#pragma unroll
        for (int i = 0; i < M; ++i) {
            double gu = 0.0;
#pragma unroll
            for (int k = 0; k < M; ++k) gu += G[i * M + k] * y[k];
#pragma unroll
            for (int j = 0; j < M; ++j)
                J[i][j] = K[i * M + j] - y[i] * G[i * M + j] - (i == j ? gu : 0.0);
        }
    }
};

/* Forward-difference Jacobian at y, given fy = f(y): column j =
 * (f(y + d_j e_j) - f(y)) / d_j with d_j = sqrt(u_r max(1e-5, |y_j|)), u_r the
 * unit roundoff (M more f evaluations). */
template <class Model>
__device__ __forceinline__ void fd_jacobian(const Model& md, const double (&y)[Model::M],
                                            const double (&fy)[Model::M],
                                            double (&J)[Model::M][Model::M]) {
    constexpr int M = Model::M;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        double yp[M], fp[M];
#pragma unroll
        for (int i = 0; i < M; ++i) yp[i] = y[i];
        const double dj = __builtin_sqrt(2.220446049250313e-16 * fmax(1e-5, __builtin_fabs(y[j])));
        yp[j] = y[j] + dj;
        md.rhs(yp, fp);
#pragma unroll
        for (int i = 0; i < M; ++i) J[i][j] = (fp[i] - fy[i]) / dj;
    }
}

/* An analytic model run with the finite-difference Jacobian instead. */
template <class Base>
struct FdJac : Base {
    static constexpr bool FD_JAC = true;
    using Base::Base;
};

/* Bytecode model: f given at run time as a register program (format in the
 * public header).  Device block, prepared and validated by the host:
 *   [0] L (instructions), [1] C (constants), [2 .. 2+C) constants, then L
 *   words, each an instruction packed as op | d << 8 | a << 16 | b << 24 in
 *   the low 32 bits of a 64-bit slot.
 * The program is the same for every cell, so the interpreter's control flow
 * and register indices are wave-uniform; the register file is a per-lane
 * array indexed by those uniform indices. */
constexpr int kBcRegs = 64;
enum : int { BC_ADD = 1, BC_SUB, BC_MUL, BC_DIV, BC_NEG, BC_EXP, BC_LOG, BC_POW, BC_OUT };

template <int M_>
struct Bytecode {
    static constexpr int M = M_;
    static constexpr bool FD_JAC = true;
    const double* __restrict__ p;
    __device__ __forceinline__ explicit Bytecode(const double* __restrict__ q) : p(q) {}
    __device__ __forceinline__ void rhs(const double (&y)[M], double (&o)[M]) const {
        const long long* w = reinterpret_cast<const long long*>(p);
        const int L = (int)w[0], C = (int)w[1];
        double r[kBcRegs];
#pragma unroll
        for (int i = 0; i < M; ++i) r[i] = y[i];
        for (int c = 0; c < C; ++c) r[M + c] = p[2 + c];
        const long long* ins = w + 2 + C;
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
#pragma unroll
                for (int i = 0; i < M; ++i)
                    if (d == i) o[i] = v;
            } else {
                r[d] = v;
            }
        }
    }
    /* no analytic Jacobian (FD_JAC is set) */
    __device__ __forceinline__ void jac(const double (&)[M], double (&J)[M][M]) const {
#pragma unroll
        for (int i = 0; i < M; ++i)
#pragma unroll
            for (int j = 0; j < M; ++j) J[i][j] = 0.0;
    }
};

/* FD_JAC trait with a default of false for the analytic models */
template <class Model, class = void>
struct fd_jac_of { static constexpr bool value = false; };
template <class Model>
struct fd_jac_of<Model, decltype((void)Model::FD_JAC)> { static constexpr bool value = Model::FD_JAC; };

}  // namespace rd
