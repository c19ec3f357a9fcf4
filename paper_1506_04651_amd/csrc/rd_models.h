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

}  // namespace rd
