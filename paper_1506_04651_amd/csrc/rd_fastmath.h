/*
 * rd_fastmath.h -- short FP64 forms of the few non-polynomial operations the
 * step control needs (reciprocal, square root, err^(-1/4), x^0.8).
 *
 * Each takes a hardware estimate (v_rcp_f64, v_rsq_f64, or the FP32
 * v_log_f32 / v_exp_f32 pair) and refines it with Newton steps in FP64, which
 * converge quadratically; two steps from an estimate good to ~1e-7 leave an
 * error of a few units in the last place, the size of the rounding
 * differences that already separate any two orderings of the same arithmetic.
 * Arguments outside the range where the estimate is safe (zero, denormal,
 * huge, non-finite) take the library operation instead, in an out-of-line
 * call that runs only in the lanes that need it (and is skipped when no lane
 * of the wave does).
 */
#pragma once
#include <hip/hip_runtime.h>

namespace rd {

constexpr double kFastLo = 1e-280, kFastHi = 1e280; /* refined forms valid inside */

/* The library operations of the out-of-range branches, kept out of line: they
 * run almost never, and inlined (pow especially) their constants would be
 * hoisted into registers of the kernels' main loops and spilled. */
__device__ __noinline__ double slow_rcp(double a) { return 1.0 / a; }
__device__ __noinline__ double slow_sqrt(double x) { return __builtin_sqrt(x); }
__device__ __noinline__ double slow_rroot4(double x) { return 1.0 / __builtin_sqrt(__builtin_sqrt(x)); }
__device__ __noinline__ double slow_pow08(double x) { return pow(x, 0.8); }
__device__ __noinline__ float slow_rcpf(float a) { return 1.0f / a; }
/* 1 / (pr + i pi) where pr^2 + pi^2 leaves the reciprocal's safe range (the
 * square overflows or underflows although the pivot itself is
 * representable): both parts are first divided by the larger magnitude.
 * Returns (Re, Im); zero in, non-finite out. */
__device__ __noinline__ double2 slow_crcp(double pr, double pi) {
    const double s = fmax(__builtin_fabs(pr), __builtin_fabs(pi));
    const double a = pr / s, b = pi / s;
    const double d = s * (a * a + b * b);
    return make_double2(a / d, -b / d);
}
__device__ __noinline__ float2 slow_crcp(float pr, float pi) {
    const float s = fmaxf(__builtin_fabsf(pr), __builtin_fabsf(pi));
    const float a = pr / s, b = pi / s;
    const float d = s * (a * a + b * b);
    return make_float2(a / d, -b / d);
}
constexpr float kSeedLo = 1e-30f, kSeedHi = 1e30f;  /* FP32 seeds valid inside */

/* 1/a for |a| in [kFastLo, kFastHi]: v_rcp_f64 and two Newton steps
 * r <- r + r (1 - a r). */
__device__ __forceinline__ double rcp_nr(double a) {
    double r = __builtin_amdgcn_rcp(a);
    r = __builtin_fma(__builtin_fma(-a, r, 1.0), r, r);
    r = __builtin_fma(__builtin_fma(-a, r, 1.0), r, r);
    return r;
}

/* a inside the range where rcp_nr is valid (false for zero, denormals,
 * huge and non-finite values) */
__device__ __forceinline__ bool rcp_nr_ok(double a) {
    const double aa = __builtin_fabs(a);
    return aa >= kFastLo && aa <= kFastHi;
}

__device__ __forceinline__ double rcp(double a) {
    double r = rcp_nr(a);
    const bool ok = rcp_nr_ok(a);
    if (!ok) r = slow_rcp(a);
    return r;
}
/* FP32: v_rcp_f32 and one Newton step, IEEE division outside [1e-36, 1e36]. */
__device__ __forceinline__ float rcp_nr(float a) {
    const float r = __builtin_amdgcn_rcpf(a);
    return __builtin_fmaf(__builtin_fmaf(-a, r, 1.0f), r, r);
}
__device__ __forceinline__ bool rcp_nr_ok(float a) {
    const float aa = __builtin_fabsf(a);
    return aa >= 1e-36f && aa <= 1e36f;
}
__device__ __forceinline__ float rcp(float a) {
    float r = rcp_nr(a);
    const bool ok = rcp_nr_ok(a);
    if (!ok) r = slow_rcpf(a);
    return r;
}

/* sqrt(x), x >= 0: v_rsq_f64 refined twice (r <- r + r (1 - x r^2) / 2), then
 * s = x r with one residual correction s <- s + (r / 2) (x - s^2). */
__device__ __forceinline__ double sqrt_nr(double x) {
    double r = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    r = __builtin_fma(__builtin_fma(-hx * r, r, 0.5), r, r);
    r = __builtin_fma(__builtin_fma(-hx * r, r, 0.5), r, r);
    double s = x * r;
    s = __builtin_fma(__builtin_fma(-s, s, x), 0.5 * r, s);
    return s;
}
__device__ __forceinline__ double sqrt_f(double x) {
    double s = sqrt_nr(x);
    const bool ok = x >= kFastLo && x <= kFastHi;
    if (!ok) s = slow_sqrt(x);
    return s;
}

/* x^(-1/4), x > 0: FP32 seed 2^(-log2(x)/4), then two Newton steps on
 * y^-4 = x:  y <- y + (y / 4) (1 - x y^4). */
__device__ __forceinline__ double rroot4(double x) {
    const float xf = (float)x;
    double y = (double)__builtin_amdgcn_exp2f(-0.25f * __builtin_amdgcn_logf(xf));
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double y2 = y * y;
        const double e = __builtin_fma(-x * y2, y2, 1.0);
        y = __builtin_fma(0.25 * y, e, y);
    }
    const bool ok = x >= (double)kSeedLo && x <= (double)kSeedHi;
    if (!ok) y = slow_rroot4(x);
    return y;
}

/* x^p with p the double nearest 0.8 (= 4/5 + 2^-53 * 2/5), x > 0: FP32 seed
 * 2^(0.8 log2 x), two Newton steps on y^5 = x^4 (y <- 0.8 y + 0.2 (x/y)^4),
 * which give x^(4/5), then the factor x^(p - 4/5) = 1 + (p - 4/5) ln x. */
__device__ __forceinline__ double pow08(double x) {
    constexpr double kDeltaLn2 = 0.4 / 9007199254740992.0 * 0.6931471805599453; /* (p - 4/5) ln 2 */
    const float lg = __builtin_amdgcn_logf((float)x);
    double y = (double)__builtin_amdgcn_exp2f(0.8f * lg);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double r = x * rcp_nr(y);
        const double r2 = r * r;
        y = __builtin_fma(0.2 * r2, r2, 0.8 * y);
    }
    y = __builtin_fma(y, kDeltaLn2 * (double)lg, y);
    const bool ok = x >= (double)kSeedLo && x <= (double)kSeedHi;
    if (!ok) y = slow_pow08(x);
    return y;
}

}  // namespace rd
