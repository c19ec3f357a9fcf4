/*
 * rd_group_fused.h -- broadcast multiply-adds of the 16-lane engine in one
 * instruction each.
 *
 * On gfx950 v_fmac_f64 and v_fmac_f32 accept a DPP source operand with the
 * row_newbcast control:  d += x(lane j of the 16-lane row) * y, rounded once
 * like fma.  The compiler does not fold a DPP move into the multiply-add, so
 * every broadcast would cost a v_mov_b64_dpp (and often a hazard s_nop) in
 * front of the FMA.  The helpers below issue the fused form as inline
 * assembly, one block per matrix-vector product, per chunk of the model's
 * right-hand side, or per Gauss-Jordan elimination step.
 *
 * Each helper performs, operation by operation and in the same order, the
 * multiply-adds of the plain loops it replaces (same operands, same single
 * rounding), so results are those of the plain code.
 *
 * Hazards: a DPP read of a register needs two wait states after a VALU
 * instruction wrote it, and the compiler's hazard tracking does not see
 * inside the blocks.  Every block therefore starts and ends with s_nop 1,
 * and inside a block no instruction reads through DPP a register that one of
 * the two instructions before it wrote.  As for every row broadcast, all 16
 * lanes of the row must be active.
 */
#pragma once
#include <hip/hip_runtime.h>

namespace rd {

/* OP: "v_fmac_f64_dpp" or "v_fmac_f32_dpp" (the FP32 form serves the
 * mixed-precision factors and solves) */
#define RD_FM(OP, D, X, Y, J) \
    OP " %" #D ", %" #X ", %" #Y " row_newbcast:" #J " row_mask:0xf bank_mask:0xf\n\t"
#define RD_FMN(OP, D, X, Y, J) \
    OP " %" #D ", %" #X ", -%" #Y " row_newbcast:" #J " row_mask:0xf bank_mask:0xf\n\t"
#define RD_F64 "v_fmac_f64_dpp"
#define RD_F32 "v_fmac_f32_dpp"
#define RD_ASM2(T, BODY, ...)                                      \
    do {                                                           \
        if constexpr (sizeof(T) == 8) __asm__ volatile(BODY(RD_F64) __VA_ARGS__); \
        else __asm__ volatile(BODY(RD_F32) __VA_ARGS__);           \
    } while (0)

/* sum_j e[j] * b(lane j), accumulated from +0 in j order (16 columns) */
#define RD_MV_BODY(OP)                                                                            \
    "s_nop 1\n\t"                                                                                 \
    RD_FM(OP, 0, 1, 2, 0) RD_FM(OP, 0, 1, 3, 1) RD_FM(OP, 0, 1, 4, 2) RD_FM(OP, 0, 1, 5, 3)       \
    RD_FM(OP, 0, 1, 6, 4) RD_FM(OP, 0, 1, 7, 5) RD_FM(OP, 0, 1, 8, 6) RD_FM(OP, 0, 1, 9, 7)       \
    RD_FM(OP, 0, 1, 10, 8) RD_FM(OP, 0, 1, 11, 9) RD_FM(OP, 0, 1, 12, 10) RD_FM(OP, 0, 1, 13, 11) \
    RD_FM(OP, 0, 1, 14, 12) RD_FM(OP, 0, 1, 15, 13) RD_FM(OP, 0, 1, 16, 14)                      \
    RD_FM(OP, 0, 1, 17, 15) "s_nop 1"
template <typename T>
__device__ __forceinline__ T fused_mv16(const T (&e)[16], T b) {
    T acc = T(0);
    RD_ASM2(T, RD_MV_BODY,
            : "+v"(acc)
            : "v"(b), "v"(e[0]), "v"(e[1]), "v"(e[2]), "v"(e[3]), "v"(e[4]), "v"(e[5]), "v"(e[6]),
              "v"(e[7]), "v"(e[8]), "v"(e[9]), "v"(e[10]), "v"(e[11]), "v"(e[12]), "v"(e[13]),
              "v"(e[14]), "v"(e[15]));
    return acc;
}
#undef RD_MV_BODY
#define RD_MV8_BODY(OP)                                                                           \
    "s_nop 1\n\t"                                                                                 \
    RD_FM(OP, 0, 1, 2, 0) RD_FM(OP, 0, 1, 3, 1) RD_FM(OP, 0, 1, 4, 2) RD_FM(OP, 0, 1, 5, 3)       \
    RD_FM(OP, 0, 1, 6, 4) RD_FM(OP, 0, 1, 7, 5) RD_FM(OP, 0, 1, 8, 6) RD_FM(OP, 0, 1, 9, 7)       \
    "s_nop 1"
/* the same product for the 8-column engine (m == 8) */
template <typename T>
__device__ __forceinline__ T fused_mv8(const T (&e)[8], T b) {
    T acc = T(0);
    RD_ASM2(T, RD_MV8_BODY,
            : "+v"(acc)
            : "v"(b), "v"(e[0]), "v"(e[1]), "v"(e[2]), "v"(e[3]), "v"(e[4]), "v"(e[5]), "v"(e[6]),
              "v"(e[7]));
    return acc;
}
#undef RD_MV8_BODY

/* Complex product, per column j in order:
 *   sr += bi_j * (-ei[j]);  sr += br_j * er[j];
 *   si += br_j * ei[j];     si += bi_j * er[j];   (from sr = si = +0) */
#define RD_CMV(OP, J, R, I) \
    RD_FMN(OP, 0, 3, I, J) RD_FM(OP, 0, 2, R, J) RD_FM(OP, 1, 2, I, J) RD_FM(OP, 1, 3, R, J)
#define RD_CMV_BODY(OP)                                                                           \
    "s_nop 1\n\t"                                                                                 \
    RD_CMV(OP, 0, 4, 20) RD_CMV(OP, 1, 5, 21) RD_CMV(OP, 2, 6, 22) RD_CMV(OP, 3, 7, 23)           \
    RD_CMV(OP, 4, 8, 24) RD_CMV(OP, 5, 9, 25) RD_CMV(OP, 6, 10, 26) RD_CMV(OP, 7, 11, 27)         \
    RD_CMV(OP, 8, 12, 28) RD_CMV(OP, 9, 13, 29) RD_CMV(OP, 10, 14, 30) RD_CMV(OP, 11, 15, 31)     \
    RD_CMV(OP, 12, 16, 32) RD_CMV(OP, 13, 17, 33) RD_CMV(OP, 14, 18, 34) RD_CMV(OP, 15, 19, 35)   \
    "s_nop 1"
template <typename T>
__device__ __forceinline__ void fused_cmv16(const T (&er)[16], const T (&ei)[16], T br, T bi, T& sr_out,
                                            T& si_out) {
    T sr = T(0), si = T(0);
    RD_ASM2(T, RD_CMV_BODY,
            : "+v"(sr), "+v"(si)
            : "v"(br), "v"(bi), "v"(er[0]), "v"(er[1]), "v"(er[2]), "v"(er[3]), "v"(er[4]),
              "v"(er[5]), "v"(er[6]), "v"(er[7]), "v"(er[8]), "v"(er[9]), "v"(er[10]), "v"(er[11]),
              "v"(er[12]), "v"(er[13]), "v"(er[14]), "v"(er[15]), "v"(ei[0]), "v"(ei[1]),
              "v"(ei[2]), "v"(ei[3]), "v"(ei[4]), "v"(ei[5]), "v"(ei[6]), "v"(ei[7]), "v"(ei[8]),
              "v"(ei[9]), "v"(ei[10]), "v"(ei[11]), "v"(ei[12]), "v"(ei[13]), "v"(ei[14]),
              "v"(ei[15]));
    sr_out = sr;
    si_out = si;
}
#undef RD_CMV_BODY
#define RD_CMV8_BODY(OP)                                                                          \
    "s_nop 1\n\t"                                                                                 \
    RD_CMV(OP, 0, 4, 12) RD_CMV(OP, 1, 5, 13) RD_CMV(OP, 2, 6, 14) RD_CMV(OP, 3, 7, 15)           \
    RD_CMV(OP, 4, 8, 16) RD_CMV(OP, 5, 9, 17) RD_CMV(OP, 6, 10, 18) RD_CMV(OP, 7, 11, 19)         \
    "s_nop 1"
/* the same product for the 8-column engine (m == 8) */
template <typename T>
__device__ __forceinline__ void fused_cmv8(const T (&er)[8], const T (&ei)[8], T br, T bi, T& sr_out,
                                           T& si_out) {
    T sr = T(0), si = T(0);
    RD_ASM2(T, RD_CMV8_BODY,
            : "+v"(sr), "+v"(si)
            : "v"(br), "v"(bi), "v"(er[0]), "v"(er[1]), "v"(er[2]), "v"(er[3]), "v"(er[4]),
              "v"(er[5]), "v"(er[6]), "v"(er[7]), "v"(ei[0]), "v"(ei[1]), "v"(ei[2]), "v"(ei[3]),
              "v"(ei[4]), "v"(ei[5]), "v"(ei[6]), "v"(ei[7]));
    sr_out = sr;
    si_out = si;
}
#undef RD_CMV8_BODY
#undef RD_CMV

/* Four columns J0..J0+3 of a model row (FP64):  lin += u(lane j) * k[j] and
 * loss += u(lane j) * g[j], column by column (lin first). */
#define RD_ROW(J, K, G) \
    RD_F64 " %0, %2, %" #K " row_newbcast:%" #J " row_mask:0xf bank_mask:0xf\n\t" \
    RD_F64 " %1, %2, %" #G " row_newbcast:%" #J " row_mask:0xf bank_mask:0xf\n\t"
template <int J0>
__device__ __forceinline__ void fused_row4(double u, const double* k, const double* g, double& lin,
                                           double& loss) {
    const double k0 = k[J0], k1 = k[J0 + 1], k2 = k[J0 + 2], k3 = k[J0 + 3];
    const double g0 = g[J0], g1 = g[J0 + 1], g2 = g[J0 + 2], g3 = g[J0 + 3];
    __asm__ volatile("s_nop 1\n\t"
                     RD_ROW(11, 3, 7) RD_ROW(12, 4, 8) RD_ROW(13, 5, 9) RD_ROW(14, 6, 10)
                     "s_nop 1"
                     : "+v"(lin), "+v"(loss)
                     : "v"(u), "v"(k0), "v"(k1), "v"(k2), "v"(k3), "v"(g0), "v"(g1), "v"(g2),
                       "v"(g3), "n"(J0), "n"(J0 + 1), "n"(J0 + 2), "n"(J0 + 3));
}
#undef RD_ROW
/* The same four columns for three arguments u1, u2, u3 at once (the three
 * stages of a Newton iteration): each k[j], g[j] is read from LDS once, and
 * each of the six sums receives its products column by column as above. */
#define RD_ROW3(J, K, G)                                                                    \
    RD_F64 " %0, %6, %" #K " row_newbcast:%" #J " row_mask:0xf bank_mask:0xf\n\t"          \
    RD_F64 " %1, %6, %" #G " row_newbcast:%" #J " row_mask:0xf bank_mask:0xf\n\t"          \
    RD_F64 " %2, %7, %" #K " row_newbcast:%" #J " row_mask:0xf bank_mask:0xf\n\t"          \
    RD_F64 " %3, %7, %" #G " row_newbcast:%" #J " row_mask:0xf bank_mask:0xf\n\t"          \
    RD_F64 " %4, %8, %" #K " row_newbcast:%" #J " row_mask:0xf bank_mask:0xf\n\t"          \
    RD_F64 " %5, %8, %" #G " row_newbcast:%" #J " row_mask:0xf bank_mask:0xf\n\t"
template <int J0>
__device__ __forceinline__ void fused_row4x3(double u1, double u2, double u3, const double* k,
                                             const double* g, double (&lin)[3], double (&loss)[3]) {
    const double k0 = k[J0], k1 = k[J0 + 1], k2 = k[J0 + 2], k3 = k[J0 + 3];
    const double g0 = g[J0], g1 = g[J0 + 1], g2 = g[J0 + 2], g3 = g[J0 + 3];
    __asm__ volatile("s_nop 1\n\t"
                     RD_ROW3(17, 9, 13) RD_ROW3(18, 10, 14) RD_ROW3(19, 11, 15) RD_ROW3(20, 12, 16)
                     "s_nop 1"
                     : "+v"(lin[0]), "+v"(loss[0]), "+v"(lin[1]), "+v"(loss[1]), "+v"(lin[2]),
                       "+v"(loss[2])
                     : "v"(u1), "v"(u2), "v"(u3), "v"(k0), "v"(k1), "v"(k2), "v"(k3), "v"(g0),
                       "v"(g1), "v"(g2), "v"(g3), "n"(J0), "n"(J0 + 1), "n"(J0 + 2), "n"(J0 + 3));
}
#undef RD_ROW3
#define RD_ROWK(J, K) RD_F64 " %0, %1, %" #K " row_newbcast:%" #J " row_mask:0xf bank_mask:0xf\n\t"
template <int J0>
__device__ __forceinline__ void fused_row4(double u, const double* k, double& lin) {
    const double k0 = k[J0], k1 = k[J0 + 1], k2 = k[J0 + 2], k3 = k[J0 + 3];
    __asm__ volatile("s_nop 1\n\t"
                     RD_ROWK(6, 2) RD_ROWK(7, 3) RD_ROWK(8, 4) RD_ROWK(9, 5)
                     "s_nop 1"
                     : "+v"(lin)
                     : "v"(u), "v"(k0), "v"(k1), "v"(k2), "v"(k3), "n"(J0), "n"(J0 + 1),
                       "n"(J0 + 2), "n"(J0 + 3));
}
#undef RD_ROWK

/* Gauss-Jordan elimination step with pivot lane KK (real):
 *   a[j] += a_j(lane KK) * (-f)  for every column j != KK
 * (column KK is overwritten by the caller afterwards).  One body per pivot
 * column, generated: each lists the fifteen other columns in order. */
#define RD_GJR(OP, J) OP " %" #J ", %" #J ", -%16 row_newbcast:%17 row_mask:0xf bank_mask:0xf\n\t"
#define RD_GJR_S0(OP) "s_nop 1\n\t" RD_GJR(OP, 1) RD_GJR(OP, 2) RD_GJR(OP, 3) RD_GJR(OP, 4) RD_GJR(OP, 5) RD_GJR(OP, 6) RD_GJR(OP, 7) RD_GJR(OP, 8) RD_GJR(OP, 9) RD_GJR(OP, 10) RD_GJR(OP, 11) RD_GJR(OP, 12) RD_GJR(OP, 13) RD_GJR(OP, 14) RD_GJR(OP, 15) "s_nop 1"
#define RD_GJR_S1(OP) "s_nop 1\n\t" RD_GJR(OP, 0) RD_GJR(OP, 2) RD_GJR(OP, 3) RD_GJR(OP, 4) RD_GJR(OP, 5) RD_GJR(OP, 6) RD_GJR(OP, 7) RD_GJR(OP, 8) RD_GJR(OP, 9) RD_GJR(OP, 10) RD_GJR(OP, 11) RD_GJR(OP, 12) RD_GJR(OP, 13) RD_GJR(OP, 14) RD_GJR(OP, 15) "s_nop 1"
#define RD_GJR_S2(OP) "s_nop 1\n\t" RD_GJR(OP, 0) RD_GJR(OP, 1) RD_GJR(OP, 3) RD_GJR(OP, 4) RD_GJR(OP, 5) RD_GJR(OP, 6) RD_GJR(OP, 7) RD_GJR(OP, 8) RD_GJR(OP, 9) RD_GJR(OP, 10) RD_GJR(OP, 11) RD_GJR(OP, 12) RD_GJR(OP, 13) RD_GJR(OP, 14) RD_GJR(OP, 15) "s_nop 1"
#define RD_GJR_S3(OP) "s_nop 1\n\t" RD_GJR(OP, 0) RD_GJR(OP, 1) RD_GJR(OP, 2) RD_GJR(OP, 4) RD_GJR(OP, 5) RD_GJR(OP, 6) RD_GJR(OP, 7) RD_GJR(OP, 8) RD_GJR(OP, 9) RD_GJR(OP, 10) RD_GJR(OP, 11) RD_GJR(OP, 12) RD_GJR(OP, 13) RD_GJR(OP, 14) RD_GJR(OP, 15) "s_nop 1"
#define RD_GJR_S4(OP) "s_nop 1\n\t" RD_GJR(OP, 0) RD_GJR(OP, 1) RD_GJR(OP, 2) RD_GJR(OP, 3) RD_GJR(OP, 5) RD_GJR(OP, 6) RD_GJR(OP, 7) RD_GJR(OP, 8) RD_GJR(OP, 9) RD_GJR(OP, 10) RD_GJR(OP, 11) RD_GJR(OP, 12) RD_GJR(OP, 13) RD_GJR(OP, 14) RD_GJR(OP, 15) "s_nop 1"
#define RD_GJR_S5(OP) "s_nop 1\n\t" RD_GJR(OP, 0) RD_GJR(OP, 1) RD_GJR(OP, 2) RD_GJR(OP, 3) RD_GJR(OP, 4) RD_GJR(OP, 6) RD_GJR(OP, 7) RD_GJR(OP, 8) RD_GJR(OP, 9) RD_GJR(OP, 10) RD_GJR(OP, 11) RD_GJR(OP, 12) RD_GJR(OP, 13) RD_GJR(OP, 14) RD_GJR(OP, 15) "s_nop 1"
#define RD_GJR_S6(OP) "s_nop 1\n\t" RD_GJR(OP, 0) RD_GJR(OP, 1) RD_GJR(OP, 2) RD_GJR(OP, 3) RD_GJR(OP, 4) RD_GJR(OP, 5) RD_GJR(OP, 7) RD_GJR(OP, 8) RD_GJR(OP, 9) RD_GJR(OP, 10) RD_GJR(OP, 11) RD_GJR(OP, 12) RD_GJR(OP, 13) RD_GJR(OP, 14) RD_GJR(OP, 15) "s_nop 1"
#define RD_GJR_S7(OP) "s_nop 1\n\t" RD_GJR(OP, 0) RD_GJR(OP, 1) RD_GJR(OP, 2) RD_GJR(OP, 3) RD_GJR(OP, 4) RD_GJR(OP, 5) RD_GJR(OP, 6) RD_GJR(OP, 8) RD_GJR(OP, 9) RD_GJR(OP, 10) RD_GJR(OP, 11) RD_GJR(OP, 12) RD_GJR(OP, 13) RD_GJR(OP, 14) RD_GJR(OP, 15) "s_nop 1"
#define RD_GJR_S8(OP) "s_nop 1\n\t" RD_GJR(OP, 0) RD_GJR(OP, 1) RD_GJR(OP, 2) RD_GJR(OP, 3) RD_GJR(OP, 4) RD_GJR(OP, 5) RD_GJR(OP, 6) RD_GJR(OP, 7) RD_GJR(OP, 9) RD_GJR(OP, 10) RD_GJR(OP, 11) RD_GJR(OP, 12) RD_GJR(OP, 13) RD_GJR(OP, 14) RD_GJR(OP, 15) "s_nop 1"
#define RD_GJR_S9(OP) "s_nop 1\n\t" RD_GJR(OP, 0) RD_GJR(OP, 1) RD_GJR(OP, 2) RD_GJR(OP, 3) RD_GJR(OP, 4) RD_GJR(OP, 5) RD_GJR(OP, 6) RD_GJR(OP, 7) RD_GJR(OP, 8) RD_GJR(OP, 10) RD_GJR(OP, 11) RD_GJR(OP, 12) RD_GJR(OP, 13) RD_GJR(OP, 14) RD_GJR(OP, 15) "s_nop 1"
#define RD_GJR_S10(OP) "s_nop 1\n\t" RD_GJR(OP, 0) RD_GJR(OP, 1) RD_GJR(OP, 2) RD_GJR(OP, 3) RD_GJR(OP, 4) RD_GJR(OP, 5) RD_GJR(OP, 6) RD_GJR(OP, 7) RD_GJR(OP, 8) RD_GJR(OP, 9) RD_GJR(OP, 11) RD_GJR(OP, 12) RD_GJR(OP, 13) RD_GJR(OP, 14) RD_GJR(OP, 15) "s_nop 1"
#define RD_GJR_S11(OP) "s_nop 1\n\t" RD_GJR(OP, 0) RD_GJR(OP, 1) RD_GJR(OP, 2) RD_GJR(OP, 3) RD_GJR(OP, 4) RD_GJR(OP, 5) RD_GJR(OP, 6) RD_GJR(OP, 7) RD_GJR(OP, 8) RD_GJR(OP, 9) RD_GJR(OP, 10) RD_GJR(OP, 12) RD_GJR(OP, 13) RD_GJR(OP, 14) RD_GJR(OP, 15) "s_nop 1"
#define RD_GJR_S12(OP) "s_nop 1\n\t" RD_GJR(OP, 0) RD_GJR(OP, 1) RD_GJR(OP, 2) RD_GJR(OP, 3) RD_GJR(OP, 4) RD_GJR(OP, 5) RD_GJR(OP, 6) RD_GJR(OP, 7) RD_GJR(OP, 8) RD_GJR(OP, 9) RD_GJR(OP, 10) RD_GJR(OP, 11) RD_GJR(OP, 13) RD_GJR(OP, 14) RD_GJR(OP, 15) "s_nop 1"
#define RD_GJR_S13(OP) "s_nop 1\n\t" RD_GJR(OP, 0) RD_GJR(OP, 1) RD_GJR(OP, 2) RD_GJR(OP, 3) RD_GJR(OP, 4) RD_GJR(OP, 5) RD_GJR(OP, 6) RD_GJR(OP, 7) RD_GJR(OP, 8) RD_GJR(OP, 9) RD_GJR(OP, 10) RD_GJR(OP, 11) RD_GJR(OP, 12) RD_GJR(OP, 14) RD_GJR(OP, 15) "s_nop 1"
#define RD_GJR_S14(OP) "s_nop 1\n\t" RD_GJR(OP, 0) RD_GJR(OP, 1) RD_GJR(OP, 2) RD_GJR(OP, 3) RD_GJR(OP, 4) RD_GJR(OP, 5) RD_GJR(OP, 6) RD_GJR(OP, 7) RD_GJR(OP, 8) RD_GJR(OP, 9) RD_GJR(OP, 10) RD_GJR(OP, 11) RD_GJR(OP, 12) RD_GJR(OP, 13) RD_GJR(OP, 15) "s_nop 1"
#define RD_GJR_S15(OP) "s_nop 1\n\t" RD_GJR(OP, 0) RD_GJR(OP, 1) RD_GJR(OP, 2) RD_GJR(OP, 3) RD_GJR(OP, 4) RD_GJR(OP, 5) RD_GJR(OP, 6) RD_GJR(OP, 7) RD_GJR(OP, 8) RD_GJR(OP, 9) RD_GJR(OP, 10) RD_GJR(OP, 11) RD_GJR(OP, 12) RD_GJR(OP, 13) RD_GJR(OP, 14) "s_nop 1"
template <int KK, typename T>
__device__ __forceinline__ void fused_gj_real_k(T (&a)[16], T f) {
#define OPERANDS                                                                                  \
    : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5]), "+v"(a[6]),        \
      "+v"(a[7]), "+v"(a[8]), "+v"(a[9]), "+v"(a[10]), "+v"(a[11]), "+v"(a[12]), "+v"(a[13]),     \
      "+v"(a[14]), "+v"(a[15])                                                                    \
    : "v"(f), "n"(KK)
    if constexpr (KK == 0) RD_ASM2(T, RD_GJR_S0, OPERANDS);
    else if constexpr (KK == 1) RD_ASM2(T, RD_GJR_S1, OPERANDS);
    else if constexpr (KK == 2) RD_ASM2(T, RD_GJR_S2, OPERANDS);
    else if constexpr (KK == 3) RD_ASM2(T, RD_GJR_S3, OPERANDS);
    else if constexpr (KK == 4) RD_ASM2(T, RD_GJR_S4, OPERANDS);
    else if constexpr (KK == 5) RD_ASM2(T, RD_GJR_S5, OPERANDS);
    else if constexpr (KK == 6) RD_ASM2(T, RD_GJR_S6, OPERANDS);
    else if constexpr (KK == 7) RD_ASM2(T, RD_GJR_S7, OPERANDS);
    else if constexpr (KK == 8) RD_ASM2(T, RD_GJR_S8, OPERANDS);
    else if constexpr (KK == 9) RD_ASM2(T, RD_GJR_S9, OPERANDS);
    else if constexpr (KK == 10) RD_ASM2(T, RD_GJR_S10, OPERANDS);
    else if constexpr (KK == 11) RD_ASM2(T, RD_GJR_S11, OPERANDS);
    else if constexpr (KK == 12) RD_ASM2(T, RD_GJR_S12, OPERANDS);
    else if constexpr (KK == 13) RD_ASM2(T, RD_GJR_S13, OPERANDS);
    else if constexpr (KK == 14) RD_ASM2(T, RD_GJR_S14, OPERANDS);
    else if constexpr (KK == 15) RD_ASM2(T, RD_GJR_S15, OPERANDS);
#undef OPERANDS
}
#undef RD_GJR_S0
#undef RD_GJR_S1
#undef RD_GJR_S2
#undef RD_GJR_S3
#undef RD_GJR_S4
#undef RD_GJR_S5
#undef RD_GJR_S6
#undef RD_GJR_S7
#undef RD_GJR_S8
#undef RD_GJR_S9
#undef RD_GJR_S10
#undef RD_GJR_S11
#undef RD_GJR_S12
#undef RD_GJR_S13
#undef RD_GJR_S14
#undef RD_GJR_S15
#undef RD_GJR

/* The same step for the 8-column engine (m <= 8). */
#define RD_GJR8(OP, J) OP " %" #J ", %" #J ", -%8 row_newbcast:%9 row_mask:0xf bank_mask:0xf\n\t"
#define RD_GJR8_S0(OP) "s_nop 1\n\t" RD_GJR8(OP, 1) RD_GJR8(OP, 2) RD_GJR8(OP, 3) RD_GJR8(OP, 4) RD_GJR8(OP, 5) RD_GJR8(OP, 6) RD_GJR8(OP, 7) "s_nop 1"
#define RD_GJR8_S1(OP) "s_nop 1\n\t" RD_GJR8(OP, 0) RD_GJR8(OP, 2) RD_GJR8(OP, 3) RD_GJR8(OP, 4) RD_GJR8(OP, 5) RD_GJR8(OP, 6) RD_GJR8(OP, 7) "s_nop 1"
#define RD_GJR8_S2(OP) "s_nop 1\n\t" RD_GJR8(OP, 0) RD_GJR8(OP, 1) RD_GJR8(OP, 3) RD_GJR8(OP, 4) RD_GJR8(OP, 5) RD_GJR8(OP, 6) RD_GJR8(OP, 7) "s_nop 1"
#define RD_GJR8_S3(OP) "s_nop 1\n\t" RD_GJR8(OP, 0) RD_GJR8(OP, 1) RD_GJR8(OP, 2) RD_GJR8(OP, 4) RD_GJR8(OP, 5) RD_GJR8(OP, 6) RD_GJR8(OP, 7) "s_nop 1"
#define RD_GJR8_S4(OP) "s_nop 1\n\t" RD_GJR8(OP, 0) RD_GJR8(OP, 1) RD_GJR8(OP, 2) RD_GJR8(OP, 3) RD_GJR8(OP, 5) RD_GJR8(OP, 6) RD_GJR8(OP, 7) "s_nop 1"
#define RD_GJR8_S5(OP) "s_nop 1\n\t" RD_GJR8(OP, 0) RD_GJR8(OP, 1) RD_GJR8(OP, 2) RD_GJR8(OP, 3) RD_GJR8(OP, 4) RD_GJR8(OP, 6) RD_GJR8(OP, 7) "s_nop 1"
#define RD_GJR8_S6(OP) "s_nop 1\n\t" RD_GJR8(OP, 0) RD_GJR8(OP, 1) RD_GJR8(OP, 2) RD_GJR8(OP, 3) RD_GJR8(OP, 4) RD_GJR8(OP, 5) RD_GJR8(OP, 7) "s_nop 1"
#define RD_GJR8_S7(OP) "s_nop 1\n\t" RD_GJR8(OP, 0) RD_GJR8(OP, 1) RD_GJR8(OP, 2) RD_GJR8(OP, 3) RD_GJR8(OP, 4) RD_GJR8(OP, 5) RD_GJR8(OP, 6) "s_nop 1"
template <int KK, typename T>
__device__ __forceinline__ void fused_gj_real8_k(T (&a)[8], T f) {
#define OPERANDS                                                                                  \
    : "+v"(a[0]), "+v"(a[1]), "+v"(a[2]), "+v"(a[3]), "+v"(a[4]), "+v"(a[5]), "+v"(a[6]),        \
      "+v"(a[7])                                                                                  \
    : "v"(f), "n"(KK)
    if constexpr (KK == 0) RD_ASM2(T, RD_GJR8_S0, OPERANDS);
    else if constexpr (KK == 1) RD_ASM2(T, RD_GJR8_S1, OPERANDS);
    else if constexpr (KK == 2) RD_ASM2(T, RD_GJR8_S2, OPERANDS);
    else if constexpr (KK == 3) RD_ASM2(T, RD_GJR8_S3, OPERANDS);
    else if constexpr (KK == 4) RD_ASM2(T, RD_GJR8_S4, OPERANDS);
    else if constexpr (KK == 5) RD_ASM2(T, RD_GJR8_S5, OPERANDS);
    else if constexpr (KK == 6) RD_ASM2(T, RD_GJR8_S6, OPERANDS);
    else if constexpr (KK == 7) RD_ASM2(T, RD_GJR8_S7, OPERANDS);
#undef OPERANDS
}
#undef RD_GJR8_S0
#undef RD_GJR8_S1
#undef RD_GJR8_S2
#undef RD_GJR8_S3
#undef RD_GJR8_S4
#undef RD_GJR8_S5
#undef RD_GJR8_S6
#undef RD_GJR8_S7
#undef RD_GJR8

/* Gauss-Jordan elimination step with pivot lane KK (complex), for every
 * column j != KK, with (ur, ui) the pivot row's entry of column j:
 *   ar[j] = (ar[j] + ui fi) - ur fr,   ai[j] = (ai[j] - ur fi) - ui fr.
 * Issued in four sweeps over the columns (ar += ui fi; ai -= ur fi;
 * ar -= ur fr; ai -= ui fr), so that a register written in one sweep is read
 * through DPP fifteen or more instructions later.  The sweeps read the pivot
 * lane's entries after the pivot lane has applied the earlier sweeps to
 * them, which add x * (+-0) there (fr = fi = 0 in the pivot lane): the
 * values read equal those of the plain order (a zero may change its sign).
 * Column KK is overwritten by the caller afterwards; one body per pivot
 * column, generated. */
#define RD_GJA(OP, R, I) OP " %" #R ", %" #I ", %33 row_newbcast:%34 row_mask:0xf bank_mask:0xf\n\t"
#define RD_GJB(OP, R, I) OP " %" #I ", %" #R ", -%33 row_newbcast:%34 row_mask:0xf bank_mask:0xf\n\t"
#define RD_GJC(OP, R, I) OP " %" #R ", %" #R ", -%32 row_newbcast:%34 row_mask:0xf bank_mask:0xf\n\t"
#define RD_GJD(OP, R, I) OP " %" #I ", %" #I ", -%32 row_newbcast:%34 row_mask:0xf bank_mask:0xf\n\t"
#define RD_GJC_S0(OP) "s_nop 1\n\t" RD_GJA(OP, 1, 17) RD_GJA(OP, 2, 18) RD_GJA(OP, 3, 19) RD_GJA(OP, 4, 20) RD_GJA(OP, 5, 21) RD_GJA(OP, 6, 22) RD_GJA(OP, 7, 23) RD_GJA(OP, 8, 24) RD_GJA(OP, 9, 25) RD_GJA(OP, 10, 26) RD_GJA(OP, 11, 27) RD_GJA(OP, 12, 28) RD_GJA(OP, 13, 29) RD_GJA(OP, 14, 30) RD_GJA(OP, 15, 31) RD_GJB(OP, 1, 17) RD_GJB(OP, 2, 18) RD_GJB(OP, 3, 19) RD_GJB(OP, 4, 20) RD_GJB(OP, 5, 21) RD_GJB(OP, 6, 22) RD_GJB(OP, 7, 23) RD_GJB(OP, 8, 24) RD_GJB(OP, 9, 25) RD_GJB(OP, 10, 26) RD_GJB(OP, 11, 27) RD_GJB(OP, 12, 28) RD_GJB(OP, 13, 29) RD_GJB(OP, 14, 30) RD_GJB(OP, 15, 31) RD_GJC(OP, 1, 17) RD_GJC(OP, 2, 18) RD_GJC(OP, 3, 19) RD_GJC(OP, 4, 20) RD_GJC(OP, 5, 21) RD_GJC(OP, 6, 22) RD_GJC(OP, 7, 23) RD_GJC(OP, 8, 24) RD_GJC(OP, 9, 25) RD_GJC(OP, 10, 26) RD_GJC(OP, 11, 27) RD_GJC(OP, 12, 28) RD_GJC(OP, 13, 29) RD_GJC(OP, 14, 30) RD_GJC(OP, 15, 31) RD_GJD(OP, 1, 17) RD_GJD(OP, 2, 18) RD_GJD(OP, 3, 19) RD_GJD(OP, 4, 20) RD_GJD(OP, 5, 21) RD_GJD(OP, 6, 22) RD_GJD(OP, 7, 23) RD_GJD(OP, 8, 24) RD_GJD(OP, 9, 25) RD_GJD(OP, 10, 26) RD_GJD(OP, 11, 27) RD_GJD(OP, 12, 28) RD_GJD(OP, 13, 29) RD_GJD(OP, 14, 30) RD_GJD(OP, 15, 31) "s_nop 1"
#define RD_GJC_S1(OP) "s_nop 1\n\t" RD_GJA(OP, 0, 16) RD_GJA(OP, 2, 18) RD_GJA(OP, 3, 19) RD_GJA(OP, 4, 20) RD_GJA(OP, 5, 21) RD_GJA(OP, 6, 22) RD_GJA(OP, 7, 23) RD_GJA(OP, 8, 24) RD_GJA(OP, 9, 25) RD_GJA(OP, 10, 26) RD_GJA(OP, 11, 27) RD_GJA(OP, 12, 28) RD_GJA(OP, 13, 29) RD_GJA(OP, 14, 30) RD_GJA(OP, 15, 31) RD_GJB(OP, 0, 16) RD_GJB(OP, 2, 18) RD_GJB(OP, 3, 19) RD_GJB(OP, 4, 20) RD_GJB(OP, 5, 21) RD_GJB(OP, 6, 22) RD_GJB(OP, 7, 23) RD_GJB(OP, 8, 24) RD_GJB(OP, 9, 25) RD_GJB(OP, 10, 26) RD_GJB(OP, 11, 27) RD_GJB(OP, 12, 28) RD_GJB(OP, 13, 29) RD_GJB(OP, 14, 30) RD_GJB(OP, 15, 31) RD_GJC(OP, 0, 16) RD_GJC(OP, 2, 18) RD_GJC(OP, 3, 19) RD_GJC(OP, 4, 20) RD_GJC(OP, 5, 21) RD_GJC(OP, 6, 22) RD_GJC(OP, 7, 23) RD_GJC(OP, 8, 24) RD_GJC(OP, 9, 25) RD_GJC(OP, 10, 26) RD_GJC(OP, 11, 27) RD_GJC(OP, 12, 28) RD_GJC(OP, 13, 29) RD_GJC(OP, 14, 30) RD_GJC(OP, 15, 31) RD_GJD(OP, 0, 16) RD_GJD(OP, 2, 18) RD_GJD(OP, 3, 19) RD_GJD(OP, 4, 20) RD_GJD(OP, 5, 21) RD_GJD(OP, 6, 22) RD_GJD(OP, 7, 23) RD_GJD(OP, 8, 24) RD_GJD(OP, 9, 25) RD_GJD(OP, 10, 26) RD_GJD(OP, 11, 27) RD_GJD(OP, 12, 28) RD_GJD(OP, 13, 29) RD_GJD(OP, 14, 30) RD_GJD(OP, 15, 31) "s_nop 1"
#define RD_GJC_S2(OP) "s_nop 1\n\t" RD_GJA(OP, 0, 16) RD_GJA(OP, 1, 17) RD_GJA(OP, 3, 19) RD_GJA(OP, 4, 20) RD_GJA(OP, 5, 21) RD_GJA(OP, 6, 22) RD_GJA(OP, 7, 23) RD_GJA(OP, 8, 24) RD_GJA(OP, 9, 25) RD_GJA(OP, 10, 26) RD_GJA(OP, 11, 27) RD_GJA(OP, 12, 28) RD_GJA(OP, 13, 29) RD_GJA(OP, 14, 30) RD_GJA(OP, 15, 31) RD_GJB(OP, 0, 16) RD_GJB(OP, 1, 17) RD_GJB(OP, 3, 19) RD_GJB(OP, 4, 20) RD_GJB(OP, 5, 21) RD_GJB(OP, 6, 22) RD_GJB(OP, 7, 23) RD_GJB(OP, 8, 24) RD_GJB(OP, 9, 25) RD_GJB(OP, 10, 26) RD_GJB(OP, 11, 27) RD_GJB(OP, 12, 28) RD_GJB(OP, 13, 29) RD_GJB(OP, 14, 30) RD_GJB(OP, 15, 31) RD_GJC(OP, 0, 16) RD_GJC(OP, 1, 17) RD_GJC(OP, 3, 19) RD_GJC(OP, 4, 20) RD_GJC(OP, 5, 21) RD_GJC(OP, 6, 22) RD_GJC(OP, 7, 23) RD_GJC(OP, 8, 24) RD_GJC(OP, 9, 25) RD_GJC(OP, 10, 26) RD_GJC(OP, 11, 27) RD_GJC(OP, 12, 28) RD_GJC(OP, 13, 29) RD_GJC(OP, 14, 30) RD_GJC(OP, 15, 31) RD_GJD(OP, 0, 16) RD_GJD(OP, 1, 17) RD_GJD(OP, 3, 19) RD_GJD(OP, 4, 20) RD_GJD(OP, 5, 21) RD_GJD(OP, 6, 22) RD_GJD(OP, 7, 23) RD_GJD(OP, 8, 24) RD_GJD(OP, 9, 25) RD_GJD(OP, 10, 26) RD_GJD(OP, 11, 27) RD_GJD(OP, 12, 28) RD_GJD(OP, 13, 29) RD_GJD(OP, 14, 30) RD_GJD(OP, 15, 31) "s_nop 1"
#define RD_GJC_S3(OP) "s_nop 1\n\t" RD_GJA(OP, 0, 16) RD_GJA(OP, 1, 17) RD_GJA(OP, 2, 18) RD_GJA(OP, 4, 20) RD_GJA(OP, 5, 21) RD_GJA(OP, 6, 22) RD_GJA(OP, 7, 23) RD_GJA(OP, 8, 24) RD_GJA(OP, 9, 25) RD_GJA(OP, 10, 26) RD_GJA(OP, 11, 27) RD_GJA(OP, 12, 28) RD_GJA(OP, 13, 29) RD_GJA(OP, 14, 30) RD_GJA(OP, 15, 31) RD_GJB(OP, 0, 16) RD_GJB(OP, 1, 17) RD_GJB(OP, 2, 18) RD_GJB(OP, 4, 20) RD_GJB(OP, 5, 21) RD_GJB(OP, 6, 22) RD_GJB(OP, 7, 23) RD_GJB(OP, 8, 24) RD_GJB(OP, 9, 25) RD_GJB(OP, 10, 26) RD_GJB(OP, 11, 27) RD_GJB(OP, 12, 28) RD_GJB(OP, 13, 29) RD_GJB(OP, 14, 30) RD_GJB(OP, 15, 31) RD_GJC(OP, 0, 16) RD_GJC(OP, 1, 17) RD_GJC(OP, 2, 18) RD_GJC(OP, 4, 20) RD_GJC(OP, 5, 21) RD_GJC(OP, 6, 22) RD_GJC(OP, 7, 23) RD_GJC(OP, 8, 24) RD_GJC(OP, 9, 25) RD_GJC(OP, 10, 26) RD_GJC(OP, 11, 27) RD_GJC(OP, 12, 28) RD_GJC(OP, 13, 29) RD_GJC(OP, 14, 30) RD_GJC(OP, 15, 31) RD_GJD(OP, 0, 16) RD_GJD(OP, 1, 17) RD_GJD(OP, 2, 18) RD_GJD(OP, 4, 20) RD_GJD(OP, 5, 21) RD_GJD(OP, 6, 22) RD_GJD(OP, 7, 23) RD_GJD(OP, 8, 24) RD_GJD(OP, 9, 25) RD_GJD(OP, 10, 26) RD_GJD(OP, 11, 27) RD_GJD(OP, 12, 28) RD_GJD(OP, 13, 29) RD_GJD(OP, 14, 30) RD_GJD(OP, 15, 31) "s_nop 1"
#define RD_GJC_S4(OP) "s_nop 1\n\t" RD_GJA(OP, 0, 16) RD_GJA(OP, 1, 17) RD_GJA(OP, 2, 18) RD_GJA(OP, 3, 19) RD_GJA(OP, 5, 21) RD_GJA(OP, 6, 22) RD_GJA(OP, 7, 23) RD_GJA(OP, 8, 24) RD_GJA(OP, 9, 25) RD_GJA(OP, 10, 26) RD_GJA(OP, 11, 27) RD_GJA(OP, 12, 28) RD_GJA(OP, 13, 29) RD_GJA(OP, 14, 30) RD_GJA(OP, 15, 31) RD_GJB(OP, 0, 16) RD_GJB(OP, 1, 17) RD_GJB(OP, 2, 18) RD_GJB(OP, 3, 19) RD_GJB(OP, 5, 21) RD_GJB(OP, 6, 22) RD_GJB(OP, 7, 23) RD_GJB(OP, 8, 24) RD_GJB(OP, 9, 25) RD_GJB(OP, 10, 26) RD_GJB(OP, 11, 27) RD_GJB(OP, 12, 28) RD_GJB(OP, 13, 29) RD_GJB(OP, 14, 30) RD_GJB(OP, 15, 31) RD_GJC(OP, 0, 16) RD_GJC(OP, 1, 17) RD_GJC(OP, 2, 18) RD_GJC(OP, 3, 19) RD_GJC(OP, 5, 21) RD_GJC(OP, 6, 22) RD_GJC(OP, 7, 23) RD_GJC(OP, 8, 24) RD_GJC(OP, 9, 25) RD_GJC(OP, 10, 26) RD_GJC(OP, 11, 27) RD_GJC(OP, 12, 28) RD_GJC(OP, 13, 29) RD_GJC(OP, 14, 30) RD_GJC(OP, 15, 31) RD_GJD(OP, 0, 16) RD_GJD(OP, 1, 17) RD_GJD(OP, 2, 18) RD_GJD(OP, 3, 19) RD_GJD(OP, 5, 21) RD_GJD(OP, 6, 22) RD_GJD(OP, 7, 23) RD_GJD(OP, 8, 24) RD_GJD(OP, 9, 25) RD_GJD(OP, 10, 26) RD_GJD(OP, 11, 27) RD_GJD(OP, 12, 28) RD_GJD(OP, 13, 29) RD_GJD(OP, 14, 30) RD_GJD(OP, 15, 31) "s_nop 1"
#define RD_GJC_S5(OP) "s_nop 1\n\t" RD_GJA(OP, 0, 16) RD_GJA(OP, 1, 17) RD_GJA(OP, 2, 18) RD_GJA(OP, 3, 19) RD_GJA(OP, 4, 20) RD_GJA(OP, 6, 22) RD_GJA(OP, 7, 23) RD_GJA(OP, 8, 24) RD_GJA(OP, 9, 25) RD_GJA(OP, 10, 26) RD_GJA(OP, 11, 27) RD_GJA(OP, 12, 28) RD_GJA(OP, 13, 29) RD_GJA(OP, 14, 30) RD_GJA(OP, 15, 31) RD_GJB(OP, 0, 16) RD_GJB(OP, 1, 17) RD_GJB(OP, 2, 18) RD_GJB(OP, 3, 19) RD_GJB(OP, 4, 20) RD_GJB(OP, 6, 22) RD_GJB(OP, 7, 23) RD_GJB(OP, 8, 24) RD_GJB(OP, 9, 25) RD_GJB(OP, 10, 26) RD_GJB(OP, 11, 27) RD_GJB(OP, 12, 28) RD_GJB(OP, 13, 29) RD_GJB(OP, 14, 30) RD_GJB(OP, 15, 31) RD_GJC(OP, 0, 16) RD_GJC(OP, 1, 17) RD_GJC(OP, 2, 18) RD_GJC(OP, 3, 19) RD_GJC(OP, 4, 20) RD_GJC(OP, 6, 22) RD_GJC(OP, 7, 23) RD_GJC(OP, 8, 24) RD_GJC(OP, 9, 25) RD_GJC(OP, 10, 26) RD_GJC(OP, 11, 27) RD_GJC(OP, 12, 28) RD_GJC(OP, 13, 29) RD_GJC(OP, 14, 30) RD_GJC(OP, 15, 31) RD_GJD(OP, 0, 16) RD_GJD(OP, 1, 17) RD_GJD(OP, 2, 18) RD_GJD(OP, 3, 19) RD_GJD(OP, 4, 20) RD_GJD(OP, 6, 22) RD_GJD(OP, 7, 23) RD_GJD(OP, 8, 24) RD_GJD(OP, 9, 25) RD_GJD(OP, 10, 26) RD_GJD(OP, 11, 27) RD_GJD(OP, 12, 28) RD_GJD(OP, 13, 29) RD_GJD(OP, 14, 30) RD_GJD(OP, 15, 31) "s_nop 1"
#define RD_GJC_S6(OP) "s_nop 1\n\t" RD_GJA(OP, 0, 16) RD_GJA(OP, 1, 17) RD_GJA(OP, 2, 18) RD_GJA(OP, 3, 19) RD_GJA(OP, 4, 20) RD_GJA(OP, 5, 21) RD_GJA(OP, 7, 23) RD_GJA(OP, 8, 24) RD_GJA(OP, 9, 25) RD_GJA(OP, 10, 26) RD_GJA(OP, 11, 27) RD_GJA(OP, 12, 28) RD_GJA(OP, 13, 29) RD_GJA(OP, 14, 30) RD_GJA(OP, 15, 31) RD_GJB(OP, 0, 16) RD_GJB(OP, 1, 17) RD_GJB(OP, 2, 18) RD_GJB(OP, 3, 19) RD_GJB(OP, 4, 20) RD_GJB(OP, 5, 21) RD_GJB(OP, 7, 23) RD_GJB(OP, 8, 24) RD_GJB(OP, 9, 25) RD_GJB(OP, 10, 26) RD_GJB(OP, 11, 27) RD_GJB(OP, 12, 28) RD_GJB(OP, 13, 29) RD_GJB(OP, 14, 30) RD_GJB(OP, 15, 31) RD_GJC(OP, 0, 16) RD_GJC(OP, 1, 17) RD_GJC(OP, 2, 18) RD_GJC(OP, 3, 19) RD_GJC(OP, 4, 20) RD_GJC(OP, 5, 21) RD_GJC(OP, 7, 23) RD_GJC(OP, 8, 24) RD_GJC(OP, 9, 25) RD_GJC(OP, 10, 26) RD_GJC(OP, 11, 27) RD_GJC(OP, 12, 28) RD_GJC(OP, 13, 29) RD_GJC(OP, 14, 30) RD_GJC(OP, 15, 31) RD_GJD(OP, 0, 16) RD_GJD(OP, 1, 17) RD_GJD(OP, 2, 18) RD_GJD(OP, 3, 19) RD_GJD(OP, 4, 20) RD_GJD(OP, 5, 21) RD_GJD(OP, 7, 23) RD_GJD(OP, 8, 24) RD_GJD(OP, 9, 25) RD_GJD(OP, 10, 26) RD_GJD(OP, 11, 27) RD_GJD(OP, 12, 28) RD_GJD(OP, 13, 29) RD_GJD(OP, 14, 30) RD_GJD(OP, 15, 31) "s_nop 1"
#define RD_GJC_S7(OP) "s_nop 1\n\t" RD_GJA(OP, 0, 16) RD_GJA(OP, 1, 17) RD_GJA(OP, 2, 18) RD_GJA(OP, 3, 19) RD_GJA(OP, 4, 20) RD_GJA(OP, 5, 21) RD_GJA(OP, 6, 22) RD_GJA(OP, 8, 24) RD_GJA(OP, 9, 25) RD_GJA(OP, 10, 26) RD_GJA(OP, 11, 27) RD_GJA(OP, 12, 28) RD_GJA(OP, 13, 29) RD_GJA(OP, 14, 30) RD_GJA(OP, 15, 31) RD_GJB(OP, 0, 16) RD_GJB(OP, 1, 17) RD_GJB(OP, 2, 18) RD_GJB(OP, 3, 19) RD_GJB(OP, 4, 20) RD_GJB(OP, 5, 21) RD_GJB(OP, 6, 22) RD_GJB(OP, 8, 24) RD_GJB(OP, 9, 25) RD_GJB(OP, 10, 26) RD_GJB(OP, 11, 27) RD_GJB(OP, 12, 28) RD_GJB(OP, 13, 29) RD_GJB(OP, 14, 30) RD_GJB(OP, 15, 31) RD_GJC(OP, 0, 16) RD_GJC(OP, 1, 17) RD_GJC(OP, 2, 18) RD_GJC(OP, 3, 19) RD_GJC(OP, 4, 20) RD_GJC(OP, 5, 21) RD_GJC(OP, 6, 22) RD_GJC(OP, 8, 24) RD_GJC(OP, 9, 25) RD_GJC(OP, 10, 26) RD_GJC(OP, 11, 27) RD_GJC(OP, 12, 28) RD_GJC(OP, 13, 29) RD_GJC(OP, 14, 30) RD_GJC(OP, 15, 31) RD_GJD(OP, 0, 16) RD_GJD(OP, 1, 17) RD_GJD(OP, 2, 18) RD_GJD(OP, 3, 19) RD_GJD(OP, 4, 20) RD_GJD(OP, 5, 21) RD_GJD(OP, 6, 22) RD_GJD(OP, 8, 24) RD_GJD(OP, 9, 25) RD_GJD(OP, 10, 26) RD_GJD(OP, 11, 27) RD_GJD(OP, 12, 28) RD_GJD(OP, 13, 29) RD_GJD(OP, 14, 30) RD_GJD(OP, 15, 31) "s_nop 1"
#define RD_GJC_S8(OP) "s_nop 1\n\t" RD_GJA(OP, 0, 16) RD_GJA(OP, 1, 17) RD_GJA(OP, 2, 18) RD_GJA(OP, 3, 19) RD_GJA(OP, 4, 20) RD_GJA(OP, 5, 21) RD_GJA(OP, 6, 22) RD_GJA(OP, 7, 23) RD_GJA(OP, 9, 25) RD_GJA(OP, 10, 26) RD_GJA(OP, 11, 27) RD_GJA(OP, 12, 28) RD_GJA(OP, 13, 29) RD_GJA(OP, 14, 30) RD_GJA(OP, 15, 31) RD_GJB(OP, 0, 16) RD_GJB(OP, 1, 17) RD_GJB(OP, 2, 18) RD_GJB(OP, 3, 19) RD_GJB(OP, 4, 20) RD_GJB(OP, 5, 21) RD_GJB(OP, 6, 22) RD_GJB(OP, 7, 23) RD_GJB(OP, 9, 25) RD_GJB(OP, 10, 26) RD_GJB(OP, 11, 27) RD_GJB(OP, 12, 28) RD_GJB(OP, 13, 29) RD_GJB(OP, 14, 30) RD_GJB(OP, 15, 31) RD_GJC(OP, 0, 16) RD_GJC(OP, 1, 17) RD_GJC(OP, 2, 18) RD_GJC(OP, 3, 19) RD_GJC(OP, 4, 20) RD_GJC(OP, 5, 21) RD_GJC(OP, 6, 22) RD_GJC(OP, 7, 23) RD_GJC(OP, 9, 25) RD_GJC(OP, 10, 26) RD_GJC(OP, 11, 27) RD_GJC(OP, 12, 28) RD_GJC(OP, 13, 29) RD_GJC(OP, 14, 30) RD_GJC(OP, 15, 31) RD_GJD(OP, 0, 16) RD_GJD(OP, 1, 17) RD_GJD(OP, 2, 18) RD_GJD(OP, 3, 19) RD_GJD(OP, 4, 20) RD_GJD(OP, 5, 21) RD_GJD(OP, 6, 22) RD_GJD(OP, 7, 23) RD_GJD(OP, 9, 25) RD_GJD(OP, 10, 26) RD_GJD(OP, 11, 27) RD_GJD(OP, 12, 28) RD_GJD(OP, 13, 29) RD_GJD(OP, 14, 30) RD_GJD(OP, 15, 31) "s_nop 1"
#define RD_GJC_S9(OP) "s_nop 1\n\t" RD_GJA(OP, 0, 16) RD_GJA(OP, 1, 17) RD_GJA(OP, 2, 18) RD_GJA(OP, 3, 19) RD_GJA(OP, 4, 20) RD_GJA(OP, 5, 21) RD_GJA(OP, 6, 22) RD_GJA(OP, 7, 23) RD_GJA(OP, 8, 24) RD_GJA(OP, 10, 26) RD_GJA(OP, 11, 27) RD_GJA(OP, 12, 28) RD_GJA(OP, 13, 29) RD_GJA(OP, 14, 30) RD_GJA(OP, 15, 31) RD_GJB(OP, 0, 16) RD_GJB(OP, 1, 17) RD_GJB(OP, 2, 18) RD_GJB(OP, 3, 19) RD_GJB(OP, 4, 20) RD_GJB(OP, 5, 21) RD_GJB(OP, 6, 22) RD_GJB(OP, 7, 23) RD_GJB(OP, 8, 24) RD_GJB(OP, 10, 26) RD_GJB(OP, 11, 27) RD_GJB(OP, 12, 28) RD_GJB(OP, 13, 29) RD_GJB(OP, 14, 30) RD_GJB(OP, 15, 31) RD_GJC(OP, 0, 16) RD_GJC(OP, 1, 17) RD_GJC(OP, 2, 18) RD_GJC(OP, 3, 19) RD_GJC(OP, 4, 20) RD_GJC(OP, 5, 21) RD_GJC(OP, 6, 22) RD_GJC(OP, 7, 23) RD_GJC(OP, 8, 24) RD_GJC(OP, 10, 26) RD_GJC(OP, 11, 27) RD_GJC(OP, 12, 28) RD_GJC(OP, 13, 29) RD_GJC(OP, 14, 30) RD_GJC(OP, 15, 31) RD_GJD(OP, 0, 16) RD_GJD(OP, 1, 17) RD_GJD(OP, 2, 18) RD_GJD(OP, 3, 19) RD_GJD(OP, 4, 20) RD_GJD(OP, 5, 21) RD_GJD(OP, 6, 22) RD_GJD(OP, 7, 23) RD_GJD(OP, 8, 24) RD_GJD(OP, 10, 26) RD_GJD(OP, 11, 27) RD_GJD(OP, 12, 28) RD_GJD(OP, 13, 29) RD_GJD(OP, 14, 30) RD_GJD(OP, 15, 31) "s_nop 1"
#define RD_GJC_S10(OP) "s_nop 1\n\t" RD_GJA(OP, 0, 16) RD_GJA(OP, 1, 17) RD_GJA(OP, 2, 18) RD_GJA(OP, 3, 19) RD_GJA(OP, 4, 20) RD_GJA(OP, 5, 21) RD_GJA(OP, 6, 22) RD_GJA(OP, 7, 23) RD_GJA(OP, 8, 24) RD_GJA(OP, 9, 25) RD_GJA(OP, 11, 27) RD_GJA(OP, 12, 28) RD_GJA(OP, 13, 29) RD_GJA(OP, 14, 30) RD_GJA(OP, 15, 31) RD_GJB(OP, 0, 16) RD_GJB(OP, 1, 17) RD_GJB(OP, 2, 18) RD_GJB(OP, 3, 19) RD_GJB(OP, 4, 20) RD_GJB(OP, 5, 21) RD_GJB(OP, 6, 22) RD_GJB(OP, 7, 23) RD_GJB(OP, 8, 24) RD_GJB(OP, 9, 25) RD_GJB(OP, 11, 27) RD_GJB(OP, 12, 28) RD_GJB(OP, 13, 29) RD_GJB(OP, 14, 30) RD_GJB(OP, 15, 31) RD_GJC(OP, 0, 16) RD_GJC(OP, 1, 17) RD_GJC(OP, 2, 18) RD_GJC(OP, 3, 19) RD_GJC(OP, 4, 20) RD_GJC(OP, 5, 21) RD_GJC(OP, 6, 22) RD_GJC(OP, 7, 23) RD_GJC(OP, 8, 24) RD_GJC(OP, 9, 25) RD_GJC(OP, 11, 27) RD_GJC(OP, 12, 28) RD_GJC(OP, 13, 29) RD_GJC(OP, 14, 30) RD_GJC(OP, 15, 31) RD_GJD(OP, 0, 16) RD_GJD(OP, 1, 17) RD_GJD(OP, 2, 18) RD_GJD(OP, 3, 19) RD_GJD(OP, 4, 20) RD_GJD(OP, 5, 21) RD_GJD(OP, 6, 22) RD_GJD(OP, 7, 23) RD_GJD(OP, 8, 24) RD_GJD(OP, 9, 25) RD_GJD(OP, 11, 27) RD_GJD(OP, 12, 28) RD_GJD(OP, 13, 29) RD_GJD(OP, 14, 30) RD_GJD(OP, 15, 31) "s_nop 1"
#define RD_GJC_S11(OP) "s_nop 1\n\t" RD_GJA(OP, 0, 16) RD_GJA(OP, 1, 17) RD_GJA(OP, 2, 18) RD_GJA(OP, 3, 19) RD_GJA(OP, 4, 20) RD_GJA(OP, 5, 21) RD_GJA(OP, 6, 22) RD_GJA(OP, 7, 23) RD_GJA(OP, 8, 24) RD_GJA(OP, 9, 25) RD_GJA(OP, 10, 26) RD_GJA(OP, 12, 28) RD_GJA(OP, 13, 29) RD_GJA(OP, 14, 30) RD_GJA(OP, 15, 31) RD_GJB(OP, 0, 16) RD_GJB(OP, 1, 17) RD_GJB(OP, 2, 18) RD_GJB(OP, 3, 19) RD_GJB(OP, 4, 20) RD_GJB(OP, 5, 21) RD_GJB(OP, 6, 22) RD_GJB(OP, 7, 23) RD_GJB(OP, 8, 24) RD_GJB(OP, 9, 25) RD_GJB(OP, 10, 26) RD_GJB(OP, 12, 28) RD_GJB(OP, 13, 29) RD_GJB(OP, 14, 30) RD_GJB(OP, 15, 31) RD_GJC(OP, 0, 16) RD_GJC(OP, 1, 17) RD_GJC(OP, 2, 18) RD_GJC(OP, 3, 19) RD_GJC(OP, 4, 20) RD_GJC(OP, 5, 21) RD_GJC(OP, 6, 22) RD_GJC(OP, 7, 23) RD_GJC(OP, 8, 24) RD_GJC(OP, 9, 25) RD_GJC(OP, 10, 26) RD_GJC(OP, 12, 28) RD_GJC(OP, 13, 29) RD_GJC(OP, 14, 30) RD_GJC(OP, 15, 31) RD_GJD(OP, 0, 16) RD_GJD(OP, 1, 17) RD_GJD(OP, 2, 18) RD_GJD(OP, 3, 19) RD_GJD(OP, 4, 20) RD_GJD(OP, 5, 21) RD_GJD(OP, 6, 22) RD_GJD(OP, 7, 23) RD_GJD(OP, 8, 24) RD_GJD(OP, 9, 25) RD_GJD(OP, 10, 26) RD_GJD(OP, 12, 28) RD_GJD(OP, 13, 29) RD_GJD(OP, 14, 30) RD_GJD(OP, 15, 31) "s_nop 1"
#define RD_GJC_S12(OP) "s_nop 1\n\t" RD_GJA(OP, 0, 16) RD_GJA(OP, 1, 17) RD_GJA(OP, 2, 18) RD_GJA(OP, 3, 19) RD_GJA(OP, 4, 20) RD_GJA(OP, 5, 21) RD_GJA(OP, 6, 22) RD_GJA(OP, 7, 23) RD_GJA(OP, 8, 24) RD_GJA(OP, 9, 25) RD_GJA(OP, 10, 26) RD_GJA(OP, 11, 27) RD_GJA(OP, 13, 29) RD_GJA(OP, 14, 30) RD_GJA(OP, 15, 31) RD_GJB(OP, 0, 16) RD_GJB(OP, 1, 17) RD_GJB(OP, 2, 18) RD_GJB(OP, 3, 19) RD_GJB(OP, 4, 20) RD_GJB(OP, 5, 21) RD_GJB(OP, 6, 22) RD_GJB(OP, 7, 23) RD_GJB(OP, 8, 24) RD_GJB(OP, 9, 25) RD_GJB(OP, 10, 26) RD_GJB(OP, 11, 27) RD_GJB(OP, 13, 29) RD_GJB(OP, 14, 30) RD_GJB(OP, 15, 31) RD_GJC(OP, 0, 16) RD_GJC(OP, 1, 17) RD_GJC(OP, 2, 18) RD_GJC(OP, 3, 19) RD_GJC(OP, 4, 20) RD_GJC(OP, 5, 21) RD_GJC(OP, 6, 22) RD_GJC(OP, 7, 23) RD_GJC(OP, 8, 24) RD_GJC(OP, 9, 25) RD_GJC(OP, 10, 26) RD_GJC(OP, 11, 27) RD_GJC(OP, 13, 29) RD_GJC(OP, 14, 30) RD_GJC(OP, 15, 31) RD_GJD(OP, 0, 16) RD_GJD(OP, 1, 17) RD_GJD(OP, 2, 18) RD_GJD(OP, 3, 19) RD_GJD(OP, 4, 20) RD_GJD(OP, 5, 21) RD_GJD(OP, 6, 22) RD_GJD(OP, 7, 23) RD_GJD(OP, 8, 24) RD_GJD(OP, 9, 25) RD_GJD(OP, 10, 26) RD_GJD(OP, 11, 27) RD_GJD(OP, 13, 29) RD_GJD(OP, 14, 30) RD_GJD(OP, 15, 31) "s_nop 1"
#define RD_GJC_S13(OP) "s_nop 1\n\t" RD_GJA(OP, 0, 16) RD_GJA(OP, 1, 17) RD_GJA(OP, 2, 18) RD_GJA(OP, 3, 19) RD_GJA(OP, 4, 20) RD_GJA(OP, 5, 21) RD_GJA(OP, 6, 22) RD_GJA(OP, 7, 23) RD_GJA(OP, 8, 24) RD_GJA(OP, 9, 25) RD_GJA(OP, 10, 26) RD_GJA(OP, 11, 27) RD_GJA(OP, 12, 28) RD_GJA(OP, 14, 30) RD_GJA(OP, 15, 31) RD_GJB(OP, 0, 16) RD_GJB(OP, 1, 17) RD_GJB(OP, 2, 18) RD_GJB(OP, 3, 19) RD_GJB(OP, 4, 20) RD_GJB(OP, 5, 21) RD_GJB(OP, 6, 22) RD_GJB(OP, 7, 23) RD_GJB(OP, 8, 24) RD_GJB(OP, 9, 25) RD_GJB(OP, 10, 26) RD_GJB(OP, 11, 27) RD_GJB(OP, 12, 28) RD_GJB(OP, 14, 30) RD_GJB(OP, 15, 31) RD_GJC(OP, 0, 16) RD_GJC(OP, 1, 17) RD_GJC(OP, 2, 18) RD_GJC(OP, 3, 19) RD_GJC(OP, 4, 20) RD_GJC(OP, 5, 21) RD_GJC(OP, 6, 22) RD_GJC(OP, 7, 23) RD_GJC(OP, 8, 24) RD_GJC(OP, 9, 25) RD_GJC(OP, 10, 26) RD_GJC(OP, 11, 27) RD_GJC(OP, 12, 28) RD_GJC(OP, 14, 30) RD_GJC(OP, 15, 31) RD_GJD(OP, 0, 16) RD_GJD(OP, 1, 17) RD_GJD(OP, 2, 18) RD_GJD(OP, 3, 19) RD_GJD(OP, 4, 20) RD_GJD(OP, 5, 21) RD_GJD(OP, 6, 22) RD_GJD(OP, 7, 23) RD_GJD(OP, 8, 24) RD_GJD(OP, 9, 25) RD_GJD(OP, 10, 26) RD_GJD(OP, 11, 27) RD_GJD(OP, 12, 28) RD_GJD(OP, 14, 30) RD_GJD(OP, 15, 31) "s_nop 1"
#define RD_GJC_S14(OP) "s_nop 1\n\t" RD_GJA(OP, 0, 16) RD_GJA(OP, 1, 17) RD_GJA(OP, 2, 18) RD_GJA(OP, 3, 19) RD_GJA(OP, 4, 20) RD_GJA(OP, 5, 21) RD_GJA(OP, 6, 22) RD_GJA(OP, 7, 23) RD_GJA(OP, 8, 24) RD_GJA(OP, 9, 25) RD_GJA(OP, 10, 26) RD_GJA(OP, 11, 27) RD_GJA(OP, 12, 28) RD_GJA(OP, 13, 29) RD_GJA(OP, 15, 31) RD_GJB(OP, 0, 16) RD_GJB(OP, 1, 17) RD_GJB(OP, 2, 18) RD_GJB(OP, 3, 19) RD_GJB(OP, 4, 20) RD_GJB(OP, 5, 21) RD_GJB(OP, 6, 22) RD_GJB(OP, 7, 23) RD_GJB(OP, 8, 24) RD_GJB(OP, 9, 25) RD_GJB(OP, 10, 26) RD_GJB(OP, 11, 27) RD_GJB(OP, 12, 28) RD_GJB(OP, 13, 29) RD_GJB(OP, 15, 31) RD_GJC(OP, 0, 16) RD_GJC(OP, 1, 17) RD_GJC(OP, 2, 18) RD_GJC(OP, 3, 19) RD_GJC(OP, 4, 20) RD_GJC(OP, 5, 21) RD_GJC(OP, 6, 22) RD_GJC(OP, 7, 23) RD_GJC(OP, 8, 24) RD_GJC(OP, 9, 25) RD_GJC(OP, 10, 26) RD_GJC(OP, 11, 27) RD_GJC(OP, 12, 28) RD_GJC(OP, 13, 29) RD_GJC(OP, 15, 31) RD_GJD(OP, 0, 16) RD_GJD(OP, 1, 17) RD_GJD(OP, 2, 18) RD_GJD(OP, 3, 19) RD_GJD(OP, 4, 20) RD_GJD(OP, 5, 21) RD_GJD(OP, 6, 22) RD_GJD(OP, 7, 23) RD_GJD(OP, 8, 24) RD_GJD(OP, 9, 25) RD_GJD(OP, 10, 26) RD_GJD(OP, 11, 27) RD_GJD(OP, 12, 28) RD_GJD(OP, 13, 29) RD_GJD(OP, 15, 31) "s_nop 1"
#define RD_GJC_S15(OP) "s_nop 1\n\t" RD_GJA(OP, 0, 16) RD_GJA(OP, 1, 17) RD_GJA(OP, 2, 18) RD_GJA(OP, 3, 19) RD_GJA(OP, 4, 20) RD_GJA(OP, 5, 21) RD_GJA(OP, 6, 22) RD_GJA(OP, 7, 23) RD_GJA(OP, 8, 24) RD_GJA(OP, 9, 25) RD_GJA(OP, 10, 26) RD_GJA(OP, 11, 27) RD_GJA(OP, 12, 28) RD_GJA(OP, 13, 29) RD_GJA(OP, 14, 30) RD_GJB(OP, 0, 16) RD_GJB(OP, 1, 17) RD_GJB(OP, 2, 18) RD_GJB(OP, 3, 19) RD_GJB(OP, 4, 20) RD_GJB(OP, 5, 21) RD_GJB(OP, 6, 22) RD_GJB(OP, 7, 23) RD_GJB(OP, 8, 24) RD_GJB(OP, 9, 25) RD_GJB(OP, 10, 26) RD_GJB(OP, 11, 27) RD_GJB(OP, 12, 28) RD_GJB(OP, 13, 29) RD_GJB(OP, 14, 30) RD_GJC(OP, 0, 16) RD_GJC(OP, 1, 17) RD_GJC(OP, 2, 18) RD_GJC(OP, 3, 19) RD_GJC(OP, 4, 20) RD_GJC(OP, 5, 21) RD_GJC(OP, 6, 22) RD_GJC(OP, 7, 23) RD_GJC(OP, 8, 24) RD_GJC(OP, 9, 25) RD_GJC(OP, 10, 26) RD_GJC(OP, 11, 27) RD_GJC(OP, 12, 28) RD_GJC(OP, 13, 29) RD_GJC(OP, 14, 30) RD_GJD(OP, 0, 16) RD_GJD(OP, 1, 17) RD_GJD(OP, 2, 18) RD_GJD(OP, 3, 19) RD_GJD(OP, 4, 20) RD_GJD(OP, 5, 21) RD_GJD(OP, 6, 22) RD_GJD(OP, 7, 23) RD_GJD(OP, 8, 24) RD_GJD(OP, 9, 25) RD_GJD(OP, 10, 26) RD_GJD(OP, 11, 27) RD_GJD(OP, 12, 28) RD_GJD(OP, 13, 29) RD_GJD(OP, 14, 30) "s_nop 1"
template <int KK, typename T>
__device__ __forceinline__ void fused_gj_cplx_k(T (&ar)[16], T (&ai)[16], T fr, T fi) {
#define OPERANDS                                                                                  \
    : "+v"(ar[0]), "+v"(ar[1]), "+v"(ar[2]), "+v"(ar[3]), "+v"(ar[4]), "+v"(ar[5]),             \
      "+v"(ar[6]), "+v"(ar[7]), "+v"(ar[8]), "+v"(ar[9]), "+v"(ar[10]), "+v"(ar[11]),            \
      "+v"(ar[12]), "+v"(ar[13]), "+v"(ar[14]), "+v"(ar[15]), "+v"(ai[0]), "+v"(ai[1]),          \
      "+v"(ai[2]), "+v"(ai[3]), "+v"(ai[4]), "+v"(ai[5]), "+v"(ai[6]), "+v"(ai[7]),              \
      "+v"(ai[8]), "+v"(ai[9]), "+v"(ai[10]), "+v"(ai[11]), "+v"(ai[12]), "+v"(ai[13]),          \
      "+v"(ai[14]), "+v"(ai[15])                                                                  \
    : "v"(fr), "v"(fi), "n"(KK)
    if constexpr (KK == 0) RD_ASM2(T, RD_GJC_S0, OPERANDS);
    else if constexpr (KK == 1) RD_ASM2(T, RD_GJC_S1, OPERANDS);
    else if constexpr (KK == 2) RD_ASM2(T, RD_GJC_S2, OPERANDS);
    else if constexpr (KK == 3) RD_ASM2(T, RD_GJC_S3, OPERANDS);
    else if constexpr (KK == 4) RD_ASM2(T, RD_GJC_S4, OPERANDS);
    else if constexpr (KK == 5) RD_ASM2(T, RD_GJC_S5, OPERANDS);
    else if constexpr (KK == 6) RD_ASM2(T, RD_GJC_S6, OPERANDS);
    else if constexpr (KK == 7) RD_ASM2(T, RD_GJC_S7, OPERANDS);
    else if constexpr (KK == 8) RD_ASM2(T, RD_GJC_S8, OPERANDS);
    else if constexpr (KK == 9) RD_ASM2(T, RD_GJC_S9, OPERANDS);
    else if constexpr (KK == 10) RD_ASM2(T, RD_GJC_S10, OPERANDS);
    else if constexpr (KK == 11) RD_ASM2(T, RD_GJC_S11, OPERANDS);
    else if constexpr (KK == 12) RD_ASM2(T, RD_GJC_S12, OPERANDS);
    else if constexpr (KK == 13) RD_ASM2(T, RD_GJC_S13, OPERANDS);
    else if constexpr (KK == 14) RD_ASM2(T, RD_GJC_S14, OPERANDS);
    else if constexpr (KK == 15) RD_ASM2(T, RD_GJC_S15, OPERANDS);
#undef OPERANDS
}
#undef RD_GJC_S0
#undef RD_GJC_S1
#undef RD_GJC_S2
#undef RD_GJC_S3
#undef RD_GJC_S4
#undef RD_GJC_S5
#undef RD_GJC_S6
#undef RD_GJC_S7
#undef RD_GJC_S8
#undef RD_GJC_S9
#undef RD_GJC_S10
#undef RD_GJC_S11
#undef RD_GJC_S12
#undef RD_GJC_S13
#undef RD_GJC_S14
#undef RD_GJC_S15
#undef RD_GJA
#undef RD_GJB
#undef RD_GJC
#undef RD_GJD

/* The same step for the 8-column engine (m <= 8); four sweeps of seven, so
 * a register written in one sweep is read through DPP seven or more
 * instructions later. */
#define RD_GJA8(OP, R, I) OP " %" #R ", %" #I ", %17 row_newbcast:%18 row_mask:0xf bank_mask:0xf\n\t"
#define RD_GJB8(OP, R, I) OP " %" #I ", %" #R ", -%17 row_newbcast:%18 row_mask:0xf bank_mask:0xf\n\t"
#define RD_GJC8(OP, R, I) OP " %" #R ", %" #R ", -%16 row_newbcast:%18 row_mask:0xf bank_mask:0xf\n\t"
#define RD_GJD8(OP, R, I) OP " %" #I ", %" #I ", -%16 row_newbcast:%18 row_mask:0xf bank_mask:0xf\n\t"
#define RD_GJC8_S0(OP) "s_nop 1\n\t" RD_GJA8(OP, 1, 9) RD_GJA8(OP, 2, 10) RD_GJA8(OP, 3, 11) RD_GJA8(OP, 4, 12) RD_GJA8(OP, 5, 13) RD_GJA8(OP, 6, 14) RD_GJA8(OP, 7, 15) RD_GJB8(OP, 1, 9) RD_GJB8(OP, 2, 10) RD_GJB8(OP, 3, 11) RD_GJB8(OP, 4, 12) RD_GJB8(OP, 5, 13) RD_GJB8(OP, 6, 14) RD_GJB8(OP, 7, 15) RD_GJC8(OP, 1, 9) RD_GJC8(OP, 2, 10) RD_GJC8(OP, 3, 11) RD_GJC8(OP, 4, 12) RD_GJC8(OP, 5, 13) RD_GJC8(OP, 6, 14) RD_GJC8(OP, 7, 15) RD_GJD8(OP, 1, 9) RD_GJD8(OP, 2, 10) RD_GJD8(OP, 3, 11) RD_GJD8(OP, 4, 12) RD_GJD8(OP, 5, 13) RD_GJD8(OP, 6, 14) RD_GJD8(OP, 7, 15) "s_nop 1"
#define RD_GJC8_S1(OP) "s_nop 1\n\t" RD_GJA8(OP, 0, 8) RD_GJA8(OP, 2, 10) RD_GJA8(OP, 3, 11) RD_GJA8(OP, 4, 12) RD_GJA8(OP, 5, 13) RD_GJA8(OP, 6, 14) RD_GJA8(OP, 7, 15) RD_GJB8(OP, 0, 8) RD_GJB8(OP, 2, 10) RD_GJB8(OP, 3, 11) RD_GJB8(OP, 4, 12) RD_GJB8(OP, 5, 13) RD_GJB8(OP, 6, 14) RD_GJB8(OP, 7, 15) RD_GJC8(OP, 0, 8) RD_GJC8(OP, 2, 10) RD_GJC8(OP, 3, 11) RD_GJC8(OP, 4, 12) RD_GJC8(OP, 5, 13) RD_GJC8(OP, 6, 14) RD_GJC8(OP, 7, 15) RD_GJD8(OP, 0, 8) RD_GJD8(OP, 2, 10) RD_GJD8(OP, 3, 11) RD_GJD8(OP, 4, 12) RD_GJD8(OP, 5, 13) RD_GJD8(OP, 6, 14) RD_GJD8(OP, 7, 15) "s_nop 1"
#define RD_GJC8_S2(OP) "s_nop 1\n\t" RD_GJA8(OP, 0, 8) RD_GJA8(OP, 1, 9) RD_GJA8(OP, 3, 11) RD_GJA8(OP, 4, 12) RD_GJA8(OP, 5, 13) RD_GJA8(OP, 6, 14) RD_GJA8(OP, 7, 15) RD_GJB8(OP, 0, 8) RD_GJB8(OP, 1, 9) RD_GJB8(OP, 3, 11) RD_GJB8(OP, 4, 12) RD_GJB8(OP, 5, 13) RD_GJB8(OP, 6, 14) RD_GJB8(OP, 7, 15) RD_GJC8(OP, 0, 8) RD_GJC8(OP, 1, 9) RD_GJC8(OP, 3, 11) RD_GJC8(OP, 4, 12) RD_GJC8(OP, 5, 13) RD_GJC8(OP, 6, 14) RD_GJC8(OP, 7, 15) RD_GJD8(OP, 0, 8) RD_GJD8(OP, 1, 9) RD_GJD8(OP, 3, 11) RD_GJD8(OP, 4, 12) RD_GJD8(OP, 5, 13) RD_GJD8(OP, 6, 14) RD_GJD8(OP, 7, 15) "s_nop 1"
#define RD_GJC8_S3(OP) "s_nop 1\n\t" RD_GJA8(OP, 0, 8) RD_GJA8(OP, 1, 9) RD_GJA8(OP, 2, 10) RD_GJA8(OP, 4, 12) RD_GJA8(OP, 5, 13) RD_GJA8(OP, 6, 14) RD_GJA8(OP, 7, 15) RD_GJB8(OP, 0, 8) RD_GJB8(OP, 1, 9) RD_GJB8(OP, 2, 10) RD_GJB8(OP, 4, 12) RD_GJB8(OP, 5, 13) RD_GJB8(OP, 6, 14) RD_GJB8(OP, 7, 15) RD_GJC8(OP, 0, 8) RD_GJC8(OP, 1, 9) RD_GJC8(OP, 2, 10) RD_GJC8(OP, 4, 12) RD_GJC8(OP, 5, 13) RD_GJC8(OP, 6, 14) RD_GJC8(OP, 7, 15) RD_GJD8(OP, 0, 8) RD_GJD8(OP, 1, 9) RD_GJD8(OP, 2, 10) RD_GJD8(OP, 4, 12) RD_GJD8(OP, 5, 13) RD_GJD8(OP, 6, 14) RD_GJD8(OP, 7, 15) "s_nop 1"
#define RD_GJC8_S4(OP) "s_nop 1\n\t" RD_GJA8(OP, 0, 8) RD_GJA8(OP, 1, 9) RD_GJA8(OP, 2, 10) RD_GJA8(OP, 3, 11) RD_GJA8(OP, 5, 13) RD_GJA8(OP, 6, 14) RD_GJA8(OP, 7, 15) RD_GJB8(OP, 0, 8) RD_GJB8(OP, 1, 9) RD_GJB8(OP, 2, 10) RD_GJB8(OP, 3, 11) RD_GJB8(OP, 5, 13) RD_GJB8(OP, 6, 14) RD_GJB8(OP, 7, 15) RD_GJC8(OP, 0, 8) RD_GJC8(OP, 1, 9) RD_GJC8(OP, 2, 10) RD_GJC8(OP, 3, 11) RD_GJC8(OP, 5, 13) RD_GJC8(OP, 6, 14) RD_GJC8(OP, 7, 15) RD_GJD8(OP, 0, 8) RD_GJD8(OP, 1, 9) RD_GJD8(OP, 2, 10) RD_GJD8(OP, 3, 11) RD_GJD8(OP, 5, 13) RD_GJD8(OP, 6, 14) RD_GJD8(OP, 7, 15) "s_nop 1"
#define RD_GJC8_S5(OP) "s_nop 1\n\t" RD_GJA8(OP, 0, 8) RD_GJA8(OP, 1, 9) RD_GJA8(OP, 2, 10) RD_GJA8(OP, 3, 11) RD_GJA8(OP, 4, 12) RD_GJA8(OP, 6, 14) RD_GJA8(OP, 7, 15) RD_GJB8(OP, 0, 8) RD_GJB8(OP, 1, 9) RD_GJB8(OP, 2, 10) RD_GJB8(OP, 3, 11) RD_GJB8(OP, 4, 12) RD_GJB8(OP, 6, 14) RD_GJB8(OP, 7, 15) RD_GJC8(OP, 0, 8) RD_GJC8(OP, 1, 9) RD_GJC8(OP, 2, 10) RD_GJC8(OP, 3, 11) RD_GJC8(OP, 4, 12) RD_GJC8(OP, 6, 14) RD_GJC8(OP, 7, 15) RD_GJD8(OP, 0, 8) RD_GJD8(OP, 1, 9) RD_GJD8(OP, 2, 10) RD_GJD8(OP, 3, 11) RD_GJD8(OP, 4, 12) RD_GJD8(OP, 6, 14) RD_GJD8(OP, 7, 15) "s_nop 1"
#define RD_GJC8_S6(OP) "s_nop 1\n\t" RD_GJA8(OP, 0, 8) RD_GJA8(OP, 1, 9) RD_GJA8(OP, 2, 10) RD_GJA8(OP, 3, 11) RD_GJA8(OP, 4, 12) RD_GJA8(OP, 5, 13) RD_GJA8(OP, 7, 15) RD_GJB8(OP, 0, 8) RD_GJB8(OP, 1, 9) RD_GJB8(OP, 2, 10) RD_GJB8(OP, 3, 11) RD_GJB8(OP, 4, 12) RD_GJB8(OP, 5, 13) RD_GJB8(OP, 7, 15) RD_GJC8(OP, 0, 8) RD_GJC8(OP, 1, 9) RD_GJC8(OP, 2, 10) RD_GJC8(OP, 3, 11) RD_GJC8(OP, 4, 12) RD_GJC8(OP, 5, 13) RD_GJC8(OP, 7, 15) RD_GJD8(OP, 0, 8) RD_GJD8(OP, 1, 9) RD_GJD8(OP, 2, 10) RD_GJD8(OP, 3, 11) RD_GJD8(OP, 4, 12) RD_GJD8(OP, 5, 13) RD_GJD8(OP, 7, 15) "s_nop 1"
#define RD_GJC8_S7(OP) "s_nop 1\n\t" RD_GJA8(OP, 0, 8) RD_GJA8(OP, 1, 9) RD_GJA8(OP, 2, 10) RD_GJA8(OP, 3, 11) RD_GJA8(OP, 4, 12) RD_GJA8(OP, 5, 13) RD_GJA8(OP, 6, 14) RD_GJB8(OP, 0, 8) RD_GJB8(OP, 1, 9) RD_GJB8(OP, 2, 10) RD_GJB8(OP, 3, 11) RD_GJB8(OP, 4, 12) RD_GJB8(OP, 5, 13) RD_GJB8(OP, 6, 14) RD_GJC8(OP, 0, 8) RD_GJC8(OP, 1, 9) RD_GJC8(OP, 2, 10) RD_GJC8(OP, 3, 11) RD_GJC8(OP, 4, 12) RD_GJC8(OP, 5, 13) RD_GJC8(OP, 6, 14) RD_GJD8(OP, 0, 8) RD_GJD8(OP, 1, 9) RD_GJD8(OP, 2, 10) RD_GJD8(OP, 3, 11) RD_GJD8(OP, 4, 12) RD_GJD8(OP, 5, 13) RD_GJD8(OP, 6, 14) "s_nop 1"
template <int KK, typename T>
__device__ __forceinline__ void fused_gj_cplx8_k(T (&ar)[8], T (&ai)[8], T fr, T fi) {
#define OPERANDS                                                                                  \
    : "+v"(ar[0]), "+v"(ar[1]), "+v"(ar[2]), "+v"(ar[3]), "+v"(ar[4]), "+v"(ar[5]),             \
      "+v"(ar[6]), "+v"(ar[7]), "+v"(ai[0]), "+v"(ai[1]), "+v"(ai[2]), "+v"(ai[3]),              \
      "+v"(ai[4]), "+v"(ai[5]), "+v"(ai[6]), "+v"(ai[7])                                         \
    : "v"(fr), "v"(fi), "n"(KK)
    if constexpr (KK == 0) RD_ASM2(T, RD_GJC8_S0, OPERANDS);
    else if constexpr (KK == 1) RD_ASM2(T, RD_GJC8_S1, OPERANDS);
    else if constexpr (KK == 2) RD_ASM2(T, RD_GJC8_S2, OPERANDS);
    else if constexpr (KK == 3) RD_ASM2(T, RD_GJC8_S3, OPERANDS);
    else if constexpr (KK == 4) RD_ASM2(T, RD_GJC8_S4, OPERANDS);
    else if constexpr (KK == 5) RD_ASM2(T, RD_GJC8_S5, OPERANDS);
    else if constexpr (KK == 6) RD_ASM2(T, RD_GJC8_S6, OPERANDS);
    else if constexpr (KK == 7) RD_ASM2(T, RD_GJC8_S7, OPERANDS);
#undef OPERANDS
}
#undef RD_GJC8_S0
#undef RD_GJC8_S1
#undef RD_GJC8_S2
#undef RD_GJC8_S3
#undef RD_GJC8_S4
#undef RD_GJC8_S5
#undef RD_GJC8_S6
#undef RD_GJC8_S7
#undef RD_GJA8
#undef RD_GJB8
#undef RD_GJC8
#undef RD_GJD8

/* Run-time pivot lane (a constant after the caller's loop is unrolled);
 * NC: columns of the engine (16, or 8 for m <= 8). */
template <int NC, typename T>
__device__ __forceinline__ void fused_gj_real(T (&a)[NC], T f, int kk) {
    static_assert(NC == 8 || NC == 16, "8 or 16 columns");
    switch (kk) {
#define RD_C(K)                                                                                   \
    case K:                                                                                       \
        if constexpr (NC == 16) fused_gj_real_k<K>(a, f);                                         \
        else if constexpr (K < 8) fused_gj_real8_k<K>(a, f);                                      \
        break;
        RD_C(0) RD_C(1) RD_C(2) RD_C(3) RD_C(4) RD_C(5) RD_C(6) RD_C(7)
        RD_C(8) RD_C(9) RD_C(10) RD_C(11) RD_C(12) RD_C(13) RD_C(14) RD_C(15)
#undef RD_C
    }
}
template <int NC, typename T>
__device__ __forceinline__ void fused_gj_cplx(T (&ar)[NC], T (&ai)[NC], T fr, T fi, int kk) {
    static_assert(NC == 8 || NC == 16, "8 or 16 columns");
    switch (kk) {
#define RD_C(K)                                                                                   \
    case K:                                                                                       \
        if constexpr (NC == 16) fused_gj_cplx_k<K>(ar, ai, fr, fi);                               \
        else if constexpr (K < 8) fused_gj_cplx8_k<K>(ar, ai, fr, fi);                            \
        break;
        RD_C(0) RD_C(1) RD_C(2) RD_C(3) RD_C(4) RD_C(5) RD_C(6) RD_C(7)
        RD_C(8) RD_C(9) RD_C(10) RD_C(11) RD_C(12) RD_C(13) RD_C(14) RD_C(15)
#undef RD_C
    }
}

#undef RD_ASM2
#undef RD_F64
#undef RD_F32
#undef RD_FM
#undef RD_FMN

}  // namespace rd
