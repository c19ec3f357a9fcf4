/*
 * rd_kernels_small.hip -- reaction-step kernels with one cell per lane
 * (m <= 4: Oregonator, Robertson, NAGUMO, small linear / kinetics models).
 *
 * Two schedules over the same per-cell engine (bitwise-identical results):
 *
 *  - one launch per batch: lane c owns cell c start to finish; a wave lives
 *    as long as its slowest cell.
 *  - persistent work stealing: a grid sized to the resident capacity of the
 *    chip; a lane whose cell has finished stores it and claims the next cell
 *    index from a global counter (one atomic per wave per refill, the claims of
 *    all idle lanes aggregated).  Every pass of the loop advances each busy
 *    lane by exactly one Newton iteration, plus step start / step end work for
 *    the lanes that need it, so lanes of one wave desynchronise freely.  This
 *    replaces the CPU design's dynamic work stealing over leaves (paper §3.2,
 *    parallel_for over a blocked range; §4.2 on the uneven reaction cost).
 *
 * Every wave leaves the loop once all cell indices are claimed and its own
 * cells are finished; each cell finishes within max_steps step attempts.
 */
#include <hip/hip_runtime.h>

#include "rd_small_kernels.h"

namespace rd {

__global__ void k_reset(unsigned long long* p, int n) {
    const int i = threadIdx.x;
    if (i < n) p[i] = 0ull;
}

hipError_t launch_reset(unsigned long long* p, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

#define RD_TUNE_SET(KIND, MODEL, M, PREC, LT, TAG)                                            \
    RD_PERS(KIND, MODEL, M, PREC, LT, false, 2, 128, 1, 1, TAG ".persistent.b128.fs1"),       \
    RD_PERS(KIND, MODEL, M, PREC, LT, false, 3, 128, 1, 24, TAG ".persistent.b128.fs24"),     \
    RD_PERS(KIND, MODEL, M, PREC, LT, false, 4, 128, 1, 32, TAG ".persistent.b128.fs32"),     \
    RD_PERS(KIND, MODEL, M, PREC, LT, false, 5, 128, 1, 48, TAG ".persistent.b128.fs48"),     \
    RD_PERS(KIND, MODEL, M, PREC, LT, false, 6, 128, 1, 56, TAG ".persistent.b128.fs56"),     \
    RD_PERS(KIND, MODEL, M, PREC, LT, false, 7, 256, 1, 40, TAG ".persistent.b256.fs40"),     \
    RD_PERS(KIND, MODEL, M, PREC, LT, false, 8, 64, 1, 40, TAG ".persistent.b64.fs40"),       \
    RD_PERS(KIND, MODEL, M, PREC, LT, false, 9, 128, 1, 40, TAG ".persistent.b128.fs40"),     \
    RD_PERS_K(KIND, MODEL, M, PREC, LT, 10, 128, 1, 40, TAG ".persistent.b128.fs40.kp"),      \
    RD_PERS_K(KIND, MODEL, M, PREC, LT, 11, 64, 1, 40, TAG ".persistent.b64.fs40.kp"),        \
    RD_PERS_K(KIND, MODEL, M, PREC, LT, 12, 256, 1, 48, TAG ".persistent.b256.fs48.kp"),      \
    RD_PERS(KIND, MODEL, M, PREC, LT, false, 13, 128, 3, 32, TAG ".persistent.b128.w3.fs32"),  \
    RD_PERS(KIND, MODEL, M, PREC, LT, false, 14, 128, 3, 48, TAG ".persistent.b128.w3.fs48"),  \
    RD_PERS(KIND, MODEL, M, PREC, LT, false, 15, 64, 3, 40, TAG ".persistent.b64.w3.fs40"),    \
    RD_PERS(KIND, MODEL, M, PREC, LT, false, 16, 192, 3, 40, TAG ".persistent.b192.w3.fs40"),  \
    RD_PERS(KIND, MODEL, M, PREC, LT, false, 17, 128, 4, 40, TAG ".persistent.b128.w4.fs40"),  \
    RD_PERS_K(KIND, MODEL, M, PREC, LT, 18, 128, 3, 40, TAG ".persistent.b128.w3.fs40.kp"),   \
    RD_PERS_P(KIND, MODEL, M, PREC, LT, 19, 128, 3, 40, 3, TAG ".persistent.b128.w3.fs40.p3"), \
    RD_PERS_P(KIND, MODEL, M, PREC, LT, 20, 128, 3, 40, 6, TAG ".persistent.b128.w3.fs40.p6"), \
    RD_PERS_P(KIND, MODEL, M, PREC, LT, 21, 128, 3, 40, 12, TAG ".persistent.b128.w3.fs40.p12"), \
    RD_PERS_P(KIND, MODEL, M, PREC, LT, 22, 128, 3, 24, 6, TAG ".persistent.b128.w3.fs24.p6"), \
    RD_PERS_P(KIND, MODEL, M, PREC, LT, 23, 128, 3, 32, 3, TAG ".persistent.b128.w3.fs32.p3"), \
    RD_PERS_P(KIND, MODEL, M, PREC, LT, 24, 128, 3, 32, 2, TAG ".persistent.b128.w3.fs32.p2"), \
    RD_PERS_P(KIND, MODEL, M, PREC, LT, 25, 128, 3, 32, 4, TAG ".persistent.b128.w3.fs32.p4"), \
    RD_PERS_P(KIND, MODEL, M, PREC, LT, 26, 128, 3, 28, 3, TAG ".persistent.b128.w3.fs28.p3"), \
    RD_PERS(KIND, MODEL, M, PREC, LT, false, 27, 128, 3, 40, TAG ".persistent.b128.w3.fs40"),  \
    RD_PERS_P(KIND, MODEL, M, PREC, LT, 28, 128, 3, 40, 2, TAG ".persistent.b128.w3.fs40.p2"), \
    RD_PERS_P(KIND, MODEL, M, PREC, LT, 29, 128, 3, 64, 2, TAG ".persistent.b128.w3.fs64.p2"), \
    RD_PERS_U(KIND, MODEL, M, PREC, LT, 30, 128, 3, 40, 2, 64, 40, TAG ".persistent.b128.w3.fs40.p2.u64"), \
    RD_PERS_U(KIND, MODEL, M, PREC, LT, 31, 128, 3, 40, 2, 40, 64, TAG ".persistent.b128.w3.fs40.p2.l64"), \
    RD_PERS_U(KIND, MODEL, M, PREC, LT, 32, 128, 3, 40, 2, 64, 64, TAG ".persistent.b128.w3.fs40.p2.u64.l64"), \
    RD_PERS_A(KIND, MODEL, M, PREC, LT, 33, 128, 3, 48, 2, 64, 64, TAG ".persistent.b128.w3.fs48.p2.u64.l64.aos"), \
    RD_PERS_U(KIND, MODEL, M, PREC, LT, 34, 128, 3, 48, 2, 64, 64, TAG ".persistent.b128.w3.fs48.p2.u64.l64"), \
    RD_PERS_C(KIND, MODEL, M, PREC, LT, 35, 128, 3, 48, 2, 64, 64, 16, TAG ".persistent.b128.w3.fs48.p2.u64.l64.c16"), \
    RD_PERS_C(KIND, MODEL, M, PREC, LT, 36, 128, 3, 48, 2, 64, 64, 24, TAG ".persistent.b128.w3.fs48.p2.u64.l64.c24"), \
    RD_PERS_C(KIND, MODEL, M, PREC, LT, 37, 128, 3, 48, 2, 64, 64, 36, TAG ".persistent.b128.w3.fs48.p2.u64.l64.c36"), \
    RD_PERS_C(KIND, MODEL, M, PREC, LT, 38, 128, 3, 56, 2, 64, 64, 28, TAG ".persistent.b128.w3.fs56.p2.u64.l64.c28"), \
    RD_PERS_C(KIND, MODEL, M, PREC, LT, 39, 128, 3, 64, 2, 64, 64, 28, TAG ".persistent.b128.w3.fs64.p2.u64.l64.c28"), \
    RD_PERS_C(KIND, MODEL, M, PREC, LT, 40, 256, 3, 48, 2, 64, 64, 28, TAG ".persistent.b256.w3.fs48.p2.u64.l64.c28"), \
    RD_PERS_C(KIND, MODEL, M, PREC, LT, 41, 128, 3, 48, 0, 48, 48, 28, TAG ".persistent.b128.w3.fs48.c28"), \
    RD_PERS_C(KIND, MODEL, M, PREC, LT, 42, 128, 3, 48, 2, 48, 48, 28, TAG ".persistent.b128.w3.fs48.p2.c28"), \
    RD_PERS_C(KIND, MODEL, M, PREC, LT, 43, 64, 3, 48, 2, 64, 64, 28, TAG ".persistent.b64.w3.fs48.p2.u64.l64.c28"), \
    RD_ONE(KIND, MODEL, M, PREC, LT, false, 2, 256, 1, 16, TAG ".onelaunch.b256.fs16"),       \
    RD_ONE(KIND, MODEL, M, PREC, LT, false, 3, 256, 1, 1, TAG ".onelaunch.b256.fs1")

static const KernelEntry g_small_table[] = {
    RD_MODEL_SET(K_OREG, Oregonator, 3, "oregonator"),
    RD_TUNE_SET(K_OREG, Oregonator, 3, 0, double, "oregonator.fp64"),
    RD_TUNE_SET(K_OREG, Oregonator, 3, 1, float, "oregonator.mixed"),
    RD_MODEL_SET(K_ROB, Robertson, 3, "robertson"),
    RD_MODEL_SET(K_NAG, Nagumo, 1, "nagumo"),
    RD_MODEL_SET(K_LIN, Linear<1>, 1, "linear1"),
    RD_MODEL_SET(K_LIN, Linear<2>, 2, "linear2"),
    RD_MODEL_SET_W(K_LIN, Linear<3>, 3, "linear3", 1),
    RD_MODEL_SET_W(K_LIN, Linear<4>, 4, "linear4", 1),
    RD_MODEL_SET(K_KIN, Kinetics<1>, 1, "kinetics1"),
    RD_MODEL_SET(K_KIN, Kinetics<2>, 2, "kinetics2"),
    RD_MODEL_SET_W(K_KIN, Kinetics<3>, 3, "kinetics3", 1),
    RD_MODEL_SET_W(K_KIN, Kinetics<4>, 4, "kinetics4", 1),
};

const KernelEntry* small_kernel_table(int* count) {
    *count = (int)(sizeof(g_small_table) / sizeof(g_small_table[0]));
    return g_small_table;
}

}  // namespace rd

RD_PH_READER(rd_phase_read_small)
