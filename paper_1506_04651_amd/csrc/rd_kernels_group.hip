/*
 * rd_kernels_group.hip -- reaction-step kernels for 5 <= m <= 16 with
 * analytic Jacobians (the synthetic stiff kinetics and linear test models) on
 * the 16-lane-group engine (rd_group_kernels.h).
 */
#include <hip/hip_runtime.h>

#include "rd_group_kernels.h"

namespace rd {

/* The 8-column kernels registered for 1 <= m <= 4 as well, as further
 * variants beside the one-lane kernels (variant 1): the same models with
 * sixteen lanes per cell instead of one, four cells per wave instead of 64.
 * Their arithmetic differs from the one-lane engine's (Gauss-Jordan inverses,
 * pivot choice R25), so they agree with it to rounding, not bitwise. */
#define RD_G16_SMALL(KIND, MODEL, TAG, M)                                                          \
    {KIND, 0, M, 0, 0, false, 2, 256, 256 / kGroup, TAG ".lanes16.g16c8.fp64.persistent.b256.w3.fs4", \
     &launch_group_pers<MODEL, double, false, 256, 3, 4, true, 8>,                                 \
     (const void*)&k_group_persistent<MODEL, double, false, 256, 3, 4, true, 8>},                  \
    {KIND, 0, M, 1, 0, false, 2, 256, 256 / kGroup, TAG ".lanes16.g16c8.mixed.persistent.b256.w4.fs4", \
     &launch_group_pers<MODEL, float, false, 256, 4, 4, true, 8>,                                  \
     (const void*)&k_group_persistent<MODEL, float, false, 256, 4, 4, true, 8>},                   \
    {KIND, 0, M, 0, 1, false, 2, 256, 256 / kGroup, TAG ".lanes16.g16c8.fp64.onelaunch.b256",       \
     &launch_group_one<MODEL, double, false, 256, 1, 1, true, 8>,                                  \
     (const void*)&k_group_onelaunch<MODEL, double, false, 256, 1, 1, true, 8>},                   \
    {KIND, 0, M, 1, 1, false, 2, 256, 256 / kGroup, TAG ".lanes16.g16c8.mixed.onelaunch.b256",      \
     &launch_group_one<MODEL, float, false, 256, 1, 1, true, 8>,                                   \
     (const void*)&k_group_onelaunch<MODEL, float, false, 256, 1, 1, true, 8>}

static const KernelEntry g_group_table[] = {
    RD_G16_SMALL(2, GroupKinetics, "kinetics", 1), RD_G16_SMALL(2, GroupKinetics, "kinetics", 2),
    RD_G16_SMALL(2, GroupKinetics, "kinetics", 3), RD_G16_SMALL(2, GroupKinetics, "kinetics", 4),
    RD_G16_SMALL(4, GroupLinear, "linear", 1), RD_G16_SMALL(4, GroupLinear, "linear", 2),
    RD_G16_SMALL(4, GroupLinear, "linear", 3), RD_G16_SMALL(4, GroupLinear, "linear", 4),
    RD_GONE(2, GroupKinetics, 0, double, false, 1, 256, 1, 1, "kinetics.g16.fp64.onelaunch.b256"),
    RD_GONE(2, GroupKinetics, 1, float, false, 1, 256, 1, 1, "kinetics.g16.mixed.onelaunch.b256"),
    RD_GPERS_C(2, GroupKinetics, 0, double, 1, 256, 3, 4, 16, "kinetics.g16.fp64.persistent.b256.w3.fs4.cold"),
    RD_GPERS(2, GroupKinetics, 1, float, false, 1, 256, 3, 4, "kinetics.g16.mixed.persistent.b256.w3.fs4"),
    RD_GPERS(2, GroupKinetics, 0, double, false, 2, 256, 1, 2, "kinetics.g16.fp64.persistent.b256.fs2"),
    RD_GPERS(2, GroupKinetics, 1, float, false, 2, 256, 1, 2, "kinetics.g16.mixed.persistent.b256.fs2"),
    RD_GPERS(2, GroupKinetics, 0, double, false, 3, 256, 2, 1, "kinetics.g16.fp64.persistent.b256.w2.fs1"),
    RD_GPERS(2, GroupKinetics, 1, float, false, 3, 256, 2, 1, "kinetics.g16.mixed.persistent.b256.w2.fs1"),
    RD_GPERS(2, GroupKinetics, 0, double, false, 4, 256, 2, 2, "kinetics.g16.fp64.persistent.b256.w2.fs2"),
    RD_GPERS(2, GroupKinetics, 1, float, false, 4, 256, 2, 2, "kinetics.g16.mixed.persistent.b256.w2.fs2"),
    RD_GPERS(2, GroupKinetics, 0, double, false, 5, 256, 3, 2, "kinetics.g16.fp64.persistent.b256.w3.fs2"),
    RD_GPERS(2, GroupKinetics, 1, float, false, 5, 256, 3, 2, "kinetics.g16.mixed.persistent.b256.w3.fs2"),
    /* the same kernel as variant 1 with separate DPP moves and FMAs */
    RD_GPERS_X(2, GroupKinetics, 0, double, false, 6, 256, 2, 4, false, 16,
               "kinetics.g16.fp64.persistent.b256.w2.fs4.unfused"),
    RD_GPERS(2, GroupKinetics, 1, float, false, 6, 256, 3, 3, "kinetics.g16.mixed.persistent.b256.w3.fs3"),
    RD_GPERS(2, GroupKinetics, 0, double, false, 7, 256, 2, 3, "kinetics.g16.fp64.persistent.b256.w2.fs3"),
    RD_GPERS(2, GroupKinetics, 1, float, false, 7, 256, 2, 3, "kinetics.g16.mixed.persistent.b256.w2.fs3"),
    RD_GPERS(2, GroupKinetics, 1, float, false, 8, 128, 3, 4, "kinetics.g16.mixed.persistent.b128.w3.fs4"),
    RD_GPERS_X(2, GroupKinetics, 1, float, false, 9, 256, 3, 4, false, 16,
               "kinetics.g16.mixed.persistent.b256.w3.fs4.unfused"),
    RD_GPERS(2, GroupKinetics, 1, float, false, 10, 256, 4, 4, "kinetics.g16.mixed.persistent.b256.w4.fs4"),
    RD_GPERS(2, GroupKinetics, 1, float, false, 11, 256, 4, 3, "kinetics.g16.mixed.persistent.b256.w4.fs3"),
    RD_GPERS(2, GroupKinetics, 0, double, false, 8, 256, 3, 4, "kinetics.g16.fp64.persistent.b256.w3.fs4"),
    RD_GPERS(2, GroupKinetics, 0, double, false, 9, 128, 2, 4, "kinetics.g16.fp64.persistent.b128.w2.fs4"),
    /* cold per-cell values in LDS */
    RD_GPERS_C(2, GroupKinetics, 1, float, 12, 256, 3, 4, 16, "kinetics.g16.mixed.persistent.b256.w3.fs4.cold"),
    RD_GPERS_C(2, GroupKinetics, 1, float, 13, 256, 3, 3, 16, "kinetics.g16.mixed.persistent.b256.w3.fs3.cold"),
    RD_GPERS(2, GroupKinetics, 0, double, false, 10, 256, 2, 4, "kinetics.g16.fp64.persistent.b256.w2.fs4"),
    RD_GPERS_C(2, GroupKinetics, 0, double, 11, 256, 2, 4, 16, "kinetics.g16.fp64.persistent.b256.w2.fs4.cold"),
    RD_GPERS_C(2, GroupKinetics, 0, double, 12, 128, 3, 4, 16, "kinetics.g16.fp64.persistent.b128.w3.fs4.cold"),
    RD_GONE(2, GroupKinetics, 0, double, true, 1, 256, 1, 1, "kinetics.g16.fp64.onelaunch.fixed"),
    RD_GPERS(2, GroupKinetics, 0, double, true, 1, 256, 1, 1, "kinetics.g16.fp64.persistent.fixed"),
    /* 8 columns (m = 5..8) */
    RD_GONE_X(2, GroupKinetics, 0, double, false, 1, 256, 1, 1, 8, "kinetics.g16c8.fp64.onelaunch.b256"),
    RD_GONE_X(2, GroupKinetics, 1, float, false, 1, 256, 1, 1, 8, "kinetics.g16c8.mixed.onelaunch.b256"),
    RD_GPERS8(2, GroupKinetics, 0, double, 1, 3, 4, "kinetics.g16c8.fp64.persistent.b256.w3.fs4"),
    RD_GPERS8(2, GroupKinetics, 1, float, 1, 4, 4, "kinetics.g16c8.mixed.persistent.b256.w4.fs4"),
    RD_GPERS8(2, GroupKinetics, 0, double, 2, 2, 4, "kinetics.g16c8.fp64.persistent.b256.w2.fs4"),
    RD_GPERS8(2, GroupKinetics, 1, float, 2, 3, 4, "kinetics.g16c8.mixed.persistent.b256.w3.fs4"),
    RD_GPERS8(2, GroupKinetics, 0, double, 3, 4, 4, "kinetics.g16c8.fp64.persistent.b256.w4.fs4"),
    RD_GPERS8(2, GroupKinetics, 1, float, 3, 3, 2, "kinetics.g16c8.mixed.persistent.b256.w3.fs2"),
    RD_GPERS_C(2, GroupKinetics, 0, double, 6, 256, 3, 4, 8, "kinetics.g16c8.fp64.persistent.b256.w3.fs4.cold"),
    RD_GPERS_C(2, GroupKinetics, 0, double, 7, 256, 4, 4, 8, "kinetics.g16c8.fp64.persistent.b256.w4.fs4.cold"),
    RD_GPERS_C(2, GroupKinetics, 1, float, 5, 256, 4, 4, 8, "kinetics.g16c8.mixed.persistent.b256.w4.fs4.cold"),
    RD_GPERS8(2, GroupKinetics, 0, double, 4, 3, 2, "kinetics.g16c8.fp64.persistent.b256.w3.fs2"),
    RD_GPERS_X(2, GroupKinetics, 0, double, false, 5, 256, 3, 4, false, 8,
               "kinetics.g16c8.fp64.persistent.b256.w3.fs4.unfused"),
    RD_GPERS_X(2, GroupKinetics, 1, float, false, 4, 256, 3, 4, false, 8,
               "kinetics.g16c8.mixed.persistent.b256.w3.fs4.unfused"),
    RD_GONE_X(2, GroupKinetics, 0, double, true, 1, 256, 1, 1, 8, "kinetics.g16c8.fp64.onelaunch.fixed"),
    RD_GPERS_X(2, GroupKinetics, 0, double, true, 1, 256, 1, 1, true, 8,
               "kinetics.g16c8.fp64.persistent.fixed"),
    RD_GONE(4, GroupLinear, 0, double, false, 1, 256, 1, 1, "linear.g16.fp64.onelaunch.b256"),
    RD_GONE(4, GroupLinear, 1, float, false, 1, 256, 1, 1, "linear.g16.mixed.onelaunch.b256"),
    RD_GPERS(4, GroupLinear, 0, double, false, 1, 256, 2, 4, "linear.g16.fp64.persistent.b256.w2.fs4"),
    RD_GPERS(4, GroupLinear, 1, float, false, 1, 256, 3, 4, "linear.g16.mixed.persistent.b256.w3.fs4"),
    RD_GPERS_X(4, GroupLinear, 0, double, false, 2, 256, 2, 4, false, 16,
               "linear.g16.fp64.persistent.b256.w2.fs4.unfused"),
    RD_GONE(4, GroupLinear, 0, double, true, 1, 256, 1, 1, "linear.g16.fp64.onelaunch.fixed"),
    RD_GPERS(4, GroupLinear, 0, double, true, 1, 256, 1, 1, "linear.g16.fp64.persistent.fixed"),
    RD_GONE_X(4, GroupLinear, 0, double, false, 1, 256, 1, 1, 8, "linear.g16c8.fp64.onelaunch.b256"),
    RD_GONE_X(4, GroupLinear, 1, float, false, 1, 256, 1, 1, 8, "linear.g16c8.mixed.onelaunch.b256"),
    RD_GPERS8(4, GroupLinear, 0, double, 1, 3, 4, "linear.g16c8.fp64.persistent.b256.w3.fs4"),
    RD_GPERS8(4, GroupLinear, 1, float, 1, 4, 4, "linear.g16c8.mixed.persistent.b256.w4.fs4"),
    RD_GPERS_X(4, GroupLinear, 0, double, false, 2, 256, 3, 4, false, 8,
               "linear.g16c8.fp64.persistent.b256.w3.fs4.unfused"),
    RD_GONE_X(4, GroupLinear, 0, double, true, 1, 256, 1, 1, 8, "linear.g16c8.fp64.onelaunch.fixed"),
    RD_GPERS_X(4, GroupLinear, 0, double, true, 1, 256, 1, 1, true, 8,
               "linear.g16c8.fp64.persistent.fixed"),
};

const KernelEntry* group_kernel_table(int* count) {
    *count = (int)(sizeof(g_group_table) / sizeof(g_group_table[0]));
    return g_group_table;
}

}  // namespace rd

RD_PH_READER(rd_phase_read_group)
