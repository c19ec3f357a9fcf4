/*
 * rd_kernels_group_fd.hip -- 16-lane-group kernels (5 <= m <= 16) whose
 * Jacobian is taken by forward differences: the kinetics model run with the
 * numerical Jacobian (the paper's STROKE runs take theirs numerically, §4 /
 * Appendix A) and the bytecode model (f supplied at run time as a register
 * program), which has no analytic Jacobian.  Each Jacobian costs m more f
 * evaluations, counted in nfev; the rows of J are kept in LDS.  The 8-column
 * kernels are registered under m = 8 (m = 5..8), the 16-column ones under
 * m = 16 (m = 9..16).
 */
#include <hip/hip_runtime.h>

#include "rd_group_kernels.h"

namespace rd {

using GroupKineticsFd = GroupFd<GroupKinetics>;

#define RD_GFD_SET(KIND, MODEL, TAG)                                                                \
    RD_GONE(KIND, MODEL, 0, double, false, 1, 256, 1, 1, TAG ".g16.fp64.onelaunch.b256"),            \
    RD_GONE(KIND, MODEL, 1, float, false, 1, 256, 1, 1, TAG ".g16.mixed.onelaunch.b256"),             \
    RD_GPERS(KIND, MODEL, 0, double, false, 1, 256, 2, 4, TAG ".g16.fp64.persistent.b256.w2.fs4"),   \
    RD_GPERS(KIND, MODEL, 1, float, false, 1, 256, 3, 4, TAG ".g16.mixed.persistent.b256.w3.fs4"),   \
    RD_GONE_X(KIND, MODEL, 0, double, false, 1, 256, 1, 1, 8, TAG ".g16c8.fp64.onelaunch.b256"),     \
    RD_GONE_X(KIND, MODEL, 1, float, false, 1, 256, 1, 1, 8, TAG ".g16c8.mixed.onelaunch.b256"),      \
    RD_GPERS8(KIND, MODEL, 0, double, 1, 3, 4, TAG ".g16c8.fp64.persistent.b256.w3.fs4"),            \
    RD_GPERS8(KIND, MODEL, 1, float, 1, 4, 4, TAG ".g16c8.mixed.persistent.b256.w4.fs4")

static const KernelEntry g_group_fd_table[] = {
    RD_GFD_SET(2, GroupKineticsFd, "kinetics.fdjac"),
    RD_GFD_SET(6, GroupBytecode, "bytecode"),
    /* fixed-step test mode of the bytecode model */
    RD_GONE(6, GroupBytecode, 0, double, true, 1, 256, 1, 1, "bytecode.g16.fp64.onelaunch.fixed"),
    RD_GPERS(6, GroupBytecode, 0, double, true, 1, 256, 1, 1, "bytecode.g16.fp64.persistent.fixed"),
    RD_GONE_X(6, GroupBytecode, 0, double, true, 1, 256, 1, 1, 8, "bytecode.g16c8.fp64.onelaunch.fixed"),
    RD_GPERS_X(6, GroupBytecode, 0, double, true, 1, 256, 1, 1, true, 8,
               "bytecode.g16c8.fp64.persistent.fixed"),
};

const KernelEntry* group_fd_kernel_table(int* count) {
    *count = (int)(sizeof(g_group_fd_table) / sizeof(g_group_fd_table[0]));
    return g_group_fd_table;
}

}  // namespace rd
