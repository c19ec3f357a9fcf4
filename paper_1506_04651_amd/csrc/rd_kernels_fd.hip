/*
 * rd_kernels_fd.hip -- one-lane reaction-step kernels whose Jacobian is taken
 * by forward differences: the Oregonator run with the numerical Jacobian (the
 * paper's STROKE runs take their Jacobian numerically, §4 / Appendix A), and
 * the bytecode model (f supplied at run time as a register program, m <= 4),
 * which has no analytic Jacobian.  Same engine and schedules as the analytic
 * kernels; each Jacobian costs m more f evaluations, counted in nfev.
 */
#include <hip/hip_runtime.h>

#include "rd_small_kernels.h"

namespace rd {

static const KernelEntry g_fd_table[] = {
    RD_MODEL_SET(K_OREG, FdJac<Oregonator>, 3, "oregonator.fdjac"),
    RD_MODEL_SET(K_BC, Bytecode<1>, 1, "bytecode1"),
    RD_MODEL_SET(K_BC, Bytecode<2>, 2, "bytecode2"),
    RD_MODEL_SET(K_BC, Bytecode<3>, 3, "bytecode3"),
    RD_MODEL_SET(K_BC, Bytecode<4>, 4, "bytecode4"),
};

const KernelEntry* fd_kernel_table(int* count) {
    *count = (int)(sizeof(g_fd_table) / sizeof(g_fd_table[0]));
    return g_fd_table;
}

}  // namespace rd
