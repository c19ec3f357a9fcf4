/*
 * rd_kernels_group.hip -- reaction-step kernels for larger systems, where a
 * group of lanes shares one cell.
 */
#include <hip/hip_runtime.h>

#include "rd_launch.h"

namespace rd {

const KernelEntry* group_kernel_table(int* count) {
    *count = 0;
    return nullptr;
}

}  // namespace rd
