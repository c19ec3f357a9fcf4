/*
 * rd_phase.h -- optional per-phase cycle accounting of the persistent kernels,
 * for diagnostic builds only: compiled in with -DRD_PHASE_PROFILE (see
 * build.build_phase_profile and phase_profile.py), empty otherwise, so the
 * product kernels are unchanged by it.
 *
 * Every wave accumulates, per phase, the shader-clock cycles between the
 * phase's start and its end, the lanes active at its end and the number of
 * times it ran, in LDS; at the end of the kernel it adds its totals to a
 * device array that rd_phase_read_small / rd_phase_read_group return.  The
 * cycles are the wave's own elapsed time, so phases in which the wave waits
 * (on memory, or for issue while other waves of its SIMD run) count fully.
 */
#pragma once
#include <hip/hip_runtime.h>

namespace rd {
enum : int { PHASE_NEWTON = 0, PHASE_FINISH, PHASE_START, PHASE_FACTOR, PHASE_CLAIM, PHASE_KERNEL,
             PHASE_N };
constexpr int kPhaseWords = 3 * PHASE_N; /* cycles, active lanes, executions */
}  // namespace rd

#ifdef RD_PHASE_PROFILE
namespace rd {
static __shared__ unsigned long long rd_phase_wave[4][kPhaseWords]; /* up to 4 waves per block */
static __device__ unsigned long long rd_phase_total[kPhaseWords];
__device__ __forceinline__ void phase_add(unsigned long long t0, int slot) {
    const unsigned long long d = __builtin_readcyclecounter() - t0;
    const unsigned long long act = __ballot(1);
    if (__lane_id() == (unsigned)(__ffsll((long long)act) - 1)) {
        unsigned long long* w = rd_phase_wave[(threadIdx.x >> 6) & 3];
        w[slot] += d;
        w[PHASE_N + slot] += (unsigned long long)__popcll(act);
        w[2 * PHASE_N + slot] += 1ull;
    }
}
}  // namespace rd
#define RD_PH_BEGIN(v) const unsigned long long v = __builtin_readcyclecounter();
#define RD_PH_END(v, slot) ::rd::phase_add((v), (slot))
#define RD_PH_KERNEL_BEGIN(v)                                                                 \
    if (__lane_id() < (unsigned)::rd::kPhaseWords)                                          \
        ::rd::rd_phase_wave[(threadIdx.x >> 6) & 3][__lane_id()] = 0ull;                    \
    RD_PH_BEGIN(v)
#define RD_PH_KERNEL_END(v)                                                                   \
    do {                                                                                      \
        RD_PH_END(v, ::rd::PHASE_KERNEL);                                                     \
        if (__lane_id() < (unsigned)::rd::kPhaseWords)                                      \
            atomicAdd(&::rd::rd_phase_total[__lane_id()],                                   \
                      ::rd::rd_phase_wave[(threadIdx.x >> 6) & 3][__lane_id()]);            \
    } while (0)
/* reader of this translation unit's totals (optionally clearing them) */
#define RD_PH_READER(NAME)                                                                    \
    extern "C" int NAME(unsigned long long* out, int clear) {                               \
        if (hipMemcpyFromSymbol(out, HIP_SYMBOL(::rd::rd_phase_total),                       \
                                sizeof(unsigned long long) * ::rd::kPhaseWords) != hipSuccess) \
            return -1;                                                                        \
        if (clear) {                                                                          \
            unsigned long long z[::rd::kPhaseWords] = {0};                                   \
            if (hipMemcpyToSymbol(HIP_SYMBOL(::rd::rd_phase_total), z, sizeof(z)) != hipSuccess) \
                return -1;                                                                    \
        }                                                                                     \
        return 0;                                                                             \
    }
#else
#define RD_PH_BEGIN(v)
#define RD_PH_END(v, slot) ((void)0)
#define RD_PH_KERNEL_BEGIN(v)
#define RD_PH_KERNEL_END(v) ((void)0)
#define RD_PH_READER(NAME)
#endif
