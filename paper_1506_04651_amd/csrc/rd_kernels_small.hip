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

#include "rd_cell_small.h"
#include "rd_launch.h"

namespace rd {

/* One pass of the scheduling loop.  Lanes in PH_NEWTON take one Newton
 * iteration; a lane whose Newton loop ends moves to PH_END.  The step-end
 * block (error estimate, control) and the step-start block (Jacobian,
 * factorization, start values) together cost about three Newton iterations
 * and run with only the lanes that need them active, so they are batched:
 * they run once at least FSMIN lanes of the wave wait for them, or when no
 * lane is left iterating.  FSMIN = 1 runs them every pass.  Batching delays
 * individual lanes but never changes what a cell computes. */
template <class Model, typename LT, bool FIXED, int BLOCK, int FSMIN>
__device__ __forceinline__ void advance(SmallCell<Model, LT, BLOCK>& cell, const Model& md,
                                        const StepParams& P) {
    if (cell.phase == PH_NEWTON) {
        const int o = cell.newton(md, P);
        if (o != NW_CONTINUE) {
            cell.outcome = o;
            cell.phase = PH_END;
        }
    }
    const bool waits = cell.phase == PH_END || cell.phase == PH_START;
    if (FSMIN > 1) {
        const unsigned long long wmask = __ballot(waits);
        if (wmask == 0ull) return;
        if ((unsigned)__popcll(wmask) < (unsigned)FSMIN && __ballot(cell.phase == PH_NEWTON) != 0ull)
            return;
    }
    if (cell.phase == PH_END) cell.template finish<FIXED>(md, P, cell.outcome);
    if (cell.phase == PH_START) cell.template start<FIXED>(md, P);
}

template <class Model, typename LT, bool FIXED, int BLOCK, int WPE, int FSMIN>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
k_onelaunch(LaunchArgs a) {
    using L = SmallLds<Model::M>;
    __shared__ double sh[L::ROWS * BLOCK];
    __shared__ StepParams sP;
    stage_params(sP, a.P);
    const int64_t c = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (c >= a.n) return;
    const Model md(a.params);
    SmallCell<Model, LT, BLOCK> cell;
    cell.lds.base = sh + threadIdx.x;
    cell.load(md, sP, a.states, a.n, c);
    while (cell.phase != PH_IDLE) {
        __asm__ volatile("" ::: "memory"); /* re-read sP from LDS each pass */
        advance<Model, LT, FIXED, BLOCK, FSMIN>(cell, md, sP);
    }
    cell.store(a.states, a.stats, a.n, c);
    if (cell.status != ST_OK) atomicAdd(a.nfail, 1ull);
}

/* Claim queue of one wave: a range [next, end) of positions in the claim
 * order already reserved from the global counter.  Idle lanes take positions
 * from it in lane order; only when it runs dry does one lane reserve a new
 * chunk (at least kClaimChunk positions) with a single atomic. */
constexpr unsigned kClaimChunk = 16;

template <class Model, typename LT, bool FIXED, int BLOCK, int WPE, int FSMIN>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
k_persistent(LaunchArgs a) {
    using L = SmallLds<Model::M>;
    __shared__ double sh[L::ROWS * BLOCK];
    __shared__ StepParams sP;
    stage_params(sP, a.P);
    const Model md(a.params);
    SmallCell<Model, LT, BLOCK> cell;
    cell.lds.base = sh + threadIdx.x;
    cell.phase = PH_IDLE;
    cell.status = ST_OK;
    int64_t c = -1;
    bool alive = true;
    const unsigned lane = __lane_id();
    const unsigned long long below = (1ull << lane) - 1ull;
    unsigned long long qnext = 0, qend = 0; /* wave-uniform */
    for (;;) {
        const bool need = alive && cell.phase == PH_IDLE;
        if (need && c >= 0) {
            cell.store(a.states, a.stats, a.n, c);
            if (cell.status != ST_OK) atomicAdd(a.nfail, 1ull);
            c = -1;
        }
        const unsigned long long mask = __ballot(need);
        if (mask) {
            const unsigned cnt = (unsigned)__popcll(mask);
            const unsigned rank = (unsigned)__popcll(mask & below);
            const unsigned long long avail = qend - qnext;
            unsigned long long pos;
            if (avail >= cnt) {
                pos = qnext + rank;
                qnext += cnt;
            } else {
                const unsigned take = (cnt - (unsigned)avail) > kClaimChunk
                                          ? cnt - (unsigned)avail : kClaimChunk;
                const int leader = __ffsll((long long)mask) - 1;
                unsigned long long base = 0;
                if (lane == (unsigned)leader) base = atomicAdd(a.counter, (unsigned long long)take);
                base = __shfl(base, leader);
                pos = rank < avail ? qnext + rank : base + (rank - avail);
                qnext = base + (cnt - avail);
                qend = base + take;
            }
            if (need) {
                if (pos < (unsigned long long)a.n) {
                    c = a.order ? (int64_t)a.order[pos] : (int64_t)pos;
                    cell.load(md, sP, a.states, a.n, c);
                } else {
                    alive = false;
                }
            }
        }
        if (__ballot(alive) == 0ull) break;
        __asm__ volatile("" ::: "memory"); /* re-read sP from LDS each pass */
        advance<Model, LT, FIXED, BLOCK, FSMIN>(cell, md, sP);
    }
}

__global__ void k_reset(unsigned long long* p, int n) {
    const int i = threadIdx.x;
    if (i < n) p[i] = 0ull;
}

hipError_t launch_reset(unsigned long long* p, int n, hipStream_t s) {
    hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

template <class Model, typename LT, bool FIXED, int BLOCK, int WPE, int FSMIN>
hipError_t launch_one(const LaunchArgs& a, int grid, hipStream_t s) {
    if (grid <= 0) grid = (int)((a.n + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL((k_onelaunch<Model, LT, FIXED, BLOCK, WPE, FSMIN>), dim3(grid), dim3(BLOCK), 0,
                       s, a);
    return hipGetLastError();
}

template <class Model, typename LT, bool FIXED, int BLOCK, int WPE, int FSMIN>
hipError_t launch_pers(const LaunchArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_persistent<Model, LT, FIXED, BLOCK, WPE, FSMIN>), dim3(grid), dim3(BLOCK), 0,
                       s, a);
    return hipGetLastError();
}

#define RD_ONE(KIND, MODEL, M, PREC, LT, FIXED, VAR, BLOCK, WPE, FS, NAME)                       \
    {KIND, M, PREC, 1, FIXED, VAR, BLOCK, BLOCK, NAME,                                          \
     &launch_one<MODEL, LT, FIXED, BLOCK, WPE, FS>,                                             \
     (const void*)&k_onelaunch<MODEL, LT, FIXED, BLOCK, WPE, FS>}
#define RD_PERS(KIND, MODEL, M, PREC, LT, FIXED, VAR, BLOCK, WPE, FS, NAME)                      \
    {KIND, M, PREC, 0, FIXED, VAR, BLOCK, BLOCK, NAME,                                          \
     &launch_pers<MODEL, LT, FIXED, BLOCK, WPE, FS>,                                            \
     (const void*)&k_persistent<MODEL, LT, FIXED, BLOCK, WPE, FS>}

/* model kinds (same numbering as the public header) */
enum { K_OREG = 1, K_KIN = 2, K_NAG = 3, K_LIN = 4, K_ROB = 5 };

#define RD_MODEL_SET(KIND, MODEL, M, TAG)                                                     \
    RD_ONE(KIND, MODEL, M, 0, double, false, 1, 256, 1, 32, TAG ".fp64.onelaunch.b256.fs32"), \
    RD_ONE(KIND, MODEL, M, 1, float, false, 1, 256, 1, 32, TAG ".mixed.onelaunch.b256.fs32"), \
    RD_PERS(KIND, MODEL, M, 0, double, false, 1, 128, 1, 40, TAG ".fp64.persistent.b128.fs40"), \
    RD_PERS(KIND, MODEL, M, 1, float, false, 1, 128, 1, 40, TAG ".mixed.persistent.b128.fs40"), \
    RD_ONE(KIND, MODEL, M, 0, double, true, 1, 256, 1, 1, TAG ".fp64.onelaunch.fixed"),       \
    RD_PERS(KIND, MODEL, M, 0, double, true, 1, 256, 1, 1, TAG ".fp64.persistent.fixed")

#define RD_TUNE_SET(KIND, MODEL, M, PREC, LT, TAG)                                            \
    RD_PERS(KIND, MODEL, M, PREC, LT, false, 2, 128, 1, 1, TAG ".persistent.b128.fs1"),       \
    RD_PERS(KIND, MODEL, M, PREC, LT, false, 3, 128, 1, 24, TAG ".persistent.b128.fs24"),     \
    RD_PERS(KIND, MODEL, M, PREC, LT, false, 4, 128, 1, 32, TAG ".persistent.b128.fs32"),     \
    RD_PERS(KIND, MODEL, M, PREC, LT, false, 5, 128, 1, 48, TAG ".persistent.b128.fs48"),     \
    RD_PERS(KIND, MODEL, M, PREC, LT, false, 6, 128, 1, 56, TAG ".persistent.b128.fs56"),     \
    RD_PERS(KIND, MODEL, M, PREC, LT, false, 7, 256, 1, 40, TAG ".persistent.b256.fs40"),     \
    RD_PERS(KIND, MODEL, M, PREC, LT, false, 8, 64, 1, 40, TAG ".persistent.b64.fs40"),       \
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
    RD_MODEL_SET(K_LIN, Linear<3>, 3, "linear3"),
    RD_MODEL_SET(K_LIN, Linear<4>, 4, "linear4"),
    RD_MODEL_SET(K_KIN, Kinetics<1>, 1, "kinetics1"),
    RD_MODEL_SET(K_KIN, Kinetics<2>, 2, "kinetics2"),
    RD_MODEL_SET(K_KIN, Kinetics<3>, 3, "kinetics3"),
    RD_MODEL_SET(K_KIN, Kinetics<4>, 4, "kinetics4"),
};

const KernelEntry* small_kernel_table(int* count) {
    *count = (int)(sizeof(g_small_table) / sizeof(g_small_table[0]));
    return g_small_table;
}

}  // namespace rd
