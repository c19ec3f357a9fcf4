/*
 * rd_small_kernels.h -- kernel templates with one cell per lane (m <= 4):
 * the scheduling-loop pass, the one-launch and the persistent work-stealing
 * kernels, their launchers and the kernel-table entry macros.  Included by
 * the translation units that instantiate them for the models.
 */
#pragma once
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
                                        const StepParams& P, int fsmin = FSMIN) {
    if (cell.phase == PH_NEWTON) {
        RD_PH_BEGIN(ph_n)
        const int o = cell.newton(md, P);
        RD_PH_END(ph_n, PHASE_NEWTON);
        if (o != NW_CONTINUE) {
            cell.outcome = o;
            cell.phase = PH_END;
        }
    }
    const bool waits = cell.phase == PH_END || cell.phase == PH_START;
    if (FSMIN > 1) {
        const unsigned long long wmask = __ballot(waits);
        if (wmask == 0ull) return;
        if ((unsigned)__popcll(wmask) < (unsigned)fsmin && __ballot(cell.phase == PH_NEWTON) != 0ull)
            return;
    }
    if (cell.phase == PH_END) {
        RD_PH_BEGIN(ph_e)
        cell.template finish<FIXED>(md, P, cell.outcome);
        RD_PH_END(ph_e, PHASE_FINISH);
    }
    if (cell.phase == PH_START) {
        RD_PH_BEGIN(ph_s)
        cell.template start<FIXED>(md, P);
        RD_PH_END(ph_s, PHASE_START);
    }
}

template <class Model, typename LT, bool FIXED, int BLOCK, int WPE, int FSMIN>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
k_onelaunch(LaunchArgs a) {
    using L = SmallLds<Model::M>;
    __shared__ double sh[L::ROWS * BLOCK];
    __shared__ int shi[L::IROWS * BLOCK];
    __shared__ StepParams sP;
    stage_params(sP, a.P);
    const int64_t c = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
    if (c >= a.n) return;
    const Model md(a.params);
    SmallCell<Model, LT, BLOCK> cell;
    cell.lds.base = sh + threadIdx.x;
    cell.ilds.base = shi + threadIdx.x;
    cell.load(md, sP, a.states, a.n, c, a.hcell);
    while (cell.phase != PH_IDLE) {
        __asm__ volatile("" ::: "memory"); /* re-read sP from LDS each pass */
        advance<Model, LT, FIXED, BLOCK, FSMIN>(cell, md, sP);
    }
    cell.store(a.states, a.stats, a.n, c, a.hcell);
    if (cell.status != ST_OK) atomicAdd(a.nfail, 1ull);
}

/* Claim queue of one wave: a range [next, end) of positions in the claim
 * order already reserved from the global counter.  Idle lanes take positions
 * from it in lane order; only when it runs dry does one lane reserve a new
 * chunk (at least kClaimChunk positions) with a single atomic. */
constexpr unsigned kClaimChunk = 16;

/* Issue priority of a wave from the claim positions of the cells it holds.
 * Under the longest-first order a small position means an expensive cell,
 * and the launch cannot end before its most expensive cells do; waves holding
 * such cells get the SIMD first, and the waves with cheap cells fill the
 * cycles in which the former stall.  span = lanes of the grid / PDIV:
 * priority 3 for a wave holding a position below span, 2 below 2 span, 1
 * below 3 span, else 0.  Priorities only arbitrate instruction issue between
 * ready waves; they change no result. */
template <int PDIV>
__device__ __forceinline__ int claim_priority(unsigned long long held, unsigned long long lanes) {
    const unsigned long long span = (lanes + PDIV - 1) / PDIV;
    if (__ballot(held < span)) { __builtin_amdgcn_s_setprio(3); return 3; }
    if (__ballot(held < 2 * span)) { __builtin_amdgcn_s_setprio(2); return 2; }
    if (__ballot(held < 3 * span)) { __builtin_amdgcn_s_setprio(1); return 1; }
    __builtin_amdgcn_s_setprio(0);
    return 0;
}

/* CMIN > 1: a wave claims new cells only once at least CMIN of its lanes are
 * idle, or none is left working; each claim round waits for the loads of the
 * claimed cells, so fewer, larger rounds trade that latency against the
 * passes an idle lane waits.  Changes when a cell starts, never its result.
 * PLDS: the step parameters are staged in LDS and re-read each pass (true),
 * or read from the kernel arguments, where the compiler keeps them in scalar
 * registers across the loop (false).  Same arithmetic either way.  PDIV > 0:
 * wave issue priorities from claim positions (claim_priority).  Step-end
 * batching threshold of a wave: FSL during its first claim round (every lane
 * started its cell in the same pass, and the claim order put cells of
 * similar cost side by side, so the lanes stay nearly in phase and waiting
 * for all of them costs little), then FSU while the wave holds cells at the
 * top priority, else FSMIN. */
template <class Model, typename LT, bool FIXED, int BLOCK, int WPE, int FSMIN, bool PLDS = true,
          int PDIV = 0, int FSU = FSMIN, int FSL = FSMIN, bool AOS = false, int CMIN = 1>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
k_persistent(LaunchArgs a) {
    using L = SmallLds<Model::M>;
    /* LDS layout of the per-lane slots: [rows][lanes] (lane columns), or
     * with AOS [lanes][rows] (lane rows, odd row count) */
    constexpr int RS = AOS ? 1 : BLOCK;
    __shared__ double sh[(AOS ? L::ROWS_AOS : L::ROWS) * BLOCK];
    __shared__ int shi[(AOS ? L::IROWS_AOS : L::IROWS) * BLOCK];
    __shared__ StepParams sPl;
    if (PLDS) stage_params(sPl, a.P);
    const StepParams& sP = PLDS ? sPl : a.P;
    const Model md(a.params);
    SmallCell<Model, LT, RS> cell;
    cell.lds.base = sh + (AOS ? threadIdx.x * L::ROWS_AOS : threadIdx.x);
    cell.ilds.base = shi + (AOS ? threadIdx.x * L::IROWS_AOS : threadIdx.x);
    cell.phase = PH_IDLE;
    cell.status = ST_OK;
    int64_t c = -1;
    bool alive = true;
    const unsigned lane = __lane_id();
    const unsigned long long below = (1ull << lane) - 1ull;
    unsigned long long qnext = 0, qend = 0; /* wave-uniform */
    unsigned long long held = ~0ull;         /* claim position of the cell held */
    int fs = FSL;                            /* wave-uniform step-end batching threshold */
    int claims = 0;                          /* claim rounds of the wave so far */
    RD_PH_KERNEL_BEGIN(ph_k)
    for (;;) {
        RD_PH_BEGIN(ph_c)
        const bool need = alive && cell.phase == PH_IDLE;
        if (need && c >= 0) {
            cell.store(a.states, a.stats, a.n, c, a.hcell);
            if (cell.status != ST_OK) atomicAdd(a.nfail, 1ull);
            c = -1;
            held = ~0ull;
        }
        const unsigned long long mask = __ballot(need);
        bool claim = mask != 0ull;
        if (CMIN > 1 && claim && (unsigned)__popcll(mask) < (unsigned)CMIN)
            claim = __ballot(alive && cell.phase != PH_IDLE) == 0ull;
        if (claim) {
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
                    held = pos;
                    cell.load(md, sP, a.states, a.n, c, a.hcell);
                } else {
                    alive = false;
                }
            }
            const int prio =
                PDIV > 0 ? claim_priority<PDIV>(held, (unsigned long long)gridDim.x * BLOCK) : 0;
            if (FSU != FSMIN || FSL != FSMIN) {
                ++claims;
                fs = claims == 1 ? FSL : (prio == 3 ? FSU : FSMIN);
            }
        }
        RD_PH_END(ph_c, PHASE_CLAIM);
        if (__ballot(alive) == 0ull) break;
        if (PLDS) __asm__ volatile("" ::: "memory"); /* re-read sP from LDS each pass */
        advance<Model, LT, FIXED, RS, FSMIN>(cell, md, sP, fs);
    }
    RD_PH_KERNEL_END(ph_k);
}

template <class Model, typename LT, bool FIXED, int BLOCK, int WPE, int FSMIN>
hipError_t launch_one(const LaunchArgs& a, int grid, hipStream_t s) {
    if (grid <= 0) grid = (int)((a.n + BLOCK - 1) / BLOCK);
    hipLaunchKernelGGL((k_onelaunch<Model, LT, FIXED, BLOCK, WPE, FSMIN>), dim3(grid), dim3(BLOCK), 0,
                       s, a);
    return hipGetLastError();
}

template <class Model, typename LT, bool FIXED, int BLOCK, int WPE, int FSMIN, bool PLDS = true,
          int PDIV = 0, int FSU = FSMIN, int FSL = FSMIN, bool AOS = false, int CMIN = 1>
hipError_t launch_pers(const LaunchArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_persistent<Model, LT, FIXED, BLOCK, WPE, FSMIN, PLDS, PDIV, FSU, FSL, AOS, CMIN>),
                       dim3(grid), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

#define RD_ONE(KIND, MODEL, M, PREC, LT, FIXED, VAR, BLOCK, WPE, FS, NAME)                       \
    {KIND, fd_jac_of<MODEL>::value ? 1 : 0, M, PREC, 1, FIXED, VAR, BLOCK, BLOCK, NAME,                                          \
     &launch_one<MODEL, LT, FIXED, BLOCK, WPE, FS>,                                             \
     (const void*)&k_onelaunch<MODEL, LT, FIXED, BLOCK, WPE, FS>}
#define RD_PERS_K(KIND, MODEL, M, PREC, LT, VAR, BLOCK, WPE, FS, NAME)                          \
    {KIND, fd_jac_of<MODEL>::value ? 1 : 0, M, PREC, 0, false, VAR, BLOCK, BLOCK, NAME,           \
     &launch_pers<MODEL, LT, false, BLOCK, WPE, FS, false>,                                     \
     (const void*)&k_persistent<MODEL, LT, false, BLOCK, WPE, FS, false>}
#define RD_PERS_P(KIND, MODEL, M, PREC, LT, VAR, BLOCK, WPE, FS, PDIV, NAME)                     \
    {KIND, fd_jac_of<MODEL>::value ? 1 : 0, M, PREC, 0, false, VAR, BLOCK, BLOCK, NAME,           \
     &launch_pers<MODEL, LT, false, BLOCK, WPE, FS, true, PDIV>,                                \
     (const void*)&k_persistent<MODEL, LT, false, BLOCK, WPE, FS, true, PDIV>}
#define RD_PERS_U(KIND, MODEL, M, PREC, LT, VAR, BLOCK, WPE, FS, PDIV, FSU, FSL, NAME)          \
    {KIND, fd_jac_of<MODEL>::value ? 1 : 0, M, PREC, 0, false, VAR, BLOCK, BLOCK, NAME,           \
     &launch_pers<MODEL, LT, false, BLOCK, WPE, FS, true, PDIV, FSU, FSL>,                      \
     (const void*)&k_persistent<MODEL, LT, false, BLOCK, WPE, FS, true, PDIV, FSU, FSL>}
#define RD_PERS_A(KIND, MODEL, M, PREC, LT, VAR, BLOCK, WPE, FS, PDIV, FSU, FSL, NAME)          \
    {KIND, fd_jac_of<MODEL>::value ? 1 : 0, M, PREC, 0, false, VAR, BLOCK, BLOCK, NAME,           \
     &launch_pers<MODEL, LT, false, BLOCK, WPE, FS, true, PDIV, FSU, FSL, true>,                \
     (const void*)&k_persistent<MODEL, LT, false, BLOCK, WPE, FS, true, PDIV, FSU, FSL, true>}
#define RD_PERS_C(KIND, MODEL, M, PREC, LT, VAR, BLOCK, WPE, FS, PDIV, FSU, FSL, CMIN, NAME)   \
    {KIND, fd_jac_of<MODEL>::value ? 1 : 0, M, PREC, 0, false, VAR, BLOCK, BLOCK, NAME,           \
     &launch_pers<MODEL, LT, false, BLOCK, WPE, FS, true, PDIV, FSU, FSL, false, CMIN>,         \
     (const void*)&k_persistent<MODEL, LT, false, BLOCK, WPE, FS, true, PDIV, FSU, FSL, false, CMIN>}
#define RD_PERS(KIND, MODEL, M, PREC, LT, FIXED, VAR, BLOCK, WPE, FS, NAME)                      \
    {KIND, fd_jac_of<MODEL>::value ? 1 : 0, M, PREC, 0, FIXED, VAR, BLOCK, BLOCK, NAME,                                          \
     &launch_pers<MODEL, LT, FIXED, BLOCK, WPE, FS>,                                            \
     (const void*)&k_persistent<MODEL, LT, FIXED, BLOCK, WPE, FS>}

/* model kinds (same numbering as the public header) */
enum { K_OREG = 1, K_KIN = 2, K_NAG = 3, K_LIN = 4, K_ROB = 5, K_BC = 6 };

#define RD_STR_(X) #X
#define RD_STR(X) RD_STR_(X)
/* the base kernels of a model; WPE: waves-per-SIMD target of the persistent
 * kernels (3 where the engine fits 168 registers with few spills, else 1);
 * the persistent kernels give waves that hold early claim positions (the
 * costliest cells under the longest-first order) a higher issue priority
 * (claim_priority with PDIV = 2), batch step ends at 48 waiting lanes,
 * or at all lanes while a wave still holds its first claims (its lanes then
 * started together on cells of similar cost) or holds the costliest cells,
 * and claim new cells in rounds of at least 28 idle lanes (CMIN) */
#define RD_MODEL_SET_W(KIND, MODEL, M, TAG, WPE)                                                      \
    RD_ONE(KIND, MODEL, M, 0, double, false, 1, 256, 1, 32, TAG ".fp64.onelaunch.b256.fs32"),        \
    RD_ONE(KIND, MODEL, M, 1, float, false, 1, 256, 1, 32, TAG ".mixed.onelaunch.b256.fs32"),         \
    RD_PERS_C(KIND, MODEL, M, 0, double, 1, 128, WPE, 48, 2, 64, 64, 28,                            \
              TAG ".fp64.persistent.b128.w" RD_STR(WPE) ".fs48.p2.u64.l64.c28"),                    \
    RD_PERS_C(KIND, MODEL, M, 1, float, 1, 128, WPE, 48, 2, 64, 64, 28,                             \
              TAG ".mixed.persistent.b128.w" RD_STR(WPE) ".fs48.p2.u64.l64.c28"),                   \
    RD_ONE(KIND, MODEL, M, 0, double, true, 1, 256, 1, 1, TAG ".fp64.onelaunch.fixed"),             \
    RD_PERS(KIND, MODEL, M, 0, double, true, 1, 256, 1, 1, TAG ".fp64.persistent.fixed")
#define RD_MODEL_SET(KIND, MODEL, M, TAG) RD_MODEL_SET_W(KIND, MODEL, M, TAG, 3)

}  // namespace rd
