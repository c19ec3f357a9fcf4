/*
 * rd_kernels_group.hip -- reaction-step kernels for 5 <= m <= 16 (the
 * synthetic stiff kinetics and linear test models): a 16-lane group of a
 * wave64 shares one cell, four cells per wave.
 *
 * Schedules as for one-lane cells: one launch per batch (a group owns one
 * cell), or persistent work stealing in which an idle group claims the next
 * position of the claim order through its wave's claim queue.  The step-end /
 * step-start block is batched across the wave's groups (at least FSMIN groups
 * waiting, or no group left iterating), which changes when a cell advances,
 * never what it computes.
 */
#include <hip/hip_runtime.h>

#include "rd_cell_group.h"
#include "rd_launch.h"

namespace rd {

constexpr unsigned kGroupClaimChunk = 4; /* cells */

/* Model rows into LDS, zero padded to 16 x 16 (K then G per row). */
template <class Model>
__device__ __forceinline__ void load_table(double* tab, const double* __restrict__ p, int m, int block) {
    for (int i = threadIdx.x; i < GroupTable::DOUBLES; i += block) {
        const int row = i / GroupTable::STRIDE, col = i % GroupTable::STRIDE;
        double v = 0.0;
        if (row < m) {
            if (col < m) v = p[row * m + col];
            else if (Model::HAS_G && col >= kGroup && col < kGroup + m) v = p[m * m + row * m + (col - kGroup)];
        }
        tab[i] = v;
    }
    __syncthreads();
}

template <class Cell>
__device__ __forceinline__ void init_cell(Cell& cell, const double* tab, int m) {
    cell.q = (int)grp_lane();
    cell.m = m;
    cell.act = cell.q < m;
    cell.inv3m = 1.0 / (3.0 * m);
    cell.invm = 1.0 / m;
    cell.kg = tab + cell.q * GroupTable::STRIDE;
    cell.phase = PH_IDLE;
    cell.status = ST_OK;
    cell.uJ = cell.gJ = 0.0;
}

template <bool FIXED, int FSMIN, class Cell>
__device__ __forceinline__ void advance_group(Cell& cell, const StepParams& P) {
    /* keep the LDS table reads inside the loop (no hoisting into registers) */
    /* keep the LDS model rows out of registers: they are re-read, not hoisted */
    __asm__ volatile("" ::: "memory");
    if (cell.phase == PH_NEWTON) {
        const int o = cell.newton(P);
        if (o != NW_CONTINUE) {
            cell.outcome = o;
            cell.phase = PH_END;
        }
    }
    const bool waits = cell.phase == PH_END || cell.phase == PH_START;
    if (FSMIN > 1) {
        const unsigned long long wmask = __ballot(waits);
        if (wmask == 0ull) return;
        if ((unsigned)__popcll(wmask) < (unsigned)(FSMIN * kGroup) &&
            __ballot(cell.phase == PH_NEWTON) != 0ull)
            return;
    }
    if (cell.phase == PH_END) cell.template finish<FIXED>(P, cell.outcome);
    if (cell.phase == PH_START) cell.template start<FIXED>(P);
}

template <class Model, typename LT, bool FIXED, int BLOCK, int WPE, int FSMIN, bool FUSE, int NC>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
k_group_onelaunch(LaunchArgs a, int m) {
    __shared__ double tab[GroupTable::DOUBLES];
    __shared__ StepParams sP;
    stage_params(sP, a.P);
    load_table<Model>(tab, a.params, m, BLOCK);
    const int64_t c = (int64_t)blockIdx.x * (BLOCK / kGroup) + threadIdx.x / kGroup;
    if (c >= a.n) return;
    GroupCell<Model, LT, FUSE, NC> cell;
    init_cell(cell, tab, m);
    cell.load(sP, a.states, a.n, c, a.hcell);
    while (cell.phase != PH_IDLE) advance_group<FIXED, FSMIN>(cell, sP);
    cell.store(a.states, a.stats, a.n, c, a.hcell);
    if (cell.status != ST_OK && cell.q == 0) atomicAdd(a.nfail, 1ull);
}

template <class Model, typename LT, bool FIXED, int BLOCK, int WPE, int FSMIN, bool FUSE, int NC>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
k_group_persistent(LaunchArgs a, int m) {
    __shared__ double tab[GroupTable::DOUBLES];
    __shared__ StepParams sP;
    stage_params(sP, a.P);
    load_table<Model>(tab, a.params, m, BLOCK);
    GroupCell<Model, LT, FUSE, NC> cell;
    init_cell(cell, tab, m);
    int64_t c = -1;
    bool alive = true;
    const unsigned lane = __lane_id();
    const unsigned long long below = (1ull << lane) - 1ull;
    unsigned long long qnext = 0, qend = 0; /* wave-uniform claim queue, in cells */
    for (;;) {
        const bool need = alive && cell.phase == PH_IDLE; /* group-uniform */
        if (need && c >= 0) {
            cell.store(a.states, a.stats, a.n, c, a.hcell);
            if (cell.status != ST_OK && cell.q == 0) atomicAdd(a.nfail, 1ull);
            c = -1;
        }
        const unsigned long long mask = __ballot(need);
        if (mask) {
            const unsigned cnt = (unsigned)__popcll(mask) / kGroup;
            const unsigned rank = (unsigned)__popcll(mask & below) / kGroup;
            const unsigned long long avail = qend - qnext;
            unsigned long long pos;
            if (avail >= cnt) {
                pos = qnext + rank;
                qnext += cnt;
            } else {
                const unsigned take = (cnt - (unsigned)avail) > kGroupClaimChunk
                                          ? cnt - (unsigned)avail : kGroupClaimChunk;
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
                    cell.load(sP, a.states, a.n, c, a.hcell);
                } else {
                    alive = false;
                }
            }
        }
        if (__ballot(alive) == 0ull) break;
        advance_group<FIXED, FSMIN>(cell, sP);
    }
}

/* the species count travels in StepParams::m */
template <class Model, typename LT, bool FIXED, int BLOCK, int WPE, int FSMIN, bool FUSE, int NC>
hipError_t launch_group_one(const LaunchArgs& a, int grid, hipStream_t s) {
    constexpr int cells = BLOCK / kGroup;
    if (grid <= 0) grid = (int)((a.n + cells - 1) / cells);
    hipLaunchKernelGGL((k_group_onelaunch<Model, LT, FIXED, BLOCK, WPE, FSMIN, FUSE, NC>), dim3(grid),
                       dim3(BLOCK), 0, s, a, (int)a.P.m);
    return hipGetLastError();
}

template <class Model, typename LT, bool FIXED, int BLOCK, int WPE, int FSMIN, bool FUSE, int NC>
hipError_t launch_group_pers(const LaunchArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_group_persistent<Model, LT, FIXED, BLOCK, WPE, FSMIN, FUSE, NC>), dim3(grid),
                       dim3(BLOCK), 0, s, a, (int)a.P.m);
    return hipGetLastError();
}

/* FUSE: broadcasts fused into the multiply-adds (rd_group_fused.h), in FP64
 * and, for the mixed kernels' factors and solves, in FP32.  NC: columns per
 * lane; the 8-column kernels are registered under m = 8 and serve m = 5..8,
 * the 16-column ones under m = 16 for m = 9..16. */
#define RD_GONE_X(KIND, MODEL, PREC, LT, FIXED, VAR, BLOCK, WPE, FS, NC, NAME)                    \
    {KIND, 0, NC, PREC, 1, FIXED, VAR, BLOCK, BLOCK / kGroup, NAME,                                 \
     &launch_group_one<MODEL, LT, FIXED, BLOCK, WPE, FS, true, NC>,                              \
     (const void*)&k_group_onelaunch<MODEL, LT, FIXED, BLOCK, WPE, FS, true, NC>}
#define RD_GPERS_X(KIND, MODEL, PREC, LT, FIXED, VAR, BLOCK, WPE, FS, FUSE, NC, NAME)             \
    {KIND, 0, NC, PREC, 0, FIXED, VAR, BLOCK, BLOCK / kGroup, NAME,                                 \
     &launch_group_pers<MODEL, LT, FIXED, BLOCK, WPE, FS, FUSE, NC>,                             \
     (const void*)&k_group_persistent<MODEL, LT, FIXED, BLOCK, WPE, FS, FUSE, NC>}
#define RD_GONE(KIND, MODEL, PREC, LT, FIXED, VAR, BLOCK, WPE, FS, NAME)                          \
    RD_GONE_X(KIND, MODEL, PREC, LT, FIXED, VAR, BLOCK, WPE, FS, 16, NAME)
#define RD_GPERS(KIND, MODEL, PREC, LT, FIXED, VAR, BLOCK, WPE, FS, NAME)                         \
    RD_GPERS_X(KIND, MODEL, PREC, LT, FIXED, VAR, BLOCK, WPE, FS, true, 16, NAME)
#define RD_GPERS8(KIND, MODEL, PREC, LT, VAR, WPE, FS, NAME)                                      \
    RD_GPERS_X(KIND, MODEL, PREC, LT, false, VAR, 256, WPE, FS, true, 8, NAME)

static const KernelEntry g_group_table[] = {
    RD_GONE(2, GroupKinetics, 0, double, false, 1, 256, 1, 1, "kinetics.g16.fp64.onelaunch.b256"),
    RD_GONE(2, GroupKinetics, 1, float, false, 1, 256, 1, 1, "kinetics.g16.mixed.onelaunch.b256"),
    RD_GPERS(2, GroupKinetics, 0, double, false, 1, 256, 2, 4, "kinetics.g16.fp64.persistent.b256.w2.fs4"),
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
