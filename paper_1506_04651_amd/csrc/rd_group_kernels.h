/*
 * rd_group_kernels.h -- kernel templates of the 16-lane-group engine
 * (5 <= m <= 16): a 16-lane group of a wave64 shares one cell, four cells per
 * wave.  The one-launch and persistent kernels, their launchers and the
 * kernel-table entry macros; included by the translation units that
 * instantiate them for the models.
 *
 * Schedules as for one-lane cells: one launch per batch (a group owns one
 * cell), or persistent work stealing in which an idle group claims the next
 * position of the claim order through its wave's claim queue.  The step-end /
 * step-start block is batched across the wave's groups (at least FSMIN groups
 * waiting, or no group left iterating), which changes when a cell advances,
 * never what it computes.
 */
#pragma once
#include <hip/hip_runtime.h>

#include "rd_cell_group.h"
#include "rd_launch.h"

namespace rd {

constexpr unsigned kGroupClaimChunk = 4; /* cells */

/* Model rows into LDS, zero padded to 16 x 16 (K then G per row), and 1/m,
 * 1/(3m) in the padding columns of every row; the bytecode model has no rows
 * (its program is read from the parameter block). */
template <class Model>
__device__ __forceinline__ void load_table(double* tab, const double* __restrict__ p, int m, int block) {
    for (int i = threadIdx.x; i < GroupTable::DOUBLES; i += block) {
        const int row = i / GroupTable::STRIDE, col = i % GroupTable::STRIDE;
        double v = 0.0;
        if (col == GroupTable::INVM) {
            v = 1.0 / m;
        } else if (col == GroupTable::INV3M) {
            v = 1.0 / (3.0 * m);
        } else if (!bytecode_of<Model>::value && row < m) {
            if (col < m) v = p[row * m + col];
            else if (Model::HAS_G && col >= kGroup && col < kGroup + m) v = p[m * m + row * m + (col - kGroup)];
        }
        tab[i] = v;
    }
    __syncthreads();
}

/* jfd: the block's LDS for forward-difference Jacobian rows, [16][BLOCK]
 * (lane t's row at column j is jfd[j * BLOCK + t]); unused otherwise. */
template <int BLOCK, class Cell>
__device__ __forceinline__ void init_cell(Cell& cell, const double* tab, double* jfd, double* cold,
                                          const double* params, int m) {
    cell.q = (int)grp_lane();
    cell.jl = jfd + threadIdx.x;
    cell.cl = cold + threadIdx.x;
    cell.jstride = BLOCK;
    cell.prog = params;
    cell.m = m;
    cell.act = cell.q < m;
    cell.kg = tab + cell.q * GroupTable::STRIDE;
    cell.phase = PH_IDLE;
    cell.status = ST_OK;
    cell.cv(Cell::C_UJ) = cell.cv(Cell::C_GJ) = 0.0;
}

template <bool FIXED, int FSMIN, class Cell>
__device__ __forceinline__ void advance_group(Cell& cell, const StepParams& P) {
    /* keep the LDS table reads inside the loop (no hoisting into registers) */
    /* keep the LDS model rows out of registers: they are re-read, not hoisted */
    __asm__ volatile("" ::: "memory");
    if (cell.phase == PH_NEWTON) {
        RD_PH_BEGIN(ph_n)
        const int o = cell.newton(P);
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
        if ((unsigned)__popcll(wmask) < (unsigned)(FSMIN * kGroup) &&
            __ballot(cell.phase == PH_NEWTON) != 0ull)
            return;
    }
    if (cell.phase == PH_END) {
        RD_PH_BEGIN(ph_e)
        cell.template finish<FIXED>(P, cell.outcome);
        RD_PH_END(ph_e, PHASE_FINISH);
    }
    if (cell.phase == PH_START) {
        RD_PH_BEGIN(ph_s)
        cell.template start<FIXED>(P);
        RD_PH_END(ph_s, PHASE_START);
    }
}

template <class Model, typename LT, bool FIXED, int BLOCK, int WPE, int FSMIN, bool FUSE, int NC,
          bool COLD = false>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
k_group_onelaunch(LaunchArgs a, int m) {
    __shared__ double tab[GroupTable::DOUBLES];
    __shared__ double jfd[fd_jac_of<Model>::value ? NC * BLOCK : 1];
    __shared__ double gcold[COLD ? GroupCell<Model, LT, FUSE, NC, COLD>::COLD_SLOTS * BLOCK : 1];
    __shared__ StepParams sP;
    stage_params(sP, a.P);
    load_table<Model>(tab, a.params, m, BLOCK);
    const int64_t c = (int64_t)blockIdx.x * (BLOCK / kGroup) + threadIdx.x / kGroup;
    if (c >= a.n) return;
    GroupCell<Model, LT, FUSE, NC, COLD> cell;
    init_cell<BLOCK>(cell, tab, jfd, gcold, a.params, m);
    cell.load(sP, a.states, a.n, c, a.hcell);
    while (cell.phase != PH_IDLE) advance_group<FIXED, FSMIN>(cell, sP);
    cell.store(a.states, a.stats, a.n, c, a.hcell);
    if (cell.status != ST_OK && cell.q == 0) atomicAdd(a.nfail, 1ull);
}

template <class Model, typename LT, bool FIXED, int BLOCK, int WPE, int FSMIN, bool FUSE, int NC,
          bool COLD = false>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(WPE, 8)))
k_group_persistent(LaunchArgs a, int m) {
    __shared__ double tab[GroupTable::DOUBLES];
    __shared__ double jfd[fd_jac_of<Model>::value ? NC * BLOCK : 1];
    __shared__ double gcold[COLD ? GroupCell<Model, LT, FUSE, NC, COLD>::COLD_SLOTS * BLOCK : 1];
    __shared__ StepParams sP;
    stage_params(sP, a.P);
    load_table<Model>(tab, a.params, m, BLOCK);
    GroupCell<Model, LT, FUSE, NC, COLD> cell;
    init_cell<BLOCK>(cell, tab, jfd, gcold, a.params, m);
    int64_t c = -1;
    bool alive = true;
    const unsigned lane = __lane_id();
    const unsigned long long below = (1ull << lane) - 1ull;
    unsigned long long qnext = 0, qend = 0; /* wave-uniform claim queue, in cells */
    RD_PH_KERNEL_BEGIN(ph_k)
    for (;;) {
        RD_PH_BEGIN(ph_c)
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
        RD_PH_END(ph_c, PHASE_CLAIM);
        if (__ballot(alive) == 0ull) break;
        advance_group<FIXED, FSMIN>(cell, sP);
    }
    RD_PH_KERNEL_END(ph_k);
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

template <class Model, typename LT, bool FIXED, int BLOCK, int WPE, int FSMIN, bool FUSE, int NC,
          bool COLD = false>
hipError_t launch_group_pers(const LaunchArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_group_persistent<Model, LT, FIXED, BLOCK, WPE, FSMIN, FUSE, NC, COLD>),
                       dim3(grid), dim3(BLOCK), 0, s, a, (int)a.P.m);
    return hipGetLastError();
}

/* FUSE: broadcasts fused into the multiply-adds (rd_group_fused.h), in FP64
 * and, for the mixed kernels' factors and solves, in FP32.  NC: columns per
 * lane; the 8-column kernels are registered under m = 8 and serve m = 5..8,
 * the 16-column ones under m = 16 for m = 9..16. */
#define RD_GONE_X(KIND, MODEL, PREC, LT, FIXED, VAR, BLOCK, WPE, FS, NC, NAME)                    \
    {KIND, fd_jac_of<MODEL>::value ? 1 : 0, NC, PREC, 1, FIXED, VAR, BLOCK, BLOCK / kGroup, NAME,                                 \
     &launch_group_one<MODEL, LT, FIXED, BLOCK, WPE, FS, true, NC>,                              \
     (const void*)&k_group_onelaunch<MODEL, LT, FIXED, BLOCK, WPE, FS, true, NC>}
#define RD_GPERS_X(KIND, MODEL, PREC, LT, FIXED, VAR, BLOCK, WPE, FS, FUSE, NC, NAME)             \
    {KIND, fd_jac_of<MODEL>::value ? 1 : 0, NC, PREC, 0, FIXED, VAR, BLOCK, BLOCK / kGroup, NAME,                                 \
     &launch_group_pers<MODEL, LT, FIXED, BLOCK, WPE, FS, FUSE, NC>,                             \
     (const void*)&k_group_persistent<MODEL, LT, FIXED, BLOCK, WPE, FS, FUSE, NC>}
#define RD_GPERS_C(KIND, MODEL, PREC, LT, VAR, BLOCK, WPE, FS, NC, NAME)                          \
    {KIND, fd_jac_of<MODEL>::value ? 1 : 0, NC, PREC, 0, false, VAR, BLOCK, BLOCK / kGroup, NAME,     \
     &launch_group_pers<MODEL, LT, false, BLOCK, WPE, FS, true, NC, true>,                          \
     (const void*)&k_group_persistent<MODEL, LT, false, BLOCK, WPE, FS, true, NC, true>}
#define RD_GONE(KIND, MODEL, PREC, LT, FIXED, VAR, BLOCK, WPE, FS, NAME)                          \
    RD_GONE_X(KIND, MODEL, PREC, LT, FIXED, VAR, BLOCK, WPE, FS, 16, NAME)
#define RD_GPERS(KIND, MODEL, PREC, LT, FIXED, VAR, BLOCK, WPE, FS, NAME)                         \
    RD_GPERS_X(KIND, MODEL, PREC, LT, FIXED, VAR, BLOCK, WPE, FS, true, 16, NAME)
#define RD_GPERS8(KIND, MODEL, PREC, LT, VAR, WPE, FS, NAME)                                      \
    RD_GPERS_X(KIND, MODEL, PREC, LT, false, VAR, 256, WPE, FS, true, 8, NAME)

}  // namespace rd
