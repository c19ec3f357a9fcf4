/*
 * rd_launch.h -- internal interface between the host library (rd_api.cpp) and
 * the kernel translation units: launch arguments and the kernel table.
 */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "rd_phase.h"

namespace rd {

/* Per-call integration constants (tolerances already transformed). */
struct StepParams {
    double dt, rtol, atol, newton_tol, h0, h_min;
    /* step-size safety factor by Newton iterations used, computed on the
     * host: fac[k] = 0.9 (2 kmax + 1) / (2 kmax + k), k = 0..kMaxTable */
    double fac[8];
    int32_t max_steps, kmax, fixed_steps, m; /* m: species per cell */
};
constexpr int kMaxFacTable = 7;

/* Copy the step parameters into the block's LDS (every thread must call it).
 * Kernels read them from there on each pass instead of holding the whole
 * block in scalar registers across the scheduling loop. */
__device__ __forceinline__ void stage_params(StepParams& dst, const StepParams& src) {
    constexpr int W = (int)(sizeof(StepParams) / sizeof(int32_t));
    static_assert(sizeof(StepParams) % sizeof(int32_t) == 0, "word-sized StepParams");
    const int32_t* s = reinterpret_cast<const int32_t*>(&src);
    int32_t* d = reinterpret_cast<int32_t*>(&dst);
    for (int i = threadIdx.x; i < W; i += blockDim.x) d[i] = s[i];
    __syncthreads();
}

struct LaunchArgs {
    double* states;                 /* [m][n] device, in place                  */
    const int32_t* order;           /* claim order (persistent), or null        */
    int32_t* stats;                 /* [9][n] device or null                    */
    const double* params;           /* device parameter block (pre-processed)  */
    int64_t n;
    unsigned long long* counter;    /* claim counter (persistent schedule)      */
    unsigned long long* nfail;      /* cells with nonzero status                */
    double* hcell;                  /* [n] per-cell warm-start step, or null    */
    StepParams P;
};

typedef hipError_t (*launch_fn)(const LaunchArgs&, int grid, hipStream_t);

struct KernelEntry {
    int kind;           /* RD_* model kind                              */
    int jac;            /* 0 analytic Jacobian, 1 forward differences   */
    int m;
    int precision;      /* 0 FP64, 1 mixed                              */
    int schedule;       /* 0 persistent, 1 one launch                   */
    int fixed;          /* 1: fixed-step test mode                      */
    int variant;        /* 1-based within (kind, m, precision, schedule) */
    int block;          /* threads per block                            */
    int cells_per_block;/* for one-launch grids                         */
    const char* name;
    launch_fn launch;
    const void* func;   /* for occupancy queries                        */
};

/* Longest-first claim order: launches the kernels that write order[n] (cell
 * indices, most expensive estimate first).  ws must hold
 * order_workspace_bytes(n) bytes.  counters (nullable): two 64-bit counters
 * the first of these kernels also clears (the persistent kernel's claim
 * counter and failure count). */
typedef hipError_t (*order_fn)(const LaunchArgs&, void* ws, int32_t* order,
                               unsigned long long* counters, hipStream_t);
size_t order_workspace_bytes(int64_t n);
order_fn find_order_fn(int kind, int m); /* m: the request's species count */

/* All kernels compiled into the library. */
const KernelEntry* kernel_table(int* count);

/* Zero two counters (graph-safe replacement for a memset). */
hipError_t launch_reset(unsigned long long* p, int n, hipStream_t s);

}  // namespace rd
