/*
 * rd_order.hip -- longest-first claim order for the persistent schedule.
 *
 * The reaction cost of a cell varies by an order of magnitude across a leaf
 * set: cells near reaction fronts need many sub-steps, cells near equilibrium
 * need one (paper Appendix A).  When the persistent kernel hands out cells in
 * storage order, the last cells claimed can be expensive ones and the launch
 * ends with a tail in which few lanes work.  Claiming the expensive cells
 * first (longest-processing-time-first list scheduling) leaves only cheap
 * cells for the end.  The cost estimate is the scaled initial rate
 *   key = max_i |f_i(u0)| dt / (atol' + rtol' |u0_i|),
 * i.e. how many tolerance units the state would move over the substep at its
 * initial speed; cells are bucketed by floor(log2(key)) and listed bucket by
 * bucket, most expensive first (a counting sort; order inside a bucket is
 * arbitrary and does not affect any cell's result).
 */
#include <hip/hip_runtime.h>

#include "rd_launch.h"
#include "rd_models.h"

namespace rd {

constexpr int kBuckets = 64;
constexpr int kLog2Min = -24; /* bucket 0 holds key < 2^-24 (and non-finite keys) */
constexpr int kOrderBlock = 256;

static size_t align_up(size_t b) { return (b + 255) & ~(size_t)255; }

size_t order_workspace_bytes(int64_t n) {
    return align_up((size_t)n) + 2 * kBuckets * sizeof(unsigned);
}

__global__ void k_order_zero(unsigned* hist) {
    if (threadIdx.x < 2 * kBuckets) hist[threadIdx.x] = 0u;
}

template <class Model>
__global__ void __launch_bounds__(kOrderBlock) k_order_cost(LaunchArgs a, unsigned char* bucket,
                                                            unsigned* hist) {
    constexpr int M = Model::M;
    __shared__ unsigned lh[kBuckets];
    if (threadIdx.x < kBuckets) lh[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t c = (int64_t)blockIdx.x * kOrderBlock + threadIdx.x;
    if (c < a.n) {
        const Model md(a.params);
        double y[M], f[M];
#pragma unroll
        for (int r = 0; r < M; ++r) y[r] = a.states[(int64_t)r * a.n + c];
        md.rhs(y, f);
        double key = 0.0;
#pragma unroll
        for (int r = 0; r < M; ++r)
            key = fmax(key, __builtin_fabs(f[r]) * a.P.dt / (a.P.atol + a.P.rtol * __builtin_fabs(y[r])));
        int b = 0;
        if (key > 0.0 && __builtin_isfinite(key)) {
            /* floor(log2(key)) from the exponent field (subnormals clamp low) */
            const int e = (int)((__double_as_longlong(key) >> 52) & 0x7ff) - 1023;
            b = e - kLog2Min;
            b = b < 0 ? 0 : (b >= kBuckets ? kBuckets - 1 : b);
        }
        bucket[c] = (unsigned char)b;
        atomicAdd(&lh[b], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kBuckets && lh[threadIdx.x]) atomicAdd(&hist[threadIdx.x], lh[threadIdx.x]);
}

/* cursor[b] = number of cells in buckets above b (descending order) */
__global__ void k_order_scan(unsigned* hist) {
    if (threadIdx.x == 0) {
        unsigned acc = 0;
        for (int b = kBuckets - 1; b >= 0; --b) {
            const unsigned h = hist[b];
            hist[kBuckets + b] = acc;
            acc += h;
        }
    }
}

__global__ void __launch_bounds__(kOrderBlock) k_order_scatter(const unsigned char* bucket,
                                                               unsigned* hist, int32_t* order,
                                                               int64_t n) {
    __shared__ unsigned lcount[kBuckets], lbase[kBuckets];
    if (threadIdx.x < kBuckets) lcount[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t c = (int64_t)blockIdx.x * kOrderBlock + threadIdx.x;
    int b = 0;
    unsigned local = 0;
    if (c < n) {
        b = bucket[c];
        local = atomicAdd(&lcount[b], 1u);
    }
    __syncthreads();
    if (threadIdx.x < kBuckets && lcount[threadIdx.x])
        lbase[threadIdx.x] = atomicAdd(&hist[kBuckets + threadIdx.x], lcount[threadIdx.x]);
    __syncthreads();
    if (c < n) order[lbase[b] + local] = (int32_t)c;
}

template <class Model>
hipError_t launch_order(const LaunchArgs& a, void* ws, int32_t* order, hipStream_t s) {
    unsigned char* bucket = (unsigned char*)ws;
    unsigned* hist = (unsigned*)((char*)ws + align_up((size_t)a.n));
    const int grid = (int)((a.n + kOrderBlock - 1) / kOrderBlock);
    hipLaunchKernelGGL(k_order_zero, dim3(1), dim3(2 * kBuckets), 0, s, hist);
    hipLaunchKernelGGL(k_order_cost<Model>, dim3(grid), dim3(kOrderBlock), 0, s, a, bucket, hist);
    hipLaunchKernelGGL(k_order_scan, dim3(1), dim3(64), 0, s, hist);
    hipLaunchKernelGGL(k_order_scatter, dim3(grid), dim3(kOrderBlock), 0, s,
                       (const unsigned char*)bucket, hist, order, a.n);
    return hipGetLastError();
}

order_fn find_order_fn(int kind, int m) {
    switch (kind) {
    case 1: return m == 3 ? &launch_order<Oregonator> : nullptr;
    case 5: return m == 3 ? &launch_order<Robertson> : nullptr;
    case 3: return m == 1 ? &launch_order<Nagumo> : nullptr;
    case 4:
        switch (m) {
        case 1: return &launch_order<Linear<1>>;
        case 2: return &launch_order<Linear<2>>;
        case 3: return &launch_order<Linear<3>>;
        case 4: return &launch_order<Linear<4>>;
        case 16: return &launch_order<Linear<16>>;
        default: return nullptr;
        }
    case 2:
        switch (m) {
        case 1: return &launch_order<Kinetics<1>>;
        case 2: return &launch_order<Kinetics<2>>;
        case 3: return &launch_order<Kinetics<3>>;
        case 4: return &launch_order<Kinetics<4>>;
        case 16: return &launch_order<Kinetics<16>>;
        default: return nullptr;
        }
    case 6:
        switch (m) {
        case 1: return &launch_order<Bytecode<1>>;
        case 2: return &launch_order<Bytecode<2>>;
        case 3: return &launch_order<Bytecode<3>>;
        case 4: return &launch_order<Bytecode<4>>;
        default: return nullptr;
        }
    default: return nullptr;
    }
}

}  // namespace rd
