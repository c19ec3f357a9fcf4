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
 * initial speed; cells are bucketed by log2(key) in quarter octaves (the
 * exponent and the two leading mantissa bits) and listed bucket by bucket,
 * most expensive first (a counting sort; order inside a bucket is arbitrary
 * and does not affect any cell's result).  On the BZ fields the most
 * expensive octave spans nearly a factor of two in cost, so whole octaves
 * would scatter the costliest cells over many more waves.
 */
#include <hip/hip_runtime.h>

#include "rd_launch.h"
#include "rd_models.h"

namespace rd {

constexpr int kSub = 4;                 /* buckets per octave */
constexpr int kBuckets = 64 * kSub;     /* 64 octaves */
constexpr int kLog2Min = -24;           /* bucket 0 holds key < 2^-24 (and non-finite keys) */
constexpr int kOrderBlock = 1024;
constexpr int kMaxGroupM = 16; /* species of the 16-lane kernels: 5..16 */

static size_t align_up(size_t b) { return (b + 255) & ~(size_t)255; }

size_t order_workspace_bytes(int64_t n) {
    return align_up((size_t)n) + 2 * kBuckets * sizeof(unsigned);
}

/* hist[0, kBuckets): cell counts per bucket; hist[kBuckets, 2 kBuckets):
 * cursors of the scatter; counters: the persistent kernel's claim counter
 * and failure count, cleared in the same launch. */
__global__ void k_order_init(unsigned* hist, unsigned long long* counters) {
    if (threadIdx.x < 2 * kBuckets) hist[threadIdx.x] = 0u;
    if (counters && threadIdx.x < 2) counters[threadIdx.x] = 0ull;
}

/* max_i |f_i(u0)| dt / (atol' + rtol' |u0_i|) of cell c, for a model with a
 * compile-time species count */
template <class Model>
struct ModelKey {
    static __device__ __forceinline__ double key(const LaunchArgs& a, int64_t c) {
        constexpr int M = Model::M;
        const Model md(a.params);
        double y[M], f[M];
#pragma unroll
        for (int r = 0; r < M; ++r) y[r] = a.states[(int64_t)r * a.n + c];
        md.rhs(y, f);
        double key = 0.0;
#pragma unroll
        for (int r = 0; r < M; ++r)
            key = fmax(key, __builtin_fabs(f[r]) * a.P.dt / (a.P.atol + a.P.rtol * __builtin_fabs(y[r])));
        return key;
    }
};

/* The same key for the kinetics (HAS_G) and linear models of the 16-lane
 * kernels, whose species count 5..16 is known at run time (StepParams::m):
 * states [m][n], parameter blocks K then G, each m x m row-major. */
template <bool HAS_G>
struct GroupKey {
    static __device__ __forceinline__ double key(const LaunchArgs& a, int64_t c) {
        const int m = a.P.m;
        double y[kMaxGroupM];
#pragma unroll
        for (int r = 0; r < kMaxGroupM; ++r) y[r] = r < m ? a.states[(int64_t)r * a.n + c] : 0.0;
        const double* K = a.params;
        const double* G = a.params + m * m;
        double key = 0.0;
        for (int i = 0; i < m; ++i) {
            double lin = 0.0, loss = 0.0;
#pragma unroll
            for (int j = 0; j < kMaxGroupM; ++j) {
                if (j < m) {
                    lin += K[i * m + j] * y[j];
                    if (HAS_G) loss += G[i * m + j] * y[j];
                }
            }
            double yi = 0.0;
#pragma unroll
            for (int r = 0; r < kMaxGroupM; ++r) yi = r == i ? y[r] : yi;
            const double f = HAS_G ? lin - yi * loss : lin;
            key = fmax(key, __builtin_fabs(f) * a.P.dt / (a.P.atol + a.P.rtol * __builtin_fabs(yi)));
        }
        return key;
    }
};

/* Cells per thread of the two counting-sort kernels: cell k * kOrderBlock +
 * threadIdx.x of the block's span of kOrderCells cells (coalesced for each
 * k).  Four cells per thread cut the blocks, and so the global atomics on
 * the 2 x kBuckets shared counters, by four. */
constexpr int kOrderCpt = 4;
constexpr int kOrderCells = kOrderBlock * kOrderCpt;

__device__ __forceinline__ int bucket_of(double key) {
    if (!(key > 0.0) || !__builtin_isfinite(key)) return 0;
    /* floor(kSub log2(key)), approximately: the exponent field and the
     * leading mantissa bits (subnormals clamp low) */
    const long long bits = __double_as_longlong(key);
    const int e = (int)((bits >> 52) & 0x7ff) - 1023;
    const int q = (int)((bits >> 50) & (kSub - 1));
    const int b = (e - kLog2Min) * kSub + q;
    return b < 0 ? 0 : (b >= kBuckets ? kBuckets - 1 : b);
}

/* Bucket of every cell, and the counts per bucket (an LDS histogram per
 * block, added to the global one with one atomic per nonzero bucket). */
template <class Key>
__global__ void __launch_bounds__(kOrderBlock) k_order_cost(LaunchArgs a, unsigned char* bucket,
                                                            unsigned* hist) {
    __shared__ unsigned lh[kBuckets];
    if (threadIdx.x < kBuckets) lh[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t c0 = (int64_t)blockIdx.x * kOrderCells + threadIdx.x;
#pragma unroll
    for (int k = 0; k < kOrderCpt; ++k) {
        const int64_t c = c0 + (int64_t)k * kOrderBlock;
        if (c < a.n) {
            const int b = bucket_of(Key::key(a, c));
            bucket[c] = (unsigned char)b;
            atomicAdd(&lh[b], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < kBuckets && lh[threadIdx.x]) atomicAdd(&hist[threadIdx.x], lh[threadIdx.x]);
}

/* Each block finds where the buckets start (most expensive bucket first:
 * start[b] = number of cells in buckets above b) from the global counts,
 * ranks its cells inside their buckets (LDS atomics: any order inside a
 * bucket is valid), reserves one range per bucket from the bucket's cursor
 * and writes the cell indices there. */
__global__ void __launch_bounds__(kOrderBlock) k_order_scatter(const unsigned char* bucket,
                                                               unsigned* hist, int32_t* order,
                                                               int64_t n) {
    static_assert(kBuckets == 64 * kSub, "the bucket scan runs on one wave, kSub buckets per lane");
    __shared__ unsigned lcount[kBuckets], lbase[kBuckets];
    if (threadIdx.x < 64) {
        /* lane l holds buckets kSub l .. kSub l + kSub - 1: suffix sums of
         * the lane totals across the wave, then inside the lane downwards */
        unsigned h[kSub], tot = 0u;
#pragma unroll
        for (int k = 0; k < kSub; ++k) {
            h[k] = hist[kSub * threadIdx.x + k];
            tot += h[k];
        }
        unsigned s = tot;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const unsigned t = __shfl_down(s, off);
            if (threadIdx.x + off < 64) s += t;
        }
        unsigned above = s - tot; /* cells in the buckets of higher lanes */
#pragma unroll
        for (int k = kSub - 1; k >= 0; --k) {
            lbase[kSub * threadIdx.x + k] = above;
            lcount[kSub * threadIdx.x + k] = 0u;
            above += h[k];
        }
    }
    __syncthreads();
    const int64_t c0 = (int64_t)blockIdx.x * kOrderCells + threadIdx.x;
    int b[kOrderCpt];
    unsigned local[kOrderCpt];
#pragma unroll
    for (int k = 0; k < kOrderCpt; ++k) {
        const int64_t c = c0 + (int64_t)k * kOrderBlock;
        b[k] = c < n ? (int)bucket[c] : 0;
        local[k] = c < n ? atomicAdd(&lcount[b[k]], 1u) : 0u;
    }
    __syncthreads();
    if (threadIdx.x < kBuckets && lcount[threadIdx.x])
        lbase[threadIdx.x] += atomicAdd(&hist[kBuckets + threadIdx.x], lcount[threadIdx.x]);
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kOrderCpt; ++k) {
        const int64_t c = c0 + (int64_t)k * kOrderBlock;
        if (c < n) order[lbase[b[k]] + local[k]] = (int32_t)c;
    }
}

template <class Key>
hipError_t launch_order(const LaunchArgs& a, void* ws, int32_t* order,
                        unsigned long long* counters, hipStream_t s) {
    unsigned char* bucket = (unsigned char*)ws;
    unsigned* hist = (unsigned*)((char*)ws + align_up((size_t)a.n));
    const int grid = (int)((a.n + kOrderCells - 1) / kOrderCells);
    hipLaunchKernelGGL(k_order_init, dim3(1), dim3(2 * kBuckets), 0, s, hist, counters);
    hipLaunchKernelGGL(k_order_cost<Key>, dim3(grid), dim3(kOrderBlock), 0, s, a, bucket, hist);
    hipLaunchKernelGGL(k_order_scatter, dim3(grid), dim3(kOrderBlock), 0, s,
                       (const unsigned char*)bucket, hist, order, a.n);
    return hipGetLastError();
}

order_fn find_order_fn(int kind, int m) {
    if ((kind == 2 || kind == 4) && m > 4 && m <= kMaxGroupM)
        return kind == 2 ? &launch_order<GroupKey<true>> : &launch_order<GroupKey<false>>;
    switch (kind) {
    case 1: return m == 3 ? &launch_order<ModelKey<Oregonator>> : nullptr;
    case 5: return m == 3 ? &launch_order<ModelKey<Robertson>> : nullptr;
    case 3: return m == 1 ? &launch_order<ModelKey<Nagumo>> : nullptr;
    case 4:
        switch (m) {
        case 1: return &launch_order<ModelKey<Linear<1>>>;
        case 2: return &launch_order<ModelKey<Linear<2>>>;
        case 3: return &launch_order<ModelKey<Linear<3>>>;
        case 4: return &launch_order<ModelKey<Linear<4>>>;
        default: return nullptr;
        }
    case 2:
        switch (m) {
        case 1: return &launch_order<ModelKey<Kinetics<1>>>;
        case 2: return &launch_order<ModelKey<Kinetics<2>>>;
        case 3: return &launch_order<ModelKey<Kinetics<3>>>;
        case 4: return &launch_order<ModelKey<Kinetics<4>>>;
        default: return nullptr;
        }
    case 6:
        switch (m) {
        case 1: return &launch_order<ModelKey<Bytecode<1>>>;
        case 2: return &launch_order<ModelKey<Bytecode<2>>>;
        case 3: return &launch_order<ModelKey<Bytecode<3>>>;
        case 4: return &launch_order<ModelKey<Bytecode<4>>>;
        default: return nullptr;
        }
    default: return nullptr;
    }
}

}  // namespace rd
