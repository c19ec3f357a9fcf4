/*
 * rd_mra.hip -- multiresolution leaf sets on the GPU (Descombes et al., §2.2
 * after Cohen et al. 2003; node keys of §3.1): from a field on the finest
 * uniform level J of the dyadic tree of [0,1]^d (d = 2, 3), build the graded
 * tree whose leaves are the adapted grid, and go back (reconstruction).
 *
 * GPU layout: every level j of the tree is a dense array of 2^(d j) nodes per
 * species, in Morton order (index = bits of x, y[, z] interleaved, x most
 * significant in each group), so the 2^d children of node p are the
 * consecutive indices 2^d p .. 2^d p + 2^d - 1 and projection reads
 * contiguous memory.  Per level a byte array R_j marks the nodes that have
 * children.  One kernel per level and operation:
 *   projection      node = average of its 2^d children;
 *   details + flags one thread per parent: predicts its 2^d children from the
 *                   3^d parent-level stencil (third order, tensor product of
 *                   the 1D operator, one direction at a time, even reflection
 *                   at the domain edge), details d = u - prediction, and
 *                   R_{j-1}[p] = some child with (1/m) sum_i (d_i/s_i)^2 >= eps_j^2,
 *                   eps_j^2 = 2^(d (j-J)) eps^2;
 *   grading         finest to coarsest: a node with children makes the
 *                   parents of its 3^d neighbours get children;
 *   leaves          one thread per finest cell finds the leaf covering it;
 *                   the first cell of each leaf emits the leaf, compacted in
 *                   Morton order by a block count, a scan and a write pass.
 * Keys: the level-j Morton index left-aligned in bits 63..16 (48-bit
 * abscissa), the level in bits 15..12, bits 11..0 free.
 *
 * The detail decision compares floating-point numbers against a threshold;
 * this file is compiled without contraction and evaluates every formula in
 * a fixed order, so the decisions are reproducible operation by operation.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <vector>

#include "rd_internal.h"

namespace rd {

/* ---------------------------------------------------------------- Morton */
__host__ __device__ __forceinline__ int64_t morton_encode(const int* c, int d, int bits) {
    int64_t out = 0;
    for (int b = 0; b < bits; ++b)
        for (int a = 0; a < d; ++a)
            out |= (int64_t)((c[a] >> b) & 1) << (d * b + (d - 1 - a));
    return out;
}
__host__ __device__ __forceinline__ void morton_decode(int64_t idx, int d, int bits, int* c) {
    for (int a = 0; a < d; ++a) c[a] = 0;
    for (int b = 0; b < bits; ++b)
        for (int a = 0; a < d; ++a) c[a] |= (int)((idx >> (d * b + (d - 1 - a))) & 1) << b;
}

struct Pyr {
    int d, J, m;
    int64_t total;          /* nodes over all levels, per species */
    int64_t off[25];        /* start of level j within a species plane */
    double* U;              /* [m][total] */
    unsigned char* R;       /* [total] refine flags (finest level unused) */
    unsigned char* T;       /* [total] tree membership (reconstruction) */
};

__device__ __forceinline__ double* lvl(const Pyr& P, int i, int j) {
    return P.U + (int64_t)i * P.total + P.off[j];
}

/* even reflection at the domain edge */
__device__ __forceinline__ int clampc(int c, int N) { return c < 0 ? 0 : (c >= N ? N - 1 : c); }

/* bit b of v moved to bit d b (b < bits) */
__device__ __forceinline__ int64_t spread_bits(int v, int d, int bits) {
    int64_t out = 0;
    for (int b = 0; b < bits; ++b) out |= (int64_t)((v >> b) & 1) << (d * b);
    return out;
}

/* Level-jc indices of the 3^D stencil around the node with coordinates pc,
 * each coordinate clamped to the domain (even reflection), x fastest then y
 * then z: the Morton index of a node is the OR of its coordinates' spread
 * bits (x most significant within each group of D bits), so the 3^D indices
 * take 3 D spreads instead of 3^D full encodings.  A level holds at most
 * 2^(d (J - 1)) <= 2^28 nodes below the finest (d J <= 30), so 32 bits hold
 * the indices. */
template <int D>
__device__ __forceinline__ void stencil_index(int jc, const int* pc, uint32_t* idx) {
    const int N = 1 << jc;
    int64_t sp[3][3];
    for (int a = 0; a < D; ++a)
        for (int o = 0; o < 3; ++o) sp[a][o] = spread_bits(clampc(pc[a] + o - 1, N), D, jc) << (D - 1 - a);
    if (D == 2) {
        for (int oy = 0; oy < 3; ++oy)
            for (int ox = 0; ox < 3; ++ox) idx[oy * 3 + ox] = (uint32_t)(sp[0][ox] | sp[1][oy]);
    } else {
        for (int oz = 0; oz < 3; ++oz)
            for (int oy = 0; oy < 3; ++oy)
                for (int ox = 0; ox < 3; ++ox)
                    idx[(oz * 3 + oy) * 3 + ox] = (uint32_t)(sp[0][ox] | sp[1][oy] | sp[2][oz]);
    }
}

/* Prediction of the child with per-axis bits cb from the parent's 3^D
 * stencil values v (ordered as stencil_index), one direction at a time: in
 * x along each row, then in y over the three rows, then in z over the three
 * planes; each step is centre + sign/8 (minus-side value - plus-side value). */
template <int D>
__device__ __forceinline__ double predict(const double* v, const int* cb) {
    double sg[3];
    for (int a = 0; a < D; ++a) sg[a] = cb[a] == 0 ? 0.125 : -0.125;
    if (D == 2) {
        double rows[3];
        for (int oy = 0; oy < 3; ++oy) {
            const double vm = v[oy * 3], v0 = v[oy * 3 + 1], vp = v[oy * 3 + 2];
            const double dif = vm - vp;
            const double t = sg[0] * dif;
            rows[oy] = v0 + t;
        }
        const double dif = rows[0] - rows[2];
        const double t = sg[1] * dif;
        return rows[1] + t;
    } else {
        double planes[3];
        for (int oz = 0; oz < 3; ++oz) {
            double rows[3];
            for (int oy = 0; oy < 3; ++oy) {
                const double* r = v + (oz * 3 + oy) * 3;
                const double dif = r[0] - r[2];
                const double t = sg[0] * dif;
                rows[oy] = r[1] + t;
            }
            const double dif = rows[0] - rows[2];
            const double t = sg[1] * dif;
            planes[oz] = rows[1] + t;
        }
        const double dif = planes[0] - planes[2];
        const double t = sg[2] * dif;
        return planes[1] + t;
    }
}

/* ---------------------------------------------------------------- kernels */
template <int D>
__global__ void k_to_morton(const double* __restrict__ fine, Pyr P) {
    const int64_t n = P.off[P.J + 1] - P.off[P.J];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int N = 1 << P.J;
    int c[3];
    int64_t t = r;
    for (int a = 0; a < D; ++a) { c[a] = (int)(t % N); t /= N; }
    const int64_t k = morton_encode(c, D, P.J);
    for (int i = 0; i < P.m; ++i) lvl(P, i, P.J)[k] = fine[(int64_t)i * n + r];
}

template <int D>
__global__ void k_from_morton(double* __restrict__ fine, Pyr P) {
    const int64_t n = P.off[P.J + 1] - P.off[P.J];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int N = 1 << P.J;
    int c[3];
    int64_t t = r;
    for (int a = 0; a < D; ++a) { c[a] = (int)(t % N); t /= N; }
    const int64_t k = morton_encode(c, D, P.J);
    for (int i = 0; i < P.m; ++i) fine[(int64_t)i * n + r] = lvl(P, i, P.J)[k];
}

/* Finest level <-> row-major field through LDS bricks: an aligned brick of
 * side 2^S (2^(D S) = 4096 cells) is one contiguous range of Morton indices,
 * brick b holding [b 4096, (b + 1) 4096) with b the Morton index of the
 * brick's coordinates.  The row-major side moves as row segments of 2^S
 * doubles, the Morton side as contiguous runs; a plain copy either way. */
constexpr int kBrickCells = 4096;
template <int D> struct Brick { static constexpr int S = D == 2 ? 6 : 4; };

template <int D, bool TO_MORTON>
__global__ void __launch_bounds__(256) k_morton_brick(const double* __restrict__ fine_in,
                                                      double* __restrict__ fine_out, Pyr P) {
    constexpr int S = Brick<D>::S;
    __shared__ double tile[kBrickCells];
    const int64_t b = blockIdx.x;
    const int64_t n = P.off[P.J + 1] - P.off[P.J];
    const int N = 1 << P.J;
    int bc[3];
    morton_decode(b, D, P.J - S, bc);
    for (int i = 0; i < P.m; ++i) {
        const double* fi = TO_MORTON ? fine_in + (int64_t)i * n : nullptr;
        double* fo = TO_MORTON ? nullptr : fine_out + (int64_t)i * n;
        double* u = lvl(P, i, P.J) + b * kBrickCells;
        if (TO_MORTON) {
            for (int q = threadIdx.x; q < kBrickCells; q += 256) {
                const int lx = q & ((1 << S) - 1), ly = (q >> S) & ((1 << S) - 1), lz = q >> (2 * S);
                const int64_t gx = ((int64_t)bc[0] << S) + lx, gy = ((int64_t)bc[1] << S) + ly;
                const int64_t gz = D == 3 ? ((int64_t)bc[2] << S) + lz : 0;
                tile[q] = fi[gx + N * (gy + N * gz)];
            }
            __syncthreads();
            for (int k = threadIdx.x; k < kBrickCells; k += 256) {
                int l[3];
                morton_decode(k, D, S, l);
                u[k] = tile[l[0] + (l[1] << S) + (D == 3 ? (l[2] << (2 * S)) : 0)];
            }
        } else {
            for (int k = threadIdx.x; k < kBrickCells; k += 256) {
                int l[3];
                morton_decode(k, D, S, l);
                tile[l[0] + (l[1] << S) + (D == 3 ? (l[2] << (2 * S)) : 0)] = u[k];
            }
            __syncthreads();
            for (int q = threadIdx.x; q < kBrickCells; q += 256) {
                const int lx = q & ((1 << S) - 1), ly = (q >> S) & ((1 << S) - 1), lz = q >> (2 * S);
                const int64_t gx = ((int64_t)bc[0] << S) + lx, gy = ((int64_t)bc[1] << S) + ly;
                const int64_t gz = D == 3 ? ((int64_t)bc[2] << S) + lz : 0;
                fo[gx + N * (gy + N * gz)] = tile[q];
            }
        }
        __syncthreads();
    }
}

/* level j -> j-1: node = average of its 2^D children (summed in child order) */
template <int D>
__global__ void k_project(Pyr P, int j) {
    const int64_t np = (int64_t)1 << (D * (j - 1));
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    constexpr int NC = 1 << D;
    for (int i = 0; i < P.m; ++i) {
        const double* u = lvl(P, i, j) + p * NC;
        double s = u[0];
        for (int c = 1; c < NC; ++c) s = s + u[c];
        lvl(P, i, j - 1)[p] = s * (1.0 / NC);
    }
}

/* details of the children of level-(j-1) node p and its refine flag; with
 * refine, a significant child below the finest level gets children too.  The
 * stencil is gathered once per species and serves all 2^D children; each
 * child's sum over the species runs in species order. */
template <int D>
__global__ void k_detail_flags(Pyr P, int j, double eps_j2, const double* __restrict__ scale,
                               int refine) {
    const int jc = j - 1;
    const int64_t np = (int64_t)1 << (D * jc);
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    constexpr int NC = 1 << D, NS = D == 2 ? 9 : 27;
    int pc[3];
    morton_decode(p, D, jc, pc);
    uint32_t idx[NS];
    stencil_index<D>(jc, pc, idx);
    double acc[NC];
    for (int i = 0; i < P.m; ++i) {
        const double* uc = lvl(P, i, jc);
        double v[NS];
        for (int q = 0; q < NS; ++q) v[q] = uc[idx[q]];
        const double* uf = lvl(P, i, j) + p * NC;
        for (int c = 0; c < NC; ++c) {
            int cb[3];
            for (int a = 0; a < D; ++a) cb[a] = (c >> (D - 1 - a)) & 1;
            const double pred = predict<D>(v, cb);
            const double dd = uf[c] - pred;
            const double q = dd / scale[i];
            acc[c] = (i == 0) ? q * q : acc[c] + q * q;
        }
    }
    bool sig = false;
    const double invm = 1.0 / P.m;
    for (int c = 0; c < NC; ++c) {
        const bool sc = acc[c] * invm >= eps_j2;
        sig = sig || sc;
        if (refine && sc && j < P.J) P.R[P.off[j] + p * NC + c] = 1;
    }
    if (sig) P.R[P.off[jc] + p] = 1;
}

/* grading: a node of level j with children makes the parents of its 3^D
 * neighbours (inside the domain) get children */
template <int D>
__global__ void k_grade(Pyr P, int j) {
    const int64_t nj = (int64_t)1 << (D * j);
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nj || !P.R[P.off[j] + k]) return;
    const int N = 1 << j;
    int c[3];
    morton_decode(k, D, j, c);
    const int lo2 = D == 3 ? -1 : 0, hi2 = D == 3 ? 1 : 0;
    for (int oz = lo2; oz <= hi2; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
                int nb[3] = {c[0] + ox, c[1] + oy, D == 3 ? c[2] + oz : 0};
                bool in = true;
                for (int a = 0; a < D; ++a) in = in && nb[a] >= 0 && nb[a] < N;
                if (!in) continue;
                const int64_t q = morton_encode(nb, D, j);
                P.R[P.off[j - 1] + (q >> D)] = 1;
            }
}

/* level of the leaf covering finest cell f (Morton), and whether f is the
 * first finest cell of that leaf */
__device__ __forceinline__ int leaf_of(const Pyr& P, int64_t f, int d, bool& first) {
    for (int j = 0; j <= P.J; ++j) {
        const int64_t k = f >> (d * (P.J - j));
        const bool exists = (j == 0) || P.R[P.off[j - 1] + (k >> d)];
        const bool refined = (j < P.J) && P.R[P.off[j] + k];
        if (exists && !refined) {
            first = (f & (((int64_t)1 << (d * (P.J - j))) - 1)) == 0;
            return j;
        }
    }
    first = false;
    return -1;
}

constexpr int kLeafBlock = 256;

constexpr int kMaxLevels = 16; /* J <= 15: the level takes 4 bits of a key */

/* leaves per block, and per block and level (level_block[l * gridDim.x + b]) */
__global__ void k_leaf_count(Pyr P, int d, unsigned* __restrict__ block_count,
                             unsigned* __restrict__ level_block) {
    const int64_t n = P.off[P.J + 1] - P.off[P.J];
    const int64_t f = (int64_t)blockIdx.x * kLeafBlock + threadIdx.x;
    __shared__ unsigned lc[kMaxLevels];
    if (threadIdx.x < kMaxLevels) lc[threadIdx.x] = 0u;
    __syncthreads();
    bool first = false;
    int j = -1;
    if (f < n) j = leaf_of(P, f, d, first);
    if (first) atomicAdd(&lc[j], 1u);
    const unsigned cnt = (unsigned)__popcll(__ballot(first));
    __shared__ unsigned wsum[kLeafBlock / 64];
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = cnt;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned s = 0;
        for (int w = 0; w < kLeafBlock / 64; ++w) s += wsum[w];
        block_count[blockIdx.x] = s;
    }
    if (threadIdx.x < kMaxLevels) level_block[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = lc[threadIdx.x];
}

/* Exclusive scan of the nb block counts in three passes: chunk sums (one
 * block per 1024 counts), a one-block scan of the chunk sums, and the scan
 * within each chunk plus its offset.  A chunk sum is at most 1024 x 256. */
constexpr int kScanChunk = 1024;

__global__ void __launch_bounds__(kScanChunk) k_chunk_sums(const unsigned* __restrict__ in, int64_t nb,
                                                           unsigned* __restrict__ chunk_sum) {
    const int64_t b = (int64_t)blockIdx.x * kScanChunk + threadIdx.x;
    const unsigned v = b < nb ? in[b] : 0u;
    __shared__ unsigned part[kScanChunk];
    part[threadIdx.x] = v;
    __syncthreads();
    for (int h = kScanChunk / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) chunk_sum[blockIdx.x] = part[0];
}

__global__ void __launch_bounds__(kScanChunk) k_chunk_apply(const unsigned* __restrict__ in, int64_t nb,
                                                            const unsigned long long* __restrict__ chunk_off,
                                                            int64_t nchunks,
                                                            unsigned long long* __restrict__ out) {
    const int t = threadIdx.x;
    const int64_t b = (int64_t)blockIdx.x * kScanChunk + t;
    const unsigned v = b < nb ? in[b] : 0u;
    __shared__ unsigned long long part[kScanChunk];
    part[t] = v;
    __syncthreads();
    for (int h = 1; h < kScanChunk; h <<= 1) {
        const unsigned long long x = t >= h ? part[t - h] : 0ull;
        __syncthreads();
        part[t] += x;
        __syncthreads();
    }
    if (b < nb) out[b] = chunk_off[blockIdx.x] + part[t] - v;
    if (blockIdx.x == 0 && t == 0) out[nb] = chunk_off[nchunks];
}

/* leaves per level: block l (1024 threads) sums level l over the nb blocks of
 * k_leaf_count */
__global__ void __launch_bounds__(1024) k_level_sum(const unsigned* __restrict__ level_block, int64_t nb,
                                                    unsigned long long* __restrict__ level_tot) {
    const unsigned* in = level_block + (int64_t)blockIdx.x * nb;
    unsigned long long s = 0;
    for (int64_t b = threadIdx.x; b < nb; b += blockDim.x) s += in[b];
    __shared__ unsigned long long part[1024];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = 512; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) level_tot[blockIdx.x] = part[0];
}

/* exclusive scan of nb block counts in one block of 1024 threads; the total
 * goes to out[nb] */
__global__ void k_scan_blocks(const unsigned* __restrict__ in, unsigned long long* __restrict__ out,
                              int64_t nb) {
    __shared__ unsigned long long part[1024];
    const int t = threadIdx.x;
    const int64_t per = (nb + 1023) / 1024;
    const int64_t b0 = t * per, b1 = (b0 + per < nb) ? b0 + per : nb;
    unsigned long long s = 0;
    for (int64_t b = b0; b < b1; ++b) s += in[b];
    part[t] = s;
    __syncthreads();
    /* inclusive scan of the 1024 partial sums in LDS (log2 1024 steps) */
    for (int h = 1; h < 1024; h <<= 1) {
        const unsigned long long v = t >= h ? part[t - h] : 0ull;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    if (t == 1023) out[nb] = part[1023];
    unsigned long long run = part[t] - s;
    for (int64_t b = b0; b < b1; ++b) {
        out[b] = run;
        run += in[b];
    }
}

__global__ void k_leaf_write(Pyr P, int d, const unsigned long long* __restrict__ block_off,
                             uint64_t* __restrict__ keys, double* __restrict__ values,
                             int64_t n_leaves) {
    const int64_t n = P.off[P.J + 1] - P.off[P.J];
    const int64_t f = (int64_t)blockIdx.x * kLeafBlock + threadIdx.x;
    bool first = false;
    int j = -1;
    if (f < n) j = leaf_of(P, f, d, first);
    const unsigned long long mask = __ballot(first);
    __shared__ unsigned wsum[kLeafBlock / 64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) wsum[w] = (unsigned)__popcll(mask);
    __syncthreads();
    if (!first) return;
    unsigned before = 0;
    for (int i = 0; i < w; ++i) before += wsum[i];
    before += (unsigned)__popcll(mask & ((1ull << lane) - 1ull));
    const int64_t pos = (int64_t)block_off[blockIdx.x] + before;
    if (pos >= n_leaves) return;
    const int64_t k = f >> (d * (P.J - j));
    keys[pos] = (j == 0 ? 0ull : ((uint64_t)k << (64 - d * j))) | ((uint64_t)j << 12);
    for (int i = 0; i < P.m; ++i) values[(int64_t)i * n_leaves + pos] = lvl(P, i, j)[k];
}

/* reconstruction: leaves into their levels, tree membership */
__global__ void k_scatter_leaves(Pyr P, int d, const uint64_t* __restrict__ keys,
                                 const double* __restrict__ values, int64_t n_leaves) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_leaves) return;
    const uint64_t key = keys[t];
    const int j = (int)((key >> 12) & 15u);
    if (j > P.J) return;
    const int64_t k = j == 0 ? 0 : (int64_t)(key >> (64 - d * j));
    if (k >= ((int64_t)1 << (d * j))) return;
    P.T[P.off[j] + k] = 1;
    for (int i = 0; i < P.m; ++i) lvl(P, i, j)[k] = values[(int64_t)i * n_leaves + t];
}

/* parents of tree nodes are tree nodes valued by the average of children */
template <int D>
__global__ void k_tree_up(Pyr P, int j) {
    const int64_t np = (int64_t)1 << (D * (j - 1));
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    constexpr int NC = 1 << D;
    bool any = false;
    for (int c = 0; c < NC; ++c) any = any || P.T[P.off[j] + p * NC + c];
    if (!any) return;
    P.T[P.off[j - 1] + p] = 1;
    for (int i = 0; i < P.m; ++i) {
        const double* u = lvl(P, i, j) + p * NC;
        double s = u[0];
        for (int c = 1; c < NC; ++c) s = s + u[c];
        lvl(P, i, j - 1)[p] = s * (1.0 / NC);
    }
}

/* nodes outside the tree are predicted from the (complete) coarser level:
 * one thread per level-(j-1) parent, its stencil gathered once per species
 * for those of its 2^D children that are outside the tree */
template <int D>
__global__ void k_fill_down(Pyr P, int j) {
    const int jc = j - 1;
    const int64_t np = (int64_t)1 << (D * jc);
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= np) return;
    constexpr int NC = 1 << D, NS = D == 2 ? 9 : 27;
    const unsigned char* t = P.T + P.off[j] + p * NC;
    bool any = false;
    for (int c = 0; c < NC; ++c) any = any || !t[c];
    if (!any) return;
    int pc[3];
    morton_decode(p, D, jc, pc);
    uint32_t idx[NS];
    stencil_index<D>(jc, pc, idx);
    for (int i = 0; i < P.m; ++i) {
        const double* uc = lvl(P, i, jc);
        double v[NS];
        for (int q = 0; q < NS; ++q) v[q] = uc[idx[q]];
        double* uf = lvl(P, i, j) + p * NC;
        for (int c = 0; c < NC; ++c) {
            if (t[c]) continue;
            int cb[3];
            for (int a = 0; a < D; ++a) cb[a] = (c >> (D - 1 - a)) & 1;
            uf[c] = predict<D>(v, cb);
        }
    }
}

/* ---------------------------------------------------------------- host */
struct MraWork {
    void* buf = nullptr;
    size_t cap = 0;
    std::vector<void*> retired;
};
static std::mutex g_mra_mu;
static std::map<std::pair<int, hipStream_t>, MraWork> g_mra;

static void* mra_workspace(hipStream_t s, size_t bytes, int* err) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) { *err = RD_EDEVICE; return nullptr; }
    std::lock_guard<std::mutex> lk(g_mra_mu);
    MraWork& w = g_mra[{dev, s}];
    if (w.cap < bytes) {
        void* p = nullptr;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            set_error("hipMalloc(MRA workspace of %zu bytes) failed", bytes);
            *err = RD_ENOMEM;
            return nullptr;
        }
        if (w.buf) w.retired.push_back(w.buf);
        w.buf = p;
        w.cap = bytes;
    }
    return w.buf;
}

static bool mra_params_valid(const rd_mra_params* p, int32_t m) {
    if (!p || (p->dim != 2 && p->dim != 3) || m < 1 || m > RD_MAX_M) return false;
    if (p->levels < 1 || p->dim * p->levels > 30) return false; /* <= 2^30 finest cells */
    if (!std::isfinite(p->eps) || p->eps < 0.0) return false;
    if (p->scale)
        for (int i = 0; i < m; ++i)
            if (!(p->scale[i] > 0.0) || !std::isfinite(p->scale[i])) return false;
    return true;
}

/* pyramid + flags + scratch, laid out in one workspace */
static int setup_pyr(const rd_mra_params* p, int32_t m, hipStream_t s, Pyr& P, double** scale_dev,
                     unsigned** bcount, unsigned long long** boff, int64_t* nblocks) {
    P.d = p->dim;
    P.J = p->levels;
    P.m = m;
    int64_t off = 0;
    for (int j = 0; j <= P.J; ++j) {
        P.off[j] = off;
        off += (int64_t)1 << (P.d * j);
    }
    P.off[P.J + 1] = off;
    P.total = off;
    const int64_t nfine = (int64_t)1 << (P.d * P.J);
    *nblocks = (nfine + kLeafBlock - 1) / kLeafBlock;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t bU = al(sizeof(double) * (size_t)m * P.total);
    const size_t bR = al((size_t)P.total);
    const size_t bS = al(sizeof(double) * m);
    const size_t nch = ((size_t)*nblocks + kScanChunk - 1) / kScanChunk;
    /* block counts, then per level and block (k_leaf_count), then the chunk sums of the scan */
    const size_t bC = al(sizeof(unsigned) * ((size_t)*nblocks * (1 + kMaxLevels) + nch));
    /* block offsets and the total, the leaves per level, then the chunk offsets and their total */
    const size_t bO = al(sizeof(unsigned long long) * ((size_t)*nblocks + 1 + kMaxLevels + nch + 1));
    int err = 0;
    char* w = (char*)mra_workspace(s, bU + 2 * bR + bS + bC + bO, &err);
    if (!w) return err ? err : RD_ENOMEM;
    P.U = (double*)w;
    P.R = (unsigned char*)(w + bU);
    P.T = (unsigned char*)(w + bU + bR);
    *scale_dev = (double*)(w + bU + 2 * bR);
    *bcount = (unsigned*)(w + bU + 2 * bR + bS);
    *boff = (unsigned long long*)(w + bU + 2 * bR + bS + bC);
    return 0;
}

static unsigned blocks_for(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

#define MRA_TRY(e)                                                                              \
    do {                                                                                        \
        hipError_t e_ = (e);                                                                    \
        if (e_ != hipSuccess) { set_error("%s: %s", #e, hipGetErrorString(e_)); return RD_EDEVICE; } \
    } while (0)

/* flags (details, optional refinement, grading) over the pyramid P.U and the
 * leaf set they define; P.U holds every level on entry */
static int64_t flags_and_leaves(Pyr& P, const rd_mra_params* p, hipStream_t s, const double* sc,
                                unsigned* bcount, unsigned long long* boff, int64_t nb,
                                uint64_t* keys, double* values, int64_t capacity,
                                int64_t* level_counts) {
    const int d = P.d, J = P.J;
    const int B = 256;
    MRA_TRY(hipMemsetAsync(P.R, 0, (size_t)P.total, s));
    for (int j = 1; j <= J; ++j) {
        const int64_t np = (int64_t)1 << (d * (j - 1));
        const double e2 = (p->eps * p->eps) * std::ldexp(1.0, d * (j - J));
        const int rf = p->refine ? 1 : 0;
        if (d == 2) hipLaunchKernelGGL(k_detail_flags<2>, dim3(blocks_for(np, B)), dim3(B), 0, s, P, j, e2, sc, rf);
        else hipLaunchKernelGGL(k_detail_flags<3>, dim3(blocks_for(np, B)), dim3(B), 0, s, P, j, e2, sc, rf);
    }
    for (int j = J - 1; j >= 1; --j) {
        const int64_t nj = (int64_t)1 << (d * j);
        if (d == 2) hipLaunchKernelGGL(k_grade<2>, dim3(blocks_for(nj, B)), dim3(B), 0, s, P, j);
        else hipLaunchKernelGGL(k_grade<3>, dim3(blocks_for(nj, B)), dim3(B), 0, s, P, j);
    }
    hipLaunchKernelGGL(k_leaf_count, dim3((unsigned)nb), dim3(kLeafBlock), 0, s, P, d, bcount, bcount + nb);
    {
        const int64_t nch = (nb + kScanChunk - 1) / kScanChunk;
        unsigned* csum = bcount + nb * (1 + kMaxLevels);
        unsigned long long* coff = boff + nb + 1 + kMaxLevels;
        hipLaunchKernelGGL(k_chunk_sums, dim3((unsigned)nch), dim3(kScanChunk), 0, s,
                           (const unsigned*)bcount, nb, csum);
        hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(1024), 0, s, (const unsigned*)csum, coff, nch);
        hipLaunchKernelGGL(k_chunk_apply, dim3((unsigned)nch), dim3(kScanChunk), 0, s,
                           (const unsigned*)bcount, nb, (const unsigned long long*)coff, nch, boff);
    }
    MRA_TRY(hipGetLastError());
    unsigned long long total = 0;
    MRA_TRY(hipMemcpyAsync(&total, boff + nb, sizeof(total), hipMemcpyDeviceToHost, s));
    MRA_TRY(hipStreamSynchronize(s));
    const int64_t nl = (int64_t)total;
    if (nl <= capacity && nl > 0) {
        if (!keys || !values) { set_error("keys / values are null"); return RD_EINVAL; }
        hipLaunchKernelGGL(k_leaf_write, dim3((unsigned)nb), dim3(kLeafBlock), 0, s, P, d,
                           (const unsigned long long*)boff, keys, values, nl);
        MRA_TRY(hipGetLastError());
        if (level_counts) {
            unsigned long long* ltot = boff + nb + 1;
            hipLaunchKernelGGL(k_level_sum, dim3((unsigned)(J + 1)), dim3(1024), 0, s,
                               (const unsigned*)(bcount + nb), nb, ltot);
            MRA_TRY(hipGetLastError());
            unsigned long long hl[kMaxLevels];
            MRA_TRY(hipMemcpyAsync(hl, ltot, sizeof(unsigned long long) * (J + 1), hipMemcpyDeviceToHost, s));
            MRA_TRY(hipStreamSynchronize(s));
            for (int j = 0; j <= J; ++j) level_counts[j] = (int64_t)hl[j];
        }
        MRA_TRY(hipStreamSynchronize(s));
    }
    return nl;
}

/* every level of the reconstruction of a leaf set into P.U: tree nodes by
 * projection of the leaves, the others predicted from the level above */
static int tree_levels(Pyr& P, const uint64_t* keys, const double* values, int64_t n_leaves,
                       hipStream_t s) {
    const int d = P.d, J = P.J;
    const int B = 256;
    MRA_TRY(hipMemsetAsync(P.T, 0, (size_t)P.total, s));
    hipLaunchKernelGGL(k_scatter_leaves, dim3(blocks_for(n_leaves, B)), dim3(B), 0, s, P, d, keys,
                       values, n_leaves);
    for (int j = J; j >= 1; --j) {
        const int64_t np = (int64_t)1 << (d * (j - 1));
        if (d == 2) hipLaunchKernelGGL(k_tree_up<2>, dim3(blocks_for(np, B)), dim3(B), 0, s, P, j);
        else hipLaunchKernelGGL(k_tree_up<3>, dim3(blocks_for(np, B)), dim3(B), 0, s, P, j);
    }
    for (int j = 1; j <= J; ++j) {
        const int64_t np = (int64_t)1 << (d * (j - 1));
        if (d == 2) hipLaunchKernelGGL(k_fill_down<2>, dim3(blocks_for(np, B)), dim3(B), 0, s, P, j);
        else hipLaunchKernelGGL(k_fill_down<3>, dim3(blocks_for(np, B)), dim3(B), 0, s, P, j);
    }
    MRA_TRY(hipGetLastError());
    return 0;
}

static int upload_scale(const rd_mra_params* p, int32_t m, double* sc, hipStream_t s) {
    std::vector<double> hs(m, 1.0);
    if (p->scale) hs.assign(p->scale, p->scale + m);
    MRA_TRY(hipMemcpyAsync(sc, hs.data(), sizeof(double) * m, hipMemcpyHostToDevice, s));
    /* the host vector is released on return: wait for the copy */
    MRA_TRY(hipStreamSynchronize(s));
    return 0;
}

}  // namespace rd

using namespace rd;

extern "C" {

int64_t rd_mra_leaves(const double* fine, int32_t m, const rd_mra_params* p, uint64_t* keys,
                      double* values, int64_t capacity, int64_t* level_counts, void* hip_stream) {
    if (!mra_params_valid(p, m) || !fine || capacity < 0) {
        set_error("invalid MRA arguments");
        return RD_EINVAL;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    Pyr P{};
    double* sc = nullptr;
    unsigned* bcount = nullptr;
    unsigned long long* boff = nullptr;
    int64_t nb = 0;
    if (int r = setup_pyr(p, m, s, P, &sc, &bcount, &boff, &nb)) return r;
    if (int r = upload_scale(p, m, sc, s)) return r;
    const int d = P.d, J = P.J;
    const int64_t nfine = (int64_t)1 << (d * J);
    const int B = 256;
    const int64_t nbrick = nfine / kBrickCells;
    if (d == 2 && J >= Brick<2>::S)
        hipLaunchKernelGGL((k_morton_brick<2, true>), dim3((unsigned)nbrick), dim3(256), 0, s, fine, nullptr, P);
    else if (d == 3 && J >= Brick<3>::S)
        hipLaunchKernelGGL((k_morton_brick<3, true>), dim3((unsigned)nbrick), dim3(256), 0, s, fine, nullptr, P);
    else if (d == 2) hipLaunchKernelGGL(k_to_morton<2>, dim3(blocks_for(nfine, B)), dim3(B), 0, s, fine, P);
    else hipLaunchKernelGGL(k_to_morton<3>, dim3(blocks_for(nfine, B)), dim3(B), 0, s, fine, P);
    for (int j = J; j >= 1; --j) {
        const int64_t np = (int64_t)1 << (d * (j - 1));
        if (d == 2) hipLaunchKernelGGL(k_project<2>, dim3(blocks_for(np, B)), dim3(B), 0, s, P, j);
        else hipLaunchKernelGGL(k_project<3>, dim3(blocks_for(np, B)), dim3(B), 0, s, P, j);
    }
    return flags_and_leaves(P, p, s, sc, bcount, boff, nb, keys, values, capacity, level_counts);
}

int64_t rd_mra_reconstruct(const uint64_t* keys, const double* values, int64_t n_leaves,
                           int32_t m, const rd_mra_params* p, double* fine, void* hip_stream) {
    if (!mra_params_valid(p, m) || !fine || n_leaves < 1 || !keys || !values) {
        set_error("invalid MRA arguments");
        return RD_EINVAL;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    Pyr P{};
    double* sc = nullptr;
    unsigned* bcount = nullptr;
    unsigned long long* boff = nullptr;
    int64_t nb = 0;
    if (int r = setup_pyr(p, m, s, P, &sc, &bcount, &boff, &nb)) return r;
    if (int r = tree_levels(P, keys, values, n_leaves, s)) return r;
    const int d = P.d, J = P.J;
    const int64_t nfine = (int64_t)1 << (d * J);
    const int B = 256;
    const int64_t nbrick = nfine / kBrickCells;
    if (d == 2 && J >= Brick<2>::S)
        hipLaunchKernelGGL((k_morton_brick<2, false>), dim3((unsigned)nbrick), dim3(256), 0, s, nullptr, fine, P);
    else if (d == 3 && J >= Brick<3>::S)
        hipLaunchKernelGGL((k_morton_brick<3, false>), dim3((unsigned)nbrick), dim3(256), 0, s, nullptr, fine, P);
    else if (d == 2) hipLaunchKernelGGL(k_from_morton<2>, dim3(blocks_for(nfine, B)), dim3(B), 0, s, fine, P);
    else hipLaunchKernelGGL(k_from_morton<3>, dim3(blocks_for(nfine, B)), dim3(B), 0, s, fine, P);
    MRA_TRY(hipGetLastError());
    MRA_TRY(hipStreamSynchronize(s));
    return 0;
}

int64_t rd_mra_adapt(const uint64_t* keys, const double* values, int64_t n_leaves, int32_t m,
                     const rd_mra_params* p, uint64_t* out_keys, double* out_values,
                     int64_t capacity, int64_t* level_counts, void* hip_stream) {
    if (!mra_params_valid(p, m) || n_leaves < 1 || !keys || !values || capacity < 0) {
        set_error("invalid MRA arguments");
        return RD_EINVAL;
    }
    hipStream_t s = (hipStream_t)hip_stream;
    Pyr P{};
    double* sc = nullptr;
    unsigned* bcount = nullptr;
    unsigned long long* boff = nullptr;
    int64_t nb = 0;
    if (int r = setup_pyr(p, m, s, P, &sc, &bcount, &boff, &nb)) return r;
    if (int r = upload_scale(p, m, sc, s)) return r;
    if (int r = tree_levels(P, keys, values, n_leaves, s)) return r;
    return flags_and_leaves(P, p, s, sc, bcount, boff, nb, out_keys, out_values, capacity,
                            level_counts);
}

}  // extern "C"
