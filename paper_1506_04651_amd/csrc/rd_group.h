/*
 * rd_group.h -- cross-lane helpers for kernels in which a 16-lane group of a
 * wave64 shares one cell (one DPP row per cell: lanes 0-15, 16-31, 32-47,
 * 48-63).  Lane q of a group owns row q of the cell's m x m matrices.
 */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rd {

constexpr int kGroup = 16;

__device__ __forceinline__ unsigned grp_lane() { return __lane_id() & 15u; }
__device__ __forceinline__ unsigned grp_base() { return __lane_id() & 48u; }

/* The 16 ballot bits of this lane's group. */
__device__ __forceinline__ unsigned grp_bits(bool pred) {
    return (unsigned)(__ballot(pred) >> grp_base()) & 0xFFFFu;
}

/* Broadcast lane SRC of every 16-lane row to the whole row (DPP
 * row_newbcast); every lane of the row must be active. */
template <int SRC>
__device__ __forceinline__ int bcast_i(int v) {
    return __builtin_amdgcn_update_dpp(v, v, 0x150 + SRC, 0xF, 0xF, false);
}

__device__ __forceinline__ float bcast_dyn(float v, int src) {
    int x = __float_as_int(v);
    switch (src) {
#define RD_BC(J) case J: x = bcast_i<J>(x); break;
        RD_BC(0) RD_BC(1) RD_BC(2) RD_BC(3) RD_BC(4) RD_BC(5) RD_BC(6) RD_BC(7)
        RD_BC(8) RD_BC(9) RD_BC(10) RD_BC(11) RD_BC(12) RD_BC(13) RD_BC(14) RD_BC(15)
#undef RD_BC
    }
    return __int_as_float(x);
}

/* src must be a compile-time constant after unrolling (the switch folds). */
__device__ __forceinline__ double bcast_dyn(double v, int src) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    switch (src) {
#define RD_BC(J) case J: lo = bcast_i<J>(lo); hi = bcast_i<J>(hi); break;
        RD_BC(0) RD_BC(1) RD_BC(2) RD_BC(3) RD_BC(4) RD_BC(5) RD_BC(6) RD_BC(7)
        RD_BC(8) RD_BC(9) RD_BC(10) RD_BC(11) RD_BC(12) RD_BC(13) RD_BC(14) RD_BC(15)
#undef RD_BC
    }
    return __hiloint2double(hi, lo);
}

/* Value of lane `src` (0..15) of this lane's group, src data dependent. */
__device__ __forceinline__ double grp_shfl(double v, int src) {
    return __shfl(v, (int)grp_base() + src, 64);
}
__device__ __forceinline__ float grp_shfl(float v, int src) {
    return __shfl(v, (int)grp_base() + src, 64);
}
__device__ __forceinline__ int grp_shfl(int v, int src) {
    return __shfl(v, (int)grp_base() + src, 64);
}

/* Sum / max over the group by an xor butterfly: every lane adds the same two
 * operands at every stage (a + b == b + a), so all 16 lanes end with the
 * bitwise-identical result and take identical decisions. */
__device__ __forceinline__ double grp_sum(double v) {
    v += __shfl_xor(v, 8, 16);
    v += __shfl_xor(v, 4, 16);
    v += __shfl_xor(v, 2, 16);
    v += __shfl_xor(v, 1, 16);
    return v;
}
template <typename T>
__device__ __forceinline__ T grp_max(T v) {
    v = fmax(v, __shfl_xor(v, 8, 16));
    v = fmax(v, __shfl_xor(v, 4, 16));
    v = fmax(v, __shfl_xor(v, 2, 16));
    v = fmax(v, __shfl_xor(v, 1, 16));
    return v;
}

}  // namespace rd
