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
/* The same, read from the hardware at this point: the compiler can neither
 * hoist it out of a loop nor keep it live (and spill it) across one. */
__device__ __forceinline__ int grp_lane_here() {
    int v;
    __asm__ volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(v));
    return v & 15;
}
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

/* src must be a compile-time constant after unrolling (the switch folds).
 * One 64-bit DPP move (row_newbcast takes 64-bit operands on this chip). */
template <int SRC>
__device__ __forceinline__ long bcast_l(long v) {
    return __builtin_amdgcn_update_dpp(0l, v, 0x150 + SRC, 0xF, 0xF, true);
}
__device__ __forceinline__ double bcast_dyn(double v, int src) {
    long x = __double_as_longlong(v);
    switch (src) {
#define RD_BC(J) case J: x = bcast_l<J>(x); break;
        RD_BC(0) RD_BC(1) RD_BC(2) RD_BC(3) RD_BC(4) RD_BC(5) RD_BC(6) RD_BC(7)
        RD_BC(8) RD_BC(9) RD_BC(10) RD_BC(11) RD_BC(12) RD_BC(13) RD_BC(14) RD_BC(15)
#undef RD_BC
    }
    return __longlong_as_double(x);
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

/* Lane exchanges inside a 16-lane row by DPP: xor 1 and xor 2 (quad
 * permutes), then the half-row mirror (i <-> 7 - i) and the row mirror
 * (i <-> 15 - i).  Applied in this order they form a butterfly over the 16
 * lanes: every partner map is an involution and the values being combined are
 * already equal within the blocks they come from. */
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, true);
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const int lo = dpp_i<CTRL>(__double2loint(v)), hi = dpp_i<CTRL>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

/* Sum over the group: at every stage each lane adds the same two operands as
 * its partner (a + b == b + a), so all 16 lanes end with the bitwise-identical
 * result and take identical decisions.  Every lane of the row must be active. */
__device__ __forceinline__ double grp_sum(double v) {
    v += dpp_d<kDppXor1>(v);
    v += dpp_d<kDppXor2>(v);
    v += dpp_d<kDppHalfMirror>(v);
    v += dpp_d<kDppMirror>(v);
    return v;
}
/* Maximum of an unsigned key over the group (same butterfly). */
__device__ __forceinline__ unsigned grp_max_u(unsigned v) {
    v = max(v, (unsigned)dpp_i<kDppXor1>((int)v));
    v = max(v, (unsigned)dpp_i<kDppXor2>((int)v));
    v = max(v, (unsigned)dpp_i<kDppHalfMirror>((int)v));
    v = max(v, (unsigned)dpp_i<kDppMirror>((int)v));
    return v;
}

/* Ordering key of a non-negative magnitude: its bit pattern (float) or the
 * high word of it (double: sign, exponent and 20 fraction bits), which orders
 * non-negative values monotonically; ties at that resolution go to the lowest
 * lane, so the chosen pivot is within a factor 1 + 2^-20 of the largest. */
__device__ __forceinline__ unsigned mag_key(float m) { return __float_as_uint(m); }
__device__ __forceinline__ unsigned mag_key(double m) { return (unsigned)__double2hiint(m); }

}  // namespace rd
