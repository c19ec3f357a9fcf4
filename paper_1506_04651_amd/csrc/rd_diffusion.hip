/*
 * rd_diffusion.hip -- the diffusion step D_dt of the Strang splitting scheme
 * (Descombes et al., §2.1): dU/dt = A_eps U, with A_eps the standard centred
 * second-order Laplacian times eps_i per species on a uniform cell-centred
 * grid of [0, 1]^d (5 / 7 points in 2D / 3D, §2) and homogeneous Neumann
 * boundaries (§1), advanced by an explicit stabilised Runge-Kutta method.
 *
 * The paper uses ROCK4 (§2.1, §3.3).  Its recurrence coefficients are tabulated
 * and not at hand, so this library uses the second-order Runge-Kutta-Chebyshev
 * method (RKC: van der Houwen & Sommeijer 1980; Sommeijer, Shampine & Verwer
 * 1997) instead, a member of the same family whose coefficients follow from
 * Chebyshev polynomials in closed form.  With damping eps = 2/13 its real
 * stability interval grows like 0.65 s^2 with the stage count s, chosen from
 * the Gershgorin bound of the spectral radius as in the paper.
 *
 * One kernel per stage, HBM bound: stage j reads Y0, Y_{j-1} (with its stencil
 * neighbours, mostly from L2), Y_{j-2} and F0 = A Y0, and writes Y_j; with
 * rows of even length each thread takes two neighbouring cells.
 * Blocks are mapped so that each XCD works on a contiguous band of rows and
 * its L2 serves the row above and below.
 */
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rd_diffusion.h"

namespace rd {

/* Logical block index: blocks of one XCD (dispatched round-robin over the 8
 * XCDs) get a contiguous range; returns false for padding blocks. */
__device__ __forceinline__ bool xcd_block(unsigned nblocks_logical, unsigned& b) {
    const unsigned g = gridDim.x; /* a multiple of 8 */
    const unsigned per = g / 8u;
    b = (blockIdx.x % 8u) * per + blockIdx.x / 8u;
    return b < nblocks_logical;
}

/* eps_i * Laplacian of species plane u at cell c (x fastest) with zero-flux
 * boundaries: only existing neighbours contribute u_nb - u_c. */
template <int DIM>
__device__ __forceinline__ double lap(const double* __restrict__ u, const DiffGrid& g, int64_t c,
                                      int x, int y, int z) {
    const double uc = u[c];
    double s = 0.0;
    if (x > 0) s += u[c - 1] - uc;
    if (x < g.nx - 1) s += u[c + 1] - uc;
    if (y > 0) s += u[c - g.nx] - uc;
    if (y < g.ny - 1) s += u[c + g.nx] - uc;
    if (DIM == 3) {
        const int64_t pl = (int64_t)g.nx * g.ny;
        if (z > 0) s += u[c - pl] - uc;
        if (z < g.nz - 1) s += u[c + pl] - uc;
    }
    return s * g.ih2;
}

/* stage 1: F0 = A Y0 (kept for later stages), Y1 = Y0 + mut1 tau F0 */
template <int DIM>
__global__ void __launch_bounds__(256) k_rkc_first(const double* __restrict__ y0,
                                                   double* __restrict__ f0,
                                                   double* __restrict__ y1, DiffGrid g,
                                                   const double* __restrict__ eps, double mut1tau,
                                                   unsigned nblocks) {
    unsigned b;
    if (!xcd_block(nblocks, b)) return;
    const int64_t c = (int64_t)b * 256 + threadIdx.x;
    if (c >= g.n) return;
    const int sp = blockIdx.y;
    const int x = (int)(c % g.nx);
    const int64_t r = c / g.nx;
    const int y = (int)(r % g.ny);
    const int z = (int)(r / g.ny);
    const int64_t off = (int64_t)sp * g.n;
    const double f = eps[sp] * lap<DIM>(y0 + off, g, c, x, y, z);
    f0[off + c] = f;
    y1[off + c] = y0[off + c] + mut1tau * f;
}

/* stage j >= 2: Yj = (1 - mu - nu) Y0 + mu Yp + nu Ypp + mut tau A Yp + gamt tau F0.
 * Yj may be the storage of Y0 (and of Ypp = Y0 when s = 2) on the last stage:
 * those are read only at the cell being written. */
template <int DIM>
__global__ void __launch_bounds__(256) k_rkc_stage(const double* y0, const double* __restrict__ f0,
                                                   const double* __restrict__ yp, const double* ypp,
                                                   double* yj, DiffGrid g,
                                                   const double* __restrict__ eps, double c0,
                                                   double mu, double nu, double muttau,
                                                   double gamttau, unsigned nblocks) {
    unsigned b;
    if (!xcd_block(nblocks, b)) return;
    const int64_t c = (int64_t)b * 256 + threadIdx.x;
    if (c >= g.n) return;
    const int sp = blockIdx.y;
    const int x = (int)(c % g.nx);
    const int64_t r = c / g.nx;
    const int y = (int)(r % g.ny);
    const int z = (int)(r / g.ny);
    const int64_t off = (int64_t)sp * g.n;
    const double ap = eps[sp] * lap<DIM>(yp + off, g, c, x, y, z);
    yj[off + c] = c0 * y0[off + c] + mu * yp[off + c] + nu * ypp[off + c] + muttau * ap +
                  gamttau * f0[off + c];
}

/* Two cells per thread, c and c + 1 with c even: with an even row length a
 * pair never straddles a row, and every vector access except the two row ends
 * of the stencil moves 16 bytes (half the memory instructions of one cell per
 * thread).  Each cell's sums are formed in lap()'s order with the same
 * expressions, so the results are bitwise those of the one-cell kernels. */

/* eps_i * Laplacian of u at cells c and c + 1; uc returns their values */
template <int DIM>
__device__ __forceinline__ double2 lap_x2(const double* __restrict__ u, const DiffGrid& g, int64_t c,
                                          int x, int y, int z, double e, double2& uc) {
    uc = *reinterpret_cast<const double2*>(u + c);
    /* x - 1 of cell c, then x + 1 (cell c + 1, always inside: x is even) */
    double s0 = 0.0, s1 = 0.0;
    if (x > 0) s0 += u[c - 1] - uc.x;
    s0 += uc.y - uc.x;
    s1 += uc.x - uc.y;
    if (x + 1 < g.nx - 1) s1 += u[c + 2] - uc.y;
    if (y > 0) {
        const double2 v = *reinterpret_cast<const double2*>(u + c - g.nx);
        s0 += v.x - uc.x;
        s1 += v.y - uc.y;
    }
    if (y < g.ny - 1) {
        const double2 v = *reinterpret_cast<const double2*>(u + c + g.nx);
        s0 += v.x - uc.x;
        s1 += v.y - uc.y;
    }
    if (DIM == 3) {
        const int64_t pl = (int64_t)g.nx * g.ny;
        if (z > 0) {
            const double2 v = *reinterpret_cast<const double2*>(u + c - pl);
            s0 += v.x - uc.x;
            s1 += v.y - uc.y;
        }
        if (z < g.nz - 1) {
            const double2 v = *reinterpret_cast<const double2*>(u + c + pl);
            s0 += v.x - uc.x;
            s1 += v.y - uc.y;
        }
    }
    const double l0 = s0 * g.ih2, l1 = s1 * g.ih2;
    return make_double2(e * l0, e * l1);
}

template <int DIM>
__global__ void __launch_bounds__(256) k_rkc_first_x2(const double* __restrict__ y0,
                                                      double* __restrict__ f0,
                                                      double* __restrict__ y1, DiffGrid g,
                                                      const double* __restrict__ eps, double mut1tau,
                                                      unsigned nblocks) {
    unsigned b;
    if (!xcd_block(nblocks, b)) return;
    const int64_t c = 2 * ((int64_t)b * 256 + threadIdx.x);
    if (c >= g.n) return;
    const int sp = blockIdx.y;
    const int x = (int)(c % g.nx);
    const int64_t r = c / g.nx;
    const int y = (int)(r % g.ny);
    const int z = (int)(r / g.ny);
    const int64_t off = (int64_t)sp * g.n;
    double2 uc;
    const double2 f = lap_x2<DIM>(y0 + off, g, c, x, y, z, eps[sp], uc);
    *reinterpret_cast<double2*>(f0 + off + c) = f;
    double2 o;
    o.x = uc.x + mut1tau * f.x;
    o.y = uc.y + mut1tau * f.y;
    *reinterpret_cast<double2*>(y1 + off + c) = o;
}

template <int DIM>
__global__ void __launch_bounds__(256) k_rkc_stage_x2(const double* y0, const double* __restrict__ f0,
                                                      const double* __restrict__ yp, const double* ypp,
                                                      double* yj, DiffGrid g,
                                                      const double* __restrict__ eps, double c0,
                                                      double mu, double nu, double muttau,
                                                      double gamttau, unsigned nblocks) {
    unsigned b;
    if (!xcd_block(nblocks, b)) return;
    const int64_t c = 2 * ((int64_t)b * 256 + threadIdx.x);
    if (c >= g.n) return;
    const int sp = blockIdx.y;
    const int x = (int)(c % g.nx);
    const int64_t r = c / g.nx;
    const int y = (int)(r % g.ny);
    const int z = (int)(r / g.ny);
    const int64_t off = (int64_t)sp * g.n;
    double2 uc;
    const double2 ap = lap_x2<DIM>(yp + off, g, c, x, y, z, eps[sp], uc);
    const double2 a0 = *reinterpret_cast<const double2*>(y0 + off + c);
    const double2 a2 = *reinterpret_cast<const double2*>(ypp + off + c);
    const double2 ff = *reinterpret_cast<const double2*>(f0 + off + c);
    double2 o;
    o.x = c0 * a0.x + mu * uc.x + nu * a2.x + muttau * ap.x + gamttau * ff.x;
    o.y = c0 * a0.y + mu * uc.y + nu * a2.y + muttau * ap.y + gamttau * ff.y;
    *reinterpret_cast<double2*>(yj + off + c) = o;
}

hipError_t launch_rkc(int dim, const double* y0, double* out, double* f0, double* w0, double* w1,
                      double* w2, int m, const DiffGrid& g, const double* eps_dev, double mut1tau,
                      const RkcStage* st, int s, hipStream_t stream) {
    const unsigned nblocks = (unsigned)((g.n + 255) / 256);
    const unsigned padded = (nblocks + 7u) / 8u * 8u;
    const dim3 grid(padded, (unsigned)m), block(256);
    double* bufs[3] = {w0, w1, w2};
    /* Y1 -> bufs[0]; Yj -> bufs[(j-1) % 3]; the last stage writes out */
    double* y1 = bufs[0]; /* s >= 2 */
    /* two cells per thread when rows have an even length and every vector
     * is 16-byte aligned */
    const uintptr_t al = (uintptr_t)y0 | (uintptr_t)out | (uintptr_t)f0 | (uintptr_t)w0 |
                         (uintptr_t)w1 | (uintptr_t)w2;
    const bool x2 = g.nx % 2 == 0 && (al & 15u) == 0;
    const unsigned nb2 = (unsigned)((g.n / 2 + 255) / 256);
    const dim3 grid2((nb2 + 7u) / 8u * 8u, (unsigned)m);
    if (x2 && dim == 3)
        hipLaunchKernelGGL(k_rkc_first_x2<3>, grid2, block, 0, stream, y0, f0, y1, g, eps_dev, mut1tau, nb2);
    else if (x2)
        hipLaunchKernelGGL(k_rkc_first_x2<2>, grid2, block, 0, stream, y0, f0, y1, g, eps_dev, mut1tau, nb2);
    else if (dim == 3)
        hipLaunchKernelGGL(k_rkc_first<3>, grid, block, 0, stream, y0, f0, y1, g, eps_dev, mut1tau, nblocks);
    else
        hipLaunchKernelGGL(k_rkc_first<2>, grid, block, 0, stream, y0, f0, y1, g, eps_dev, mut1tau, nblocks);
    const double* ypp = y0;
    const double* yp = y1;
    for (int j = 2; j <= s; ++j) {
        double* yj = (j == s) ? out : bufs[(j - 1) % 3];
        const RkcStage& c = st[j];
        if (x2 && dim == 3)
            hipLaunchKernelGGL(k_rkc_stage_x2<3>, grid2, block, 0, stream, y0, f0, yp, ypp, yj, g,
                               eps_dev, c.c0, c.mu, c.nu, c.muttau, c.gamttau, nb2);
        else if (x2)
            hipLaunchKernelGGL(k_rkc_stage_x2<2>, grid2, block, 0, stream, y0, f0, yp, ypp, yj, g,
                               eps_dev, c.c0, c.mu, c.nu, c.muttau, c.gamttau, nb2);
        else if (dim == 3)
            hipLaunchKernelGGL(k_rkc_stage<3>, grid, block, 0, stream, y0, f0, yp, ypp, yj, g, eps_dev,
                               c.c0, c.mu, c.nu, c.muttau, c.gamttau, nblocks);
        else
            hipLaunchKernelGGL(k_rkc_stage<2>, grid, block, 0, stream, y0, f0, yp, ypp, yj, g, eps_dev,
                               c.c0, c.mu, c.nu, c.muttau, c.gamttau, nblocks);
        ypp = yp;
        yp = yj;
    }
    return hipGetLastError();
}

}  // namespace rd
