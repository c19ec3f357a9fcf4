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
 * neighbours, mostly from L2), Y_{j-2} and F0 = A Y0, and writes Y_j.
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

hipError_t launch_rkc(int dim, const double* y0, double* out, double* f0, double* w0, double* w1,
                      double* w2, int m, const DiffGrid& g, const double* eps_dev, double mut1tau,
                      const RkcStage* st, int s, hipStream_t stream) {
    const unsigned nblocks = (unsigned)((g.n + 255) / 256);
    const unsigned padded = (nblocks + 7u) / 8u * 8u;
    const dim3 grid(padded, (unsigned)m), block(256);
    double* bufs[3] = {w0, w1, w2};
    /* Y1 -> bufs[0]; Yj -> bufs[(j-1) % 3]; the last stage writes out */
    double* y1 = bufs[0]; /* s >= 2 */
    if (dim == 3)
        hipLaunchKernelGGL(k_rkc_first<3>, grid, block, 0, stream, y0, f0, y1, g, eps_dev, mut1tau, nblocks);
    else
        hipLaunchKernelGGL(k_rkc_first<2>, grid, block, 0, stream, y0, f0, y1, g, eps_dev, mut1tau, nblocks);
    const double* ypp = y0;
    const double* yp = y1;
    for (int j = 2; j <= s; ++j) {
        double* yj = (j == s) ? out : bufs[(j - 1) % 3];
        const RkcStage& c = st[j];
        if (dim == 3)
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
