/*
 * rd_diffusion.h -- interface between the diffusion-step host code
 * (rd_strang.cpp) and its kernels (rd_diffusion.hip).
 */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rd {

struct DiffGrid {
    int nx, ny, nz;
    int64_t n;  /* cells per species */
    double ih2; /* 1 / h^2 */
};

/* Weights of RKC stage j >= 2:
 * Y_j = c0 Y0 + mu Y_{j-1} + nu Y_{j-2} + muttau A Y_{j-1} + gamttau A Y0 */
struct RkcStage {
    double c0, mu, nu, muttau, gamttau;
};

/* Enqueue the s stages (s >= 2) of one RKC step of y0 on `stream`; the result
 * goes to out, which may be y0 itself (the last stage reads y0 only at the
 * cell it writes).  f0 and w0..w2 are m*n-double work vectors, eps_dev the m
 * diffusion coefficients on the device, st[2..s] the stage weights. */
hipError_t launch_rkc(int dim, const double* y0, double* out, double* f0, double* w0, double* w1,
                      double* w2, int m, const DiffGrid& g, const double* eps_dev, double mut1tau,
                      const RkcStage* st, int s, hipStream_t stream);

}  // namespace rd
