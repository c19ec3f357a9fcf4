"""Oracle of the diffusion step and of the Strang splitting step (numpy, FP64).

TEST INFRASTRUCTURE ONLY: used by the tests and never by the product path;
it shares no code with the GPU library.

What it computes (Descombes et al., §2):
- the diffusion operator A_eps of the semi-discrete system dU/dt = A_eps U +
  F(U): per species i, eps_i times the standard centred second-order
  Laplacian on the uniform cell-centred grid of [0, 1]^d, h = 1/N, with
  homogeneous Neumann boundary conditions (zero flux: a missing neighbour
  contributes nothing), 5 / 7 points in 2D / 3D (paper §2, §1 on the
  boundary conditions);
- the diffusion step D_dt by an explicit stabilised Runge-Kutta method.  The
  paper uses ROCK4 (§2.1, §3.3), whose recurrence coefficients are tabulated
  and not available here; in its place this oracle uses the second-order
  Runge-Kutta-Chebyshev method RKC (Sommeijer, Shampine & Verwer, J. Comput.
  Appl. Math. 88 (1997); van der Houwen & Sommeijer 1980) with damping
  eps = 2/13, written from its published three-term recurrence;
- the Strang step U_{n+1} = R_{dt/2} D_dt R_{dt/2} U_n (paper §2.1), with R
  the oracle's Radau5 reaction step.

Grid layout: states[i, c], c = x + nx (y + ny z) (x fastest).
"""
from __future__ import annotations

import math

import numpy as np

RKC_EPS = 2.0 / 13.0


# ---------------------------------------------------------------------------
# Chebyshev polynomials of the first kind and their first two derivatives at
# a point, by the three-term recurrence T_{j+1} = 2x T_j - T_{j-1}.
# ---------------------------------------------------------------------------
def chebyshev_values(s: int, x: float):
    T = np.zeros(s + 1)
    dT = np.zeros(s + 1)
    d2T = np.zeros(s + 1)
    T[0], dT[0], d2T[0] = 1.0, 0.0, 0.0
    if s >= 1:
        T[1], dT[1], d2T[1] = x, 1.0, 0.0
    for j in range(1, s):
        T[j + 1] = 2 * x * T[j] - T[j - 1]
        dT[j + 1] = 2 * T[j] + 2 * x * dT[j] - dT[j - 1]
        d2T[j + 1] = 4 * dT[j] + 2 * x * d2T[j] - d2T[j - 1]
    return T, dT, d2T


def rkc_coefficients(s: int, eps: float = RKC_EPS):
    """Coefficients of the s-stage RKC2 method (s >= 2):
        w0 = 1 + eps / s^2, w1 = T_s'(w0) / T_s''(w0),
        b_j = T_j''(w0) / T_j'(w0)^2 (j >= 2), b_0 = b_1 = b_2, a_j = 1 - b_j T_j(w0),
        mut_1 = b_1 w1,
        mu_j = 2 b_j w0 / b_{j-1}, nu_j = -b_j / b_{j-2}, mut_j = 2 b_j w1 / b_{j-1},
        gamt_j = -a_{j-1} mut_j                                  (j = 2..s)
    Stages: Y0 = y, Y1 = Y0 + mut_1 tau F(Y0),
        Yj = (1 - mu_j - nu_j) Y0 + mu_j Y_{j-1} + nu_j Y_{j-2}
             + mut_j tau F(Y_{j-1}) + gamt_j tau F(Y0),   y_new = Y_s.
    Returns dict with arrays indexed by stage j (entries 0/1 unused where
    undefined) and the scalars w0, w1, a_s, b_s."""
    if s < 2:
        raise ValueError("RKC needs s >= 2")
    w0 = 1.0 + eps / (s * s)
    T, dT, d2T = chebyshev_values(s, w0)
    w1 = dT[s] / d2T[s]
    b = np.zeros(s + 1)
    for j in range(2, s + 1):
        b[j] = d2T[j] / (dT[j] ** 2)
    b[0] = b[1] = b[2]
    a = 1.0 - b * T
    mu = np.zeros(s + 1)
    nu = np.zeros(s + 1)
    mut = np.zeros(s + 1)
    gamt = np.zeros(s + 1)
    mut[1] = b[1] * w1
    for j in range(2, s + 1):
        mu[j] = 2.0 * b[j] * w0 / b[j - 1]
        nu[j] = -b[j] / b[j - 2]
        mut[j] = 2.0 * b[j] * w1 / b[j - 1]
        gamt[j] = -a[j - 1] * mut[j]
    return {"s": s, "w0": w0, "w1": w1, "a_s": a[s], "b_s": b[s], "mu": mu, "nu": nu,
            "mut": mut, "gamt": gamt}


def rkc_stages(tau_rho: float) -> int:
    """Stage count for a step tau with spectral radius rho: the smallest s
    the RKC authors recommend, s = 1 + floor(sqrt(1 + 1.54 tau rho)), at
    least 2 (the stability interval grows like 0.65 s^2)."""
    return max(2, 1 + int(math.sqrt(1.0 + 1.54 * tau_rho)))


# ---------------------------------------------------------------------------
# Diffusion operator
# ---------------------------------------------------------------------------
def laplacian(u: np.ndarray, shape, h: float) -> np.ndarray:
    """Centred 5/7-point Laplacian of one species (flat, x fastest) on the
    cell-centred grid with homogeneous Neumann boundaries."""
    g = u.reshape(tuple(reversed(shape)))          # (ny, nx) or (nz, ny, nx)
    out = np.zeros_like(g)
    for ax in range(g.ndim):
        n = g.shape[ax]
        if n < 2:
            continue
        fwd = np.diff(g, axis=ax)                   # u[k+1] - u[k]
        lo = [slice(None)] * g.ndim
        hi = [slice(None)] * g.ndim
        lo[ax] = slice(0, n - 1)
        hi[ax] = slice(1, n)
        out[tuple(lo)] += fwd                       # neighbour above
        out[tuple(hi)] -= fwd                       # neighbour below
    return (out / (h * h)).ravel()


def spectral_radius_bound(diff, dim: int, h: float) -> float:
    """Gershgorin bound of rho(A_eps): each row of eps_i Lap_h has diagonal
    -2 d eps_i / h^2 and off-diagonal sum 2 d eps_i / h^2."""
    return 4.0 * dim * float(np.max(diff)) / (h * h)


def apply_A(states, shape, h, diff):
    return np.vstack([diff[i] * laplacian(states[i], shape, h) for i in range(states.shape[0])])


def diffusion_step(states, shape, h, diff, dt, stages: int | None = None):
    """D_dt: one RKC2 step of size dt for dU/dt = A_eps U; stage count from
    the Gershgorin bound unless given.  Returns (new states, s)."""
    diff = np.asarray(diff, dtype=np.float64)
    y0 = np.array(states, dtype=np.float64)
    s = stages or rkc_stages(dt * spectral_radius_bound(diff, len(shape), h))
    c = rkc_coefficients(s)
    F0 = apply_A(y0, shape, h, diff)
    y_prev2 = y0
    y_prev = y0 + c["mut"][1] * dt * F0
    for j in range(2, s + 1):
        Fj = apply_A(y_prev, shape, h, diff)
        y_new = ((1.0 - c["mu"][j] - c["nu"][j]) * y0 + c["mu"][j] * y_prev
                 + c["nu"][j] * y_prev2 + c["mut"][j] * dt * Fj + c["gamt"][j] * dt * F0)
        y_prev2, y_prev = y_prev, y_new
    return y_prev, s


def strang_step(orc, states, shape, h, diff, dt, rtol, atol, kind, params, **ropts):
    """U_{n+1} = R_{dt/2} D_dt R_{dt/2} U_n with the oracle's Radau5 R.
    Returns (new states, stats of the two reaction halves, s)."""
    y, st1, r1 = orc.reaction_step(states, dt / 2, rtol, atol, kind, params, **ropts)
    y, s = diffusion_step(y, shape, h, diff, dt)
    y, st2, r2 = orc.reaction_step(y, dt / 2, rtol, atol, kind, params, **ropts)
    return y, (st1, st2), (r1, r2), s
