"""Seeded synthetic workloads for the reaction substep.

This module holds input generators only -- no integrator arithmetic -- so
that the GPU path and the CPU oracle can be fed identical inputs.

The paper's own inputs are leaf sets of an adaptive multiresolution grid for
the BZ model (Descombes et al. §1 model II, §4.1): localized reaction fronts on
a near-equilibrium background, with 80-83 % of the fine grid compressed away
(§4.1).  None of those leaf sets is available, so the generators below build
fields with that structure: tanh fronts between a plateau at the Oregonator
steady state and an excited state, plus small noise, stored one array per
species (paper §3.2), cells in Morton order where the lattice is 3D.

Every generator returns a ``Workload`` with ``states`` as a float64 array of
shape [m, n] (``states[i, c]`` = species i of cell c).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

KIND_OREGONATOR = 1
KIND_KINETICS = 2
KIND_NAGUMO = 3
KIND_LINEAR = 4
KIND_ROBERTSON = 5
KIND_BYTECODE = 6

# register-program opcodes of the bytecode model (format in include/rd.h)
BC_ADD, BC_SUB, BC_MUL, BC_DIV, BC_NEG, BC_EXP, BC_LOG, BC_POW, BC_OUT = range(1, 10)

# Oregonator (BZ) constants of the benchmark: da/dt = (-q a - a b + f c)/mu,
# db/dt = (q a - a b + b(1-b))/eps, dc/dt = b - c.  The paper prints q = 0.02
# (§1, model II); the benchmark runs q = 2e-3 with the same eps, mu, f.
OREG_EPS, OREG_MU, OREG_F, OREG_Q = 1e-2, 1e-5, 1.6, 2e-3
OREG_PARAMS = np.array([OREG_EPS, OREG_MU, OREG_F, OREG_Q])
OREG_PARAMS_PAPER = np.array([OREG_EPS, OREG_MU, OREG_F, 0.02])


@dataclasses.dataclass
class Workload:
    name: str
    states: np.ndarray          # [m, n] float64
    kind: int
    params: np.ndarray          # flat float64
    dt: float
    rtol: float
    atol: float
    info: dict = dataclasses.field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.states.shape[0])

    @property
    def n(self) -> int:
        return int(self.states.shape[1])

    def subset(self, idx) -> "Workload":
        return dataclasses.replace(self, name=f"{self.name}[sample]",
                                   states=np.ascontiguousarray(self.states[:, idx]))


def oregonator_plateau(params=OREG_PARAMS) -> np.ndarray:
    """Rest state used as the background plateau: the positive root of
    f1 = f2 = f3 = 0 (c = b, a = f b/(q + b), b^2 + (f+q-1) b - q(1+f) = 0)."""
    _, _, f, q = params
    s = f + q - 1.0
    b = 0.5 * (-s + math.sqrt(s * s + 4.0 * q * (f + 1.0)))
    return np.array([f * b / (q + b), b, b])


def oregonator_excited(params=OREG_PARAMS) -> np.ndarray:
    """Excited plateau: b = 1, c = 0.1 and a on its fast manifold f c/(q + b)."""
    _, _, f, q = params
    return np.array([f * 0.1 / (q + 1.0), 1.0, 0.1])


def _noise_clip(rng, u, sigma=1e-3):
    u = u + rng.normal(0.0, sigma, size=u.shape)
    return np.ascontiguousarray(np.maximum(u, 0.0))


# --------------------------------------------------------------------------
# 1D front profile, 4096 cells, dt = 1/256, rtol = atol = 1e-5
# --------------------------------------------------------------------------
def oregonator_1d(n: int = 4096, seed: int = 1, dt: float = 1.0 / 256,
                  rtol: float = 1e-5, atol: float = 1e-5,
                  params=OREG_PARAMS) -> Workload:
    rng = np.random.default_rng(seed)
    x = (np.arange(n) + 0.5) / n
    p = np.sort(rng.uniform(0.05, 0.95, 4))
    delta = 4.0 / 4096
    w = np.zeros(n)
    for j, pj in enumerate(p):
        w += (1.0 if j % 2 == 0 else -1.0) * 0.5 * (1.0 + np.tanh((x - pj) / delta))
    R, E = oregonator_plateau(params), oregonator_excited(params)
    u = R[:, None] + w[None, :] * (E - R)[:, None]
    return Workload("oregonator_1d_4096", _noise_clip(rng, u), KIND_OREGONATOR,
                    np.asarray(params, float).copy(), dt, rtol, atol,
                    {"fronts": p.tolist()})


# --------------------------------------------------------------------------
# Spiral fields (2D) and twisted scroll waves (3D)
# --------------------------------------------------------------------------
def _spiral_state(s, lam, half_width, params, rng):
    """States for signed front distance s (cells): a tanh front of half width
    `half_width` from the rest plateau (s < 0) to the excited plateau (s > 0),
    an excited band whose recovery variable c grows linearly behind the front,
    and the rest plateau elsewhere."""
    R, E = oregonator_plateau(params), oregonator_excited(params)
    front = np.abs(s) <= half_width
    excited = (~front) & (s > 0)
    n = s.size
    u = np.repeat(R[:, None], n, axis=1)
    prof = 0.5 * (1.0 + np.tanh(s[front] / (0.5 * half_width)))
    u[:, front] = R[:, None] + prof[None, :] * (E - R)[:, None]
    if excited.any():
        ramp = (s[excited] - half_width) / max(lam / 2 - half_width, 1e-9)
        c = E[2] + 0.4 * ramp
        u[0, excited] = E[0]
        u[1, excited] = E[1]
        u[2, excited] = c
    return _noise_clip(rng, u), front


def _signed_phase_distance(psi, lam):
    """psi in [0, 1): signed distance in cells to the nearest front psi = 0."""
    return lam * np.where(psi < 0.5, psi, psi - 1.0)


def oregonator_2d(side: int = 512, seed: int = 2, dt: float = 1.0 / 64,
                  rtol: float = 1e-5, atol: float = 1e-8, lam: float = 35.0,
                  params=OREG_PARAMS) -> Workload:
    """512 x 512 spiral-front field; 20 % of cells lie within 3 cells of a
    front (a 7-cell band out of a 35-cell wavelength)."""
    rng = np.random.default_rng(seed)
    cx, cy = side / 2 + rng.uniform(-64, 64, 2)
    iy, ix = np.mgrid[0:side, 0:side]
    dx, dy = ix + 0.5 - cx, iy + 0.5 - cy
    r = np.hypot(dx, dy)
    th = np.arctan2(dy, dx)
    psi = np.mod(r / lam - th / (2 * np.pi), 1.0).ravel()
    s = _signed_phase_distance(psi, lam)
    u, front = _spiral_state(s, lam, 3.5, params, rng)
    frac = float(front.mean())
    # the band share converges to 7/35 as the grid grows; small test grids
    # see a few wavelengths only
    assert abs(frac - 0.20) <= (0.01 if side >= 256 else 0.03), frac
    return Workload(f"oregonator_2d_{side}x{side}", u, KIND_OREGONATOR,
                    np.asarray(params, float).copy(), dt, rtol, atol,
                    {"front_fraction": frac, "centre": (float(cx), float(cy))})


def _morton3(x, y, z, bits):
    code = np.zeros(x.shape, dtype=np.int64)
    for b in range(bits):
        code |= ((x >> b) & 1).astype(np.int64) << (3 * b)
        code |= ((y >> b) & 1).astype(np.int64) << (3 * b + 1)
        code |= ((z >> b) & 1).astype(np.int64) << (3 * b + 2)
    return code


def oregonator_3d(side: int = 160, n_total: int = 1 << 22, seed: int = 3,
                  dt: float = 1.0 / 64, rtol: float = 1e-5, atol: float = 1e-8,
                  lam: float = 60.0, params=OREG_PARAMS,
                  check: bool = True) -> Workload:
    """160^3 twisted scroll wave in Morton order, 5 % front cells (within one
    cell of a front: a 3-cell band out of a 60-cell wavelength), padded to
    n_total cells by sampling the lattice with replacement."""
    rng = np.random.default_rng(seed)
    cx, cy = side / 2 + rng.uniform(-side / 8, side / 8, 2)
    twist = rng.uniform(0.5, 1.5)
    iz, iy, ix = np.meshgrid(np.arange(side), np.arange(side), np.arange(side),
                             indexing="ij")
    dx, dy = ix + 0.5 - cx, iy + 0.5 - cy
    r = np.hypot(dx, dy)
    th = np.arctan2(dy, dx) + 2 * np.pi * twist * (iz + 0.5) / side
    psi = np.mod(r / lam - th / (2 * np.pi), 1.0)
    order = np.argsort(_morton3(ix.ravel(), iy.ravel(), iz.ravel(), 8), kind="stable")
    s = _signed_phase_distance(psi.ravel()[order], lam)
    del iz, iy, ix, dx, dy, r, th, psi
    u, front = _spiral_state(s, lam, 1.5, params, rng)
    n_lat = u.shape[1]
    if n_total > n_lat:
        extra = rng.integers(0, n_lat, n_total - n_lat)
        u = np.ascontiguousarray(np.concatenate([u, u[:, extra]], axis=1))
        front = np.concatenate([front, front[extra]])
    elif n_total < n_lat:
        u = np.ascontiguousarray(u[:, :n_total])
        front = front[:n_total]
    frac = float(front.mean())
    if check:
        assert abs(frac - 0.05) <= 0.01, frac
    return Workload(f"oregonator_3d_{side}cubed_{u.shape[1]}", u, KIND_OREGONATOR,
                    np.asarray(params, float).copy(), dt, rtol, atol,
                    {"front_fraction": frac, "twist": float(twist)})


# --------------------------------------------------------------------------
# m = 16 synthetic stiff kinetics
# --------------------------------------------------------------------------
def kinetics_matrices(m: int = 16, seed: int = 4, k_density: float = 0.3,
                      g_density: float = 0.2, rng=None):
    """K: column-conserving rate matrix (off-diagonals 10^U(-1,5) with
    probability k_density, K_jj = -sum_{i != j} K_ij so 1^T K = 0).
    G: nonnegative, entries 10^U(-2,3) with probability g_density."""
    rng = np.random.default_rng(seed) if rng is None else rng
    K = np.where(rng.random((m, m)) < k_density, 10.0 ** rng.uniform(-1, 5, (m, m)), 0.0)
    np.fill_diagonal(K, 0.0)
    np.fill_diagonal(K, -K.sum(axis=0))
    G = np.where(rng.random((m, m)) < g_density, 10.0 ** rng.uniform(-2, 3, (m, m)), 0.0)
    return K, G


def kinetics16(n: int = 1 << 20, seed: int = 4, dt: float = 1e-2,
               rtol: float = 1e-6, atol: float = 1e-10, m: int = 16,
               zero_g: bool = False) -> Workload:
    rng = np.random.default_rng(seed)
    K, G = kinetics_matrices(m, rng=rng)
    if zero_g:
        G = np.zeros_like(G)
    u = 10.0 ** rng.uniform(-8, 0, (m, n))
    params = np.concatenate([K.ravel(), G.ravel()])
    return Workload(f"kinetics{m}_{n}", np.ascontiguousarray(u), KIND_KINETICS,
                    params, dt, rtol, atol, {"K": K, "G": G})


# --------------------------------------------------------------------------
# Serving stream
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Request:
    t_arrival: float
    pool: str
    idx: np.ndarray
    dt: float


def serving_stream(n_requests: int = 2000, seed: int = 5, mean_gap: float = 5e-3,
                   pool_sizes=None):
    """Poisson arrivals (exponential gaps, mean 5 ms), sizes floor(10^U(3,6))
    cells, generator uniform over the 2D / 3D Oregonator and m=16 pools, dt
    uniform over {1/256, 1/64, 1e-2}.  Returns a list of Request (cell indices
    into the chosen pool, drawn with replacement when needed)."""
    rng = np.random.default_rng(seed)
    pool_sizes = pool_sizes or {"oreg2d": 512 * 512, "oreg3d": 1 << 22, "kin16": 1 << 20}
    pools = ["oreg2d", "oreg3d", "kin16"]
    t = 0.0
    out = []
    for _ in range(n_requests):
        t += rng.exponential(mean_gap)
        n = int(math.floor(10.0 ** rng.uniform(3, 6)))
        pool = pools[int(rng.integers(0, 3))]
        size = pool_sizes[pool]
        if n <= size:
            start = int(rng.integers(0, size - n + 1))
            idx = np.arange(start, start + n)
        else:
            idx = rng.integers(0, size, n)
        dt = [1.0 / 256, 1.0 / 64, 1e-2][int(rng.integers(0, 3))]
        out.append(Request(t, pool, idx, dt))
    return out


def _program(m, consts, code):
    """Flatten (constants, [(op, d, a, b), ...]) into the bytecode params."""
    out = [float(len(code)), float(len(consts))] + [float(c) for c in consts]
    for ins in code:
        out += [float(v) for v in ins]
    return np.array(out)


def oregonator_program(params=OREG_PARAMS) -> np.ndarray:
    """The BZ right-hand side (paper §1, model II) as a register program,
    operation for operation the same as the closed form
    f1 = ((-q) a - a b + f c) / mu, f2 = (q a - a b + b (1 - b)) / eps,
    f3 = b - c  (registers: 0 a, 1 b, 2 c, 3 -q, 4 q, 5 f, 6 mu, 7 eps, 8 one)."""
    eps, mu, f, q = (float(v) for v in params)
    consts = [-q, q, f, mu, eps, 1.0]
    code = [(BC_MUL, 9, 3, 0), (BC_MUL, 10, 0, 1), (BC_SUB, 11, 9, 10), (BC_MUL, 12, 5, 2),
            (BC_ADD, 13, 11, 12), (BC_DIV, 14, 13, 6), (BC_OUT, 0, 14, 0),
            (BC_MUL, 15, 4, 0), (BC_SUB, 16, 15, 10), (BC_SUB, 17, 8, 1), (BC_MUL, 18, 1, 17),
            (BC_ADD, 19, 16, 18), (BC_DIV, 20, 19, 7), (BC_OUT, 1, 20, 0),
            (BC_SUB, 21, 1, 2), (BC_OUT, 2, 21, 0)]
    return _program(3, consts, code)


def robertson_program(k=(0.04, 1e4, 3e7)) -> np.ndarray:
    """Robertson kinetics as a register program: f1 = (-k1) u1 + k2 u2 u3,
    f2 = k1 u1 - k2 u2 u3 - k3 u2 u2, f3 = k3 u2 u2
    (registers: 0..2 u, 3 -k1, 4 k1, 5 k2, 6 k3)."""
    k1, k2, k3 = (float(v) for v in k)
    consts = [-k1, k1, k2, k3]
    code = [(BC_MUL, 7, 5, 1), (BC_MUL, 8, 7, 2),          # k2 u2 u3
            (BC_MUL, 9, 6, 1), (BC_MUL, 10, 9, 1),         # k3 u2 u2
            (BC_MUL, 11, 3, 0), (BC_ADD, 12, 11, 8), (BC_OUT, 0, 12, 0),
            (BC_MUL, 13, 4, 0), (BC_SUB, 14, 13, 8), (BC_SUB, 15, 14, 10), (BC_OUT, 1, 15, 0),
            (BC_OUT, 2, 10, 0)]
    return _program(3, consts, code)


def nagumo_program(k=1.0) -> np.ndarray:
    """NAGUMO (paper §1, model I) f = k u^2 (1 - u) as ((k u) u) (1 - u)
    (registers: 0 u, 1 k, 2 one)."""
    code = [(BC_MUL, 3, 1, 0), (BC_MUL, 4, 3, 0), (BC_SUB, 5, 2, 0), (BC_MUL, 6, 4, 5),
            (BC_OUT, 0, 6, 0)]
    return _program(1, [float(k), 1.0], code)


def oregonator_2d_paper(side: int = 1024, seed: int = 6, dt: float = 5e-4,
                        rtol: float = 1e-5, atol: float = 1e-8) -> Workload:
    """The spiral-front field with the paper's BZ constants (q = 0.02, §1)
    on a 1024 x 1024 grid, and the paper's reaction substep for BZ:
    dt = Delta t / 2 with Delta t = 1e-3 (§2.1).  The setting of the paper's
    complexity histogram (Appendix A).  With q = 0.02 the kinetics has a limit
    cycle and no stable rest state, so these states are not yet on the slow
    manifold: the histogram is taken after a relaxation of the field."""
    w = oregonator_2d(side=side, seed=seed, dt=dt, rtol=rtol, atol=atol,
                      params=OREG_PARAMS_PAPER)
    w.name = f"oregonator_2d_paper_q_{side}x{side}"
    return w


def sample_indices(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct sorted cell indices in [0, n)."""
    rng = np.random.default_rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, size=k, replace=False))


CONFIGS = {
    "oregonator_1d": oregonator_1d,
    "oregonator_2d": oregonator_2d,
    "oregonator_3d": oregonator_3d,
    "kinetics16": kinetics16,
    "oregonator_2d_paper": oregonator_2d_paper,
}
