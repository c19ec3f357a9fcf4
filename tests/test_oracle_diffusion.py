"""Pins of the diffusion / Strang oracle (CPU).

- RKC coefficients: the stage recurrence applied to y' = lambda y reproduces
  the method's defining stability polynomial P_s(z) = a_s + b_s T_s(w0 + w1 z)
  evaluated independently (numpy's Chebyshev series), is consistent to second
  order (P_s(z) = 1 + z + z^2/2 + O(z^3)), and is bounded by 1 on the real
  interval the stage-count rule promises.
- Laplacian: annihilates constants, conserves the total (zero-flux
  boundaries), and has the cosine modes of the Neumann problem as exact
  eigenvectors with eigenvalues -(4/h^2) sin^2(k pi / 2N) per direction.
- Diffusion step on a cosine mode = P_s(tau lambda) times the mode, within
  O((tau lambda)^3) of exp(tau lambda); mass conserved.
- Strang step: second-order self-convergence on a smooth Nagumo problem.
"""
import numpy as np
import pytest
from numpy.polynomial import chebyshev as C

from oracle import diffusion as D
from paper_1506_04651_amd import workloads as W


def stage_recurrence_scalar(s, z):
    c = D.rkc_coefficients(s)
    y0 = 1.0
    prev2, prev = y0, y0 + c["mut"][1] * z * y0
    for j in range(2, s + 1):
        new = ((1 - c["mu"][j] - c["nu"][j]) * y0 + c["mu"][j] * prev + c["nu"][j] * prev2
               + c["mut"][j] * z * prev + c["gamt"][j] * z * y0)
        prev2, prev = prev, new
    return prev


@pytest.mark.parametrize("s", [2, 3, 5, 10, 31])
def test_rkc_stability_polynomial(s):
    c = D.rkc_coefficients(s)
    Ts = np.zeros(s + 1)
    Ts[s] = 1.0                       # T_s as a Chebyshev series
    for z in np.linspace(-0.6 * s * s, 0.0, 37):
        want = c["a_s"] + c["b_s"] * C.chebval(c["w0"] + c["w1"] * z, Ts)
        got = stage_recurrence_scalar(s, z)
        assert abs(got - want) <= 1e-11 * max(1.0, abs(want)), (s, z)


@pytest.mark.parametrize("s", [2, 4, 9, 20])
def test_rkc_second_order(s):
    for z in [-1e-2, -2e-3, 1e-3]:
        p = stage_recurrence_scalar(s, z)
        assert abs(p - (1 + z + z * z / 2)) <= 2.0 * s ** 4 * abs(z) ** 3, (s, z)
    # and not third order in general (the z^3 coefficient differs from 1/6)
    z = -1e-2
    assert abs(stage_recurrence_scalar(5, z) - np.exp(z)) > 1e-9


@pytest.mark.parametrize("tau_rho", [0.5, 3.0, 21.0, 400.0, 5000.0])
def test_rkc_stage_rule_is_stable(tau_rho):
    s = D.rkc_stages(tau_rho)
    for z in np.linspace(-tau_rho, 0.0, 2001):
        assert abs(stage_recurrence_scalar(s, z)) <= 1.0 + 1e-12, (s, z)


@pytest.mark.parametrize("shape", [(16, 12), (8, 6, 5)])
def test_laplacian_constants_mass_and_modes(shape):
    h = 1.0 / shape[0]
    n = int(np.prod(shape))
    assert np.allclose(D.laplacian(np.full(n, 3.7), shape, h), 0.0, atol=1e-12)
    rng = np.random.default_rng(1)
    u = rng.normal(size=n)
    assert abs(D.laplacian(u, shape, h).sum()) <= 1e-9 * np.abs(u).sum() / h ** 2
    # Neumann modes: prod_d cos(k_d pi (x_d + 1/2) / N_d)
    ks = [1, 2, 3][:len(shape)]
    grids = np.meshgrid(*[np.arange(N) for N in reversed(shape)], indexing="ij")
    mode = np.ones(grids[0].shape)
    lam = 0.0
    for d, N in enumerate(reversed(shape)):
        k = ks[len(shape) - 1 - d]
        mode = mode * np.cos(k * np.pi * (grids[d] + 0.5) / N)
        lam += -(4.0 / h ** 2) * np.sin(k * np.pi / (2 * N)) ** 2
    got = D.laplacian(mode.ravel(), shape, h)
    assert np.allclose(got, lam * mode.ravel(), rtol=0, atol=1e-9 * abs(lam))


def test_diffusion_step_on_a_mode_and_mass():
    shape, h, eps = (32, 32), 1.0 / 32, 2.5e-3
    x = (np.arange(32) + 0.5) / 32
    mode = np.outer(np.cos(2 * np.pi * x), np.cos(np.pi * x)).ravel()  # (y, x) order
    lam = eps * (-(4 / h ** 2) * np.sin(np.pi / 64) ** 2 - (4 / h ** 2) * np.sin(2 * np.pi / 64) ** 2)
    for dt in [1e-2, 1e-1, 1.0]:
        y, s = D.diffusion_step(mode[None, :], shape, h, [eps], dt)
        c = D.rkc_coefficients(s)
        Ts = np.zeros(s + 1)
        Ts[s] = 1.0
        P = c["a_s"] + c["b_s"] * C.chebval(c["w0"] + c["w1"] * dt * lam, Ts)
        assert np.allclose(y[0], P * mode, atol=1e-13)
        z = abs(dt * lam)  # second order: the z^3 term of P differs from 1/6 (0 for s = 2)
        assert abs(P - np.exp(dt * lam)) <= 0.2 * z ** 3 + 0.1 * z ** 4 + 1e-15
    rng = np.random.default_rng(2)
    u = rng.uniform(0, 1, (3, 32 * 32))
    y, s = D.diffusion_step(u, shape, h, [2.5e-3, 2.5e-3, 1.5e-3], 1e-2)
    assert s >= 2
    assert np.allclose(y.sum(axis=1), u.sum(axis=1), rtol=1e-13)


def test_strang_second_order_self_convergence(orc):
    """Nagumo (paper §1, model I) on 2D 24^2 with a smooth bump: the Strang
    error halves twice per halving of dt, i.e. drops by ~4."""
    N = 24
    shape, h = (N, N), 1.0 / N
    x = (np.arange(N) + 0.5) / N
    X, Y = np.meshgrid(x, x)
    u0 = (0.9 * np.exp(-((X - 0.4) ** 2 + (Y - 0.5) ** 2) / 0.05)).ravel()[None, :]
    T, k, eps = 0.08, 10.0, 0.1

    def run(nsteps):
        u = u0.copy()
        dt = T / nsteps
        for _ in range(nsteps):
            u, _, rets, _ = D.strang_step(orc, u, shape, h, [eps], dt, 1e-10, 1e-12,
                                          W.KIND_NAGUMO, [k], tol_transform=0)
            assert rets == (0, 0)
        return u

    u1, u2, u3 = run(2), run(4), run(8)
    e1 = np.max(np.abs(u1 - u2))
    e2 = np.max(np.abs(u2 - u3))
    ratio = e1 / e2
    assert 3.0 <= ratio <= 5.0, ratio
