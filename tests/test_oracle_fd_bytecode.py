"""Pins of the oracle's finite-difference Jacobian, bytecode model and
per-cell warm-start step (CPU only).

- The forward-difference Jacobian is checked against the analytic Jacobians
  (themselves pinned against central differences in test_oracle_pins), and
  its cost (m more f evaluations per Jacobian) against the counters.
- The register-program interpreter is checked against direct evaluation of
  randomly generated expression graphs, against the built-in models (a program
  written operation for operation like the closed form must give bitwise the
  same f and, inside the integrator, bitwise the same trajectory), and its
  validation against malformed programs.
- The warm-start step is checked for the properties its definition fixes:
  no warm start changes nothing, a warm start equals the same first trial step
  given as h0, fixed-step mode returns dt/N, a single full step returns dt,
  and chained warm-started calls stay on the reference solution.

Finite-difference Jacobians are what the paper's STROKE runs use (paper §4 and
Appendix A); the complexity measure counts f evaluations per node (Appendix A).
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

from paper_1506_04651_amd import workloads as W
from tests.bytecode_models import kinetics_program, sparse_kinetics

BC = W  # opcode names


# ---------------------------------------------------------------------------
# finite-difference Jacobian
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", ["oregonator", "robertson", "nagumo"])
def test_fd_jacobian_matches_analytic(orc, case):
    rng = np.random.default_rng(11)
    if case == "oregonator":
        kind, params, prog, m = orc.OREGONATOR, W.OREG_PARAMS, W.oregonator_program(), 3
        ys = rng.uniform([1e-6, 1e-6, 1e-6], [0.05, 0.9, 0.2], (20, 3))
    elif case == "robertson":
        kind, params, prog, m = orc.ROBERTSON, [0.04, 1e4, 3e7], W.robertson_program(), 3
        ys = rng.uniform([0.5, 1e-6, 1e-3], [1.0, 4e-5, 0.5], (20, 3))
    else:
        kind, params, prog, m = orc.NAGUMO, [3.0], W.nagumo_program(3.0), 1
        ys = rng.uniform(-0.2, 1.2, (20, 1))
    for y in ys:
        f_a, J_a = orc.model_eval(kind, params, y)
        f_b, J_fd = orc.model_eval(orc.BYTECODE, prog, y, m=m)
        assert np.array_equal(f_a, f_b)
        scale = np.abs(J_a).max(axis=1, keepdims=True) + 1e-300
        # forward differences: O(d_j) truncation, relative ~sqrt(u_r / |u_j|)
        # (Robertson's k3 u2^2 column: ~1e-5 at u2 ~ 1e-6; that column is
        # pinned exactly by test_fd_increment)
        tol = 1e-4 if case == "robertson" else 1e-5
        assert np.all(np.abs(J_fd - J_a) <= tol * scale), (case, y)


@pytest.mark.parametrize("u2", [3e-6, 2e-5, 4e-3])
def test_fd_increment(orc, u2):
    """Robertson's f3 = k3 u2^2 is quadratic in u2, so its forward difference
    exceeds the derivative by exactly k3 d_2: the increment d_j =
    sqrt(u_r max(1e-5, |u_j|)) is read back from the Jacobian."""
    k = [0.04, 1e4, 3e7]
    y = np.array([0.9, u2, 0.1])
    _, J_a = orc.model_eval(orc.ROBERTSON, k, y)
    _, J_fd = orc.model_eval(orc.BYTECODE, W.robertson_program(k), y, m=3)
    d_expected = np.sqrt(2.0 ** -52 * max(1e-5, u2))
    d_read = (J_fd[2, 1] - J_a[2, 1]) / k[2]
    # (rounding of the f difference limits the read-back to ~1e-3 at large u2)
    assert abs(d_read - d_expected) <= 1e-2 * d_expected


def test_fd_costs_m_evaluations_per_jacobian(orc):
    w = W.oregonator_1d(n=128)
    _, sa, ra = orc.reaction_step(w.states, w.dt, w.rtol, w.atol, w.kind, w.params)
    _, sf, rf = orc.reaction_step(w.states, w.dt, w.rtol, w.atol, w.kind, w.params, jacobian=1)
    assert ra == rf == 0
    same = np.all(sa[[1, 2, 3, 5, 6, 8]] == sf[[1, 2, 3, 5, 6, 8]], axis=0)
    assert same.mean() > 0.9
    # on identical traces nfev grows by exactly m = 3 per Jacobian
    assert np.array_equal(sf[4][same], sa[4][same] + 3 * sa[5][same])


def test_fd_solution_within_tolerance_of_analytic(orc):
    w = W.oregonator_1d(n=256)
    ya, _, _ = orc.reaction_step(w.states, w.dt, w.rtol, w.atol, w.kind, w.params)
    yf, _, _ = orc.reaction_step(w.states, w.dt, w.rtol, w.atol, w.kind, w.params, jacobian=1)
    assert np.max(np.abs(ya - yf) / (w.atol + w.rtol * np.abs(ya))) < 1.0


# ---------------------------------------------------------------------------
# bytecode interpreter
# ---------------------------------------------------------------------------
def random_program(rng, m, n_ops):
    """A random valid program together with the numpy closure computing it
    directly (not by interpreting the program)."""
    consts = list(rng.uniform(0.5, 2.0, 3))
    C = len(consts)
    regs = {}                      # register -> function of y
    for i in range(m):
        regs[i] = (lambda i: lambda y: y[i])(i)
    for c in range(C):
        regs[m + c] = (lambda v: lambda y: v)(consts[c])
    code = []
    nxt = m + C
    for _ in range(n_ops):
        op = int(rng.choice([BC.BC_ADD, BC.BC_SUB, BC.BC_MUL, BC.BC_DIV, BC.BC_NEG,
                             BC.BC_EXP, BC.BC_POW]))
        a, b = (int(v) for v in rng.choice(sorted(regs), 2))
        fa, fb = regs[a], regs[b]
        if op == BC.BC_ADD:
            fn = lambda y, fa=fa, fb=fb: fa(y) + fb(y)
        elif op == BC.BC_SUB:
            fn = lambda y, fa=fa, fb=fb: fa(y) - fb(y)
        elif op == BC.BC_MUL:
            fn = lambda y, fa=fa, fb=fb: fa(y) * fb(y)
        elif op == BC.BC_DIV:
            fn = lambda y, fa=fa, fb=fb: fa(y) / fb(y)
        elif op == BC.BC_NEG:
            fn = lambda y, fa=fa: -fa(y)
        elif op == BC.BC_EXP:
            fn = lambda y, fa=fa: np.exp(fa(y))
        else:
            fn = lambda y, fa=fa, fb=fb: np.power(fa(y), fb(y))
        if nxt >= 64:
            break
        code.append((op, nxt, a, b))
        regs[nxt] = fn
        nxt += 1
    temps = [r for r in regs if r >= m + C] or [0]
    outs = []
    for i in range(m):
        src = int(rng.choice(temps))
        code.append((BC.BC_OUT, i, src, 0))
        outs.append(regs[src])
    prog = [float(len(code)), float(C)] + consts
    for ins in code:
        prog += [float(v) for v in ins]
    return np.array(prog), (lambda y: np.array([g(y) for g in outs]))


@pytest.mark.parametrize("m", [1, 2, 3, 4, 8, 16])
def test_bytecode_random_programs(orc, m):
    rng = np.random.default_rng(100 + m)
    checked = 0
    for _ in range(40):
        prog, ref = random_program(rng, m, int(rng.integers(1, 20)))
        y = rng.uniform(0.2, 1.5, m)
        with np.errstate(all="ignore"):
            want = ref(y)
        f, _ = orc.model_eval(orc.BYTECODE, prog, y, m=m)
        ok = np.isfinite(want)
        assert np.array_equal(np.isfinite(f), ok)
        assert np.allclose(f[ok], want[ok], rtol=1e-14, atol=0.0)
        checked += int(ok.sum())
    assert checked >= 20 * m


@pytest.mark.parametrize("prog_fn,kind,params,m", [
    (lambda: W.oregonator_program(W.OREG_PARAMS), 1, W.OREG_PARAMS, 3),
    (lambda: W.robertson_program(), 5, [0.04, 1e4, 3e7], 3),
])
def test_bytecode_integrates_like_builtin(orc, prog_fn, kind, params, m):
    if kind == 1:
        w = W.oregonator_1d(n=256)
        states, dt, rtol, atol = w.states, w.dt, w.rtol, w.atol
    else:
        rng = np.random.default_rng(3)
        states = np.vstack([1 - rng.uniform(0, 0.1, 64), np.zeros(64), rng.uniform(0, 0.1, 64)])
        dt, rtol, atol = 1.0, 1e-6, 1e-10
    yb, sb, rb = orc.reaction_step(states, dt, rtol, atol, orc.BYTECODE, prog_fn())
    ya, sa, ra = orc.reaction_step(states, dt, rtol, atol, kind, params, jacobian=1)
    assert rb == ra == 0
    assert np.array_equal(yb, ya) and np.array_equal(sb, sa)


@pytest.mark.parametrize("m", [8, 16])
def test_bytecode_kinetics_integrates_like_builtin(orc, m):
    """A kinetics model with 8 and 16 species written as a register program
    gives bitwise the f of the built-in kinetics model and, inside the
    integrator, bitwise its trajectory and counters with the forward-difference
    Jacobian."""
    K, G = sparse_kinetics(m, 50 + m)
    prog = kinetics_program(K, G)
    params = np.concatenate([K.ravel(), G.ravel()])
    rng = np.random.default_rng(60 + m)
    states = 10.0 ** rng.uniform(-3, 0, (m, 96))
    for y in states.T[:20]:
        fb, _ = orc.model_eval(orc.BYTECODE, prog, y, m=m)
        fk, _ = orc.model_eval(orc.KINETICS, params, y, m=m)
        assert np.array_equal(fb, fk)
    yb, sb, rb = orc.reaction_step(states, 0.05, 1e-6, 1e-10, orc.BYTECODE, prog)
    yk, sk, rk = orc.reaction_step(states, 0.05, 1e-6, 1e-10, orc.KINETICS, params, jacobian=1)
    assert rb == rk == 0
    assert np.array_equal(yb, yk) and np.array_equal(sb, sk)


@pytest.mark.parametrize("m", [8, 16])
def test_fd_jacobian_kinetics_many_species(orc, m):
    """The forward-difference Jacobian with 8 and 16 species (through the
    register program of a kinetics model) against the analytic kinetics
    Jacobian, and its cost: on identical traces nfev grows by exactly m per
    Jacobian."""
    K, G = sparse_kinetics(m, 80 + m)
    prog = kinetics_program(K, G)
    params = np.concatenate([K.ravel(), G.ravel()])
    rng = np.random.default_rng(90 + m)
    states = 10.0 ** rng.uniform(-3, 0, (m, 128))
    for y in states.T[:10]:
        _, Ja = orc.model_eval(orc.KINETICS, params, y, m=m)
        _, Jf = orc.model_eval(orc.BYTECODE, prog, y, m=m)
        scale = np.abs(Ja).max(axis=1, keepdims=True) + 1e-300
        assert np.all(np.abs(Jf - Ja) <= 1e-5 * scale)
    _, sa, ra = orc.reaction_step(states, 0.05, 1e-6, 1e-10, orc.KINETICS, params)
    _, sf, rf = orc.reaction_step(states, 0.05, 1e-6, 1e-10, orc.KINETICS, params, jacobian=1)
    assert ra == rf == 0
    same = np.all(sa[[1, 2, 3, 5, 6, 8]] == sf[[1, 2, 3, 5, 6, 8]], axis=0)
    assert same.mean() > 0.5
    assert np.array_equal(sf[4][same], sa[4][same] + m * sa[5][same])


def _bad(prog):
    return np.array(prog, dtype=float)


@pytest.mark.parametrize("prog,m", [
    (_bad([1, 0, 10, 0, 0, 0]), 1),                        # unknown op
    (_bad([1, 0, 0, 0, 0, 0]), 1),                         # unknown op
    (_bad([1, 0, W.BC_OUT, 1, 0, 0]), 1),                  # output index >= m
    (_bad([2, 0, W.BC_OUT, 0, 0, 0, W.BC_OUT, 0, 0, 0]), 1),  # output written twice
    (_bad([1, 0, W.BC_ADD, 5, 0, 0]), 1),                  # no output at all
    (_bad([2, 0, W.BC_ADD, 1, 2, 0, W.BC_OUT, 0, 1, 0]), 1),  # reads r2 before it is written
    (_bad([2, 1, 2.0, W.BC_ADD, 1, 0, 0, W.BC_OUT, 0, 1, 0]), 1),  # writes a constant register
    (_bad([1, 0, W.BC_OUT, 0, 70, 0]), 1),                 # register out of range
    (_bad([1, 0, W.BC_OUT, 0, 0.5, 0]), 1),                # non-integer field
    (_bad([1, 0, W.BC_OUT, 0, 0]), 1),                     # truncated
    (_bad([1, 0, W.BC_OUT, 0, 0, 0]), 17),                 # m > 16
])
def test_bytecode_invalid_programs_rejected(orc, prog, m):
    y, st, ret = orc.reaction_step(np.ones((m, 3)), 0.1, 1e-5, 1e-8, orc.BYTECODE, prog)
    assert ret == -1


# ---------------------------------------------------------------------------
# warm-start step
# ---------------------------------------------------------------------------
def test_warm_start_absent_changes_nothing(orc):
    w = W.oregonator_1d(n=200)
    y0, s0, _ = orc.reaction_step(w.states, w.dt, w.rtol, w.atol, w.kind, w.params)
    h = np.zeros(w.n)
    y1, s1, _ = orc.reaction_step(w.states, w.dt, w.rtol, w.atol, w.kind, w.params, h_cells=h)
    assert np.array_equal(y0, y1) and np.array_equal(s0, s1)
    assert np.all(np.isfinite(h)) and np.all(h > 0) and np.all(h <= 8 * w.dt)


def test_warm_start_equals_h0(orc):
    w = W.oregonator_1d(n=100)
    hin = w.dt / 7
    y0, s0, _ = orc.reaction_step(w.states, w.dt, w.rtol, w.atol, w.kind, w.params, h0=hin)
    h = np.full(w.n, hin)
    y1, s1, _ = orc.reaction_step(w.states, w.dt, w.rtol, w.atol, w.kind, w.params, h_cells=h)
    assert np.array_equal(y0, y1) and np.array_equal(s0, s1)


def test_warm_start_fixed_and_single_step(orc):
    w = W.oregonator_1d(n=50)
    h = np.zeros(w.n)
    orc.reaction_step(w.states, w.dt, w.rtol, w.atol, w.kind, w.params, fixed_steps=4, h_cells=h)
    assert np.all(h == w.dt / 4)
    # y' = -y over a short interval: the first trial step h = dt is accepted
    # and is not shortened, so the held step size is dt itself
    y0 = np.ones((1, 8))
    h = np.zeros(8)
    _, st, ret = orc.reaction_step(y0, 1e-3, 1e-6, 1e-10, orc.LINEAR, [-1.0], h_cells=h)
    assert ret == 0 and np.all(st[1] == 1) and np.all(h == 1e-3)


def test_warm_start_chain_stays_on_reference(orc):
    w = W.oregonator_1d(n=24)
    y = w.states
    h = np.zeros(w.n)
    for _ in range(4):
        y, st, ret = orc.reaction_step(y, w.dt, w.rtol, w.atol, w.kind, w.params, h_cells=h)
        assert ret == 0
    eps, mu, f, q = W.OREG_PARAMS

    def rhs(t, u):
        a, b, c = u
        return [(-q * a - a * b + f * c) / mu, (q * a - a * b + b * (1 - b)) / eps, b - c]

    for c in range(w.n):
        ref = solve_ivp(rhs, (0, 4 * w.dt), w.states[:, c], method="Radau", rtol=1e-11,
                        atol=1e-14).y[:, -1]
        assert np.all(np.abs(y[:, c] - ref) <= 50 * (w.atol + w.rtol * np.abs(ref))), c
