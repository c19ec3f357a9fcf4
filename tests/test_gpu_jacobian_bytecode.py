"""GPU parity of the finite-difference-Jacobian kernels and of the bytecode
model (f given at run time as a register program) against the CPU oracle.

The oracle runs the same program with its own interpreter and the same
forward-difference formula, so per-cell results must meet the FP64 bar
(1e-8, identical counter traces up to rare rounding-flipped decisions)."""
import numpy as np
import pytest

from paper_1506_04651_amd import workloads as W
from tests.parity import compare, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def rd():
    import paper_1506_04651_amd as rd
    rd.load()
    assert torch.cuda.is_available()
    return rd


def run_gpu(rd, w, **opts):
    u = torch.tensor(w.states, dtype=torch.float64, device="cuda")
    st = torch.zeros((9, w.n), dtype=torch.int32, device="cuda")
    ret = rd.reaction_step(u, w.dt, w.rtol, w.atol, w.kind, w.params, stats=st, **opts)
    torch.cuda.synchronize()
    return u.cpu().numpy(), st.cpu().numpy(), ret


def run_oracle(orc, w, **opts):
    return orc.reaction_step(w.states, w.dt, w.rtol, w.atol, w.kind, w.params, **opts)


def check(rep, n, rtol):
    assert rep["max_err_same_trace"] <= 1e-8
    assert rep["trace_divergent"] <= max(2, int(2e-3 * n))
    assert rep["max_err_divergent"] <= 10 * rtol


def program(m, consts, code):
    out = [float(len(code)), float(len(consts))] + [float(c) for c in consts]
    for ins in code:
        out += [float(v) for v in ins]
    return np.array(out)


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("precision", [0, 1])
def test_fd_jacobian_oregonator(rd, orc, schedule, precision):
    w = W.oregonator_1d()
    say("oregonator fd-jacobian schedule", schedule, "precision", precision)
    y, st, ret = run_gpu(rd, w, schedule=schedule, precision=precision, jacobian=1)
    yo, sto, reto = run_oracle(orc, w, jacobian=1)
    assert ret == reto == 0
    rep = compare(y, st, yo, sto, w.atol, label=f"fd s{schedule} p{precision}")
    check(rep, w.n, w.rtol)


def test_bytecode_oregonator_2d(rd, orc):
    w = W.oregonator_2d()
    idx = W.sample_indices(w.n, 16384, 7)
    w = W.Workload("bc_oreg", np.ascontiguousarray(w.states[:, idx]), W.KIND_BYTECODE,
                   W.oregonator_program(w.params), w.dt, w.rtol, w.atol)
    say("bytecode oregonator, n", w.n)
    for schedule in (0, 1):
        y, st, ret = run_gpu(rd, w, schedule=schedule)
        yo, sto, reto = run_oracle(orc, w)
        assert ret == reto == 0
        check(compare(y, st, yo, sto, w.atol, label=f"bc oreg s{schedule}"), w.n, w.rtol)


def test_bytecode_robertson_and_nagumo(rd, orc):
    rng = np.random.default_rng(8)
    y0 = rng.random((3, 512))
    y0 /= y0.sum(axis=0, keepdims=True)
    w = W.Workload("bc_rober", y0, W.KIND_BYTECODE, W.robertson_program(), 40.0, 1e-6, 1e-10)
    say("bytecode robertson")
    y, st, ret = run_gpu(rd, w)
    yo, sto, reto = run_oracle(orc, w)
    assert ret == reto == 0
    check(compare(y, st, yo, sto, w.atol, label="bc rober"), w.n, w.rtol)
    assert np.max(np.abs(y.sum(axis=0) - 1.0)) <= 1e-12
    x = np.linspace(-10, 10, 2048)
    w = W.Workload("bc_nagumo", (0.5 * (1 - np.tanh(x)))[None, :].copy(), W.KIND_BYTECODE,
                   W.nagumo_program(4.0), 0.5, 1e-6, 1e-10)
    say("bytecode nagumo")
    y, st, ret = run_gpu(rd, w)
    yo, sto, reto = run_oracle(orc, w)
    assert ret == reto == 0
    check(compare(y, st, yo, sto, w.atol, label="bc nagumo"), w.n, w.rtol)


def test_bytecode_two_and_four_species(rd, orc):
    # Brusselator: f1 = A - (B + 1) x + x^2 y, f2 = B x - x^2 y
    # registers: 0 x, 1 y, 2 A, 3 B+1, 4 B
    bru = program(2, [1.0, 4.0, 3.0], [
        (3, 5, 0, 0),              # x*x
        (3, 6, 5, 1),              # x^2 y
        (3, 7, 3, 0),              # (B+1) x
        (2, 8, 2, 7), (1, 9, 8, 6), (9, 0, 9, 0),
        (3, 10, 4, 0), (2, 11, 10, 6), (9, 1, 11, 0)])
    rng = np.random.default_rng(9)
    w = W.Workload("bc_bru", rng.uniform(0.5, 3.5, (2, 1024)), W.KIND_BYTECODE, bru, 1.0,
                   1e-6, 1e-9)
    say("bytecode brusselator")
    y, st, ret = run_gpu(rd, w)
    yo, sto, reto = run_oracle(orc, w)
    assert ret == reto == 0
    check(compare(y, st, yo, sto, w.atol, label="bc bru"), w.n, w.rtol)
    # stiff 4-species chain u0 -> u1 -> u2 -> u3 (rates 20, 1e3, 1; the fast
    # middle link makes it stiff, every component stays far above atol), and a
    # quadratic sink on u3: f = (-k0 u0, k0 u0 - k1 u1, k1 u1 - k2 u2, k2 u2 - s u3^2)
    # registers: 0..3 u, 4 k0, 5 k1, 6 k2, 7 s
    chain = program(4, [20.0, 1e3, 1.0, 0.5], [
        (3, 8, 4, 0), (5, 9, 8, 0), (9, 0, 9, 0),
        (3, 10, 5, 1), (2, 11, 8, 10), (9, 1, 11, 0),
        (3, 12, 6, 2), (2, 13, 10, 12), (9, 2, 13, 0),
        (3, 14, 3, 3), (3, 15, 7, 14), (2, 16, 12, 15), (9, 3, 16, 0)])
    w = W.Workload("bc_chain", rng.uniform(0.2, 1.0, (4, 1024)), W.KIND_BYTECODE, chain, 0.5,
                   1e-6, 1e-10)
    say("bytecode 4-species chain")
    y, st, ret = run_gpu(rd, w)
    yo, sto, reto = run_oracle(orc, w)
    assert ret == reto == 0
    check(compare(y, st, yo, sto, w.atol, label="bc chain"), w.n, w.rtol)


def test_bytecode_invalid_program_raises(rd):
    u = torch.ones((1, 16), dtype=torch.float64, device="cuda")
    with pytest.raises(rd.RdError) as ei:
        rd.reaction_step(u, 0.1, 1e-5, 1e-8, rd.BYTECODE, [1, 0, 9, 3, 0, 0])
    assert ei.value.code == -1
    assert torch.all(u == 1.0)


@pytest.mark.parametrize("m", [8, 16])
@pytest.mark.parametrize("precision", [0, 1])
def test_group_engine_bytecode(rd, orc, m, precision):
    """The bytecode model with 8 and 16 species on the 16-lane-group kernels
    (the register program of a sparse kinetics model, Jacobian by forward
    differences), both schedules, against the oracle running the same
    program."""
    from tests.bytecode_models import kinetics_program, sparse_kinetics
    K, G = sparse_kinetics(m, 200 + m)
    prog = kinetics_program(K, G)
    rng = np.random.default_rng(210 + m)
    n = 3000
    w = W.Workload(f"bc_kin{m}", 10.0 ** rng.uniform(-3, 0, (m, n)), W.KIND_BYTECODE, prog,
                   0.05, 1e-6, 1e-10)
    yo, sto, reto = run_oracle(orc, w)
    for schedule in (0, 1):
        say("group bytecode m", m, "precision", precision, "schedule", schedule)
        y, st, ret = run_gpu(rd, w, schedule=schedule, precision=precision)
        assert ret == reto == 0
        check(compare(y, st, yo, sto, w.atol, label=f"bc kin{m} p{precision} s{schedule}"),
              w.n, w.rtol)


@pytest.mark.parametrize("m", [8, 16])
@pytest.mark.parametrize("precision", [0, 1])
def test_group_engine_fd_jacobian(rd, orc, m, precision):
    """The built-in kinetics model with the forward-difference Jacobian on the
    16-lane-group kernels (8 and 16 species), against the oracle with the
    same Jacobian; nfev carries m evaluations per Jacobian."""
    w = W.kinetics16(n=2048, m=m, seed=300 + m)
    yo, sto, reto = run_oracle(orc, w, jacobian=1)
    for schedule in (0, 1):
        say("group fd-jacobian m", m, "precision", precision, "schedule", schedule)
        y, st, ret = run_gpu(rd, w, schedule=schedule, precision=precision, jacobian=1)
        assert ret == reto == 0
        rep = compare(y, st, yo, sto, w.atol, label=f"fd kin{m} p{precision} s{schedule}")
        check(rep, w.n, w.rtol)
        same = np.all(st[1:] == sto[1:], axis=0)
        assert np.array_equal(st[4][same], sto[4][same])
    ya, sa, _ = run_gpu(rd, w, precision=precision)
    same = np.all(sa[[1, 2, 3, 5, 6, 8]] == st[[1, 2, 3, 5, 6, 8]], axis=0)
    assert np.array_equal(st[4][same], sa[4][same] + m * sa[5][same])
