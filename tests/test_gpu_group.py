"""GPU parity of the 16-lane-group kernels (5 <= m <= 16): synthetic stiff
kinetics (the m = 16 workload and other m), linear test models, failure codes,
schedule equivalence and mixed precision, against the CPU FP64 oracle."""
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


def run_gpu(rd, w, stats=True, **opts):
    u = torch.tensor(w.states, dtype=torch.float64, device="cuda")
    st = torch.zeros((9, w.n), dtype=torch.int32, device="cuda") if stats else None
    ret = rd.reaction_step(u, w.dt, w.rtol, w.atol, w.kind, w.params, stats=st, **opts)
    torch.cuda.synchronize()
    return u.cpu().numpy(), (st.cpu().numpy() if stats else None), ret


def run_oracle(orc, w, **opts):
    return orc.reaction_step(w.states, w.dt, w.rtol, w.atol, w.kind, w.params, **opts)


@pytest.mark.parametrize("schedule", [0, 1])
def test_kinetics16_parity(rd, orc, schedule):
    w = W.kinetics16(n=2048)
    say("kinetics16 fp64 schedule", schedule, "n", w.n)
    y, st, ret = run_gpu(rd, w, schedule=schedule)
    yo, sto, reto = run_oracle(orc, w)
    assert ret == reto == 0
    rep = compare(y, st, yo, sto, w.atol, label=f"kin16 sched{schedule}")
    assert rep["max_err"] <= 1e-8
    assert rep["trace_divergent"] == 0


def test_kinetics16_full_batch_sampled(rd, orc):
    """The full 1 048 576-cell batch in the benchmark's launch configuration;
    a seeded sample of cells recomputed by the oracle."""
    w = W.kinetics16()
    say("kinetics16 full batch n", w.n)
    y, st, ret = run_gpu(rd, w)
    assert ret == 0
    idx = W.sample_indices(w.n, 8192, 41)
    s = w.subset(idx)
    yo, sto, reto = run_oracle(orc, s)
    assert reto == 0
    rep = compare(y[:, idx], st[:, idx], yo, sto, w.atol, label="kin16 full sampled")
    assert rep["max_err"] <= 1e-8
    assert rep["trace_divergent"] == 0
    # invariant of every cell at any size: with G >= 0 and 1^T K = 0 the total
    # mass can only decrease, by the quadratic loss term
    s0, s1 = w.states.sum(axis=0), y.sum(axis=0)
    assert np.all(s1 <= s0 * (1 + 10 * w.rtol))


@pytest.mark.parametrize("m", [5, 7, 8, 9, 12, 16])
def test_kinetics_other_m(rd, orc, m):
    w = W.kinetics16(n=384, m=m, seed=100 + m)
    say("kinetics m", m)
    for sched in (0, 1):
        y, st, ret = run_gpu(rd, w, schedule=sched)
        yo, sto, reto = run_oracle(orc, w)
        assert ret == reto
        rep = compare(y, st, yo, sto, w.atol, label=f"kin m{m} sched{sched}")
        assert rep["max_err_same_trace"] <= 1e-8
        assert rep["trace_divergent"] <= 3


def test_linear_chain_exact_fixed_steps(rd, orc):
    """y' = K y with K the 6 x 6 lower shift: solutions of degree 5 are
    integrated exactly by Radau IIA (order 5); fixed steps on the group
    kernel against the closed form and the oracle."""
    m, T = 6, 1.7
    K = np.zeros((m, m))
    for i in range(m - 1):
        K[i + 1, i] = 1.0
    y0 = np.zeros((m, 8))
    y0[0] = np.arange(1, 9)
    w = W.Workload("chain", y0, W.KIND_LINEAR, K.ravel(), T, 1e-8, 1e-8)
    exact = np.array([T ** k / np.prod(np.arange(1, k + 1)) for k in range(m)])[:, None] * y0[0]
    for fixed in (1, 3):
        say("linear chain fixed", fixed)
        y, st, ret = run_gpu(rd, w, fixed_steps=fixed)
        assert ret == 0
        assert np.max(np.abs(y - exact)) <= 1e-13 * np.max(np.abs(exact))
        yo, sto, _ = run_oracle(orc, w, fixed_steps=fixed)
        assert np.array_equal(st[1:], sto[1:])


def test_singular_five_in_a_row(rd, orc):
    g = orc.constants()["gamma_hat"]
    dt = 0.5
    K = np.diag([g / (dt * 0.5 ** i) for i in range(5)])
    w = W.Workload("sing5", np.ones((5, 7)), W.KIND_LINEAR, K.ravel(), dt, 1e-5, 1e-5)
    say("singular m=5")
    y, st, ret = run_gpu(rd, w)
    yo, sto, reto = run_oracle(orc, w)
    assert ret == reto == 7
    assert np.all(st[0] == 3) and np.array_equal(st[6], sto[6])
    assert np.array_equal(y, w.states)


def test_group_nonfinite_and_maxsteps(rd, orc):
    w = W.kinetics16(n=64, seed=9)
    s = w.states.copy()
    s[3, 10] = np.nan
    bad = W.Workload("bad16", s, w.kind, w.params, w.dt, w.rtol, w.atol)
    say("kinetics16 nonfinite")
    y, st, ret = run_gpu(rd, bad)
    yo, sto, reto = run_oracle(orc, bad)
    assert ret == reto == 1 and np.array_equal(st[0], sto[0])
    say("kinetics16 max_steps=5")
    y, st, ret = run_gpu(rd, w, max_steps=5)
    yo, sto, reto = run_oracle(orc, w, max_steps=5)
    assert ret == reto and np.array_equal(st[0], sto[0])


def test_group_schedules_and_order_bitwise(rd):
    w = W.kinetics16(n=20000, seed=12)
    say("kinetics16 schedule/order equivalence")
    a, sa, _ = run_gpu(rd, w, schedule=0, order=1)
    b, sb, _ = run_gpu(rd, w, schedule=0, order=0)
    c, sc, _ = run_gpu(rd, w, schedule=1)
    assert np.array_equal(a, b) and np.array_equal(a, c)
    assert np.array_equal(sa, sb) and np.array_equal(sa, sc)
    for v in range(1, rd.variant_count(rd.KINETICS, 16, 0, 0) + 1):
        d, sd, _ = run_gpu(rd, w, variant=v)
        assert np.array_equal(a, d), v


@pytest.mark.parametrize("m", [7, 12])
def test_group_claim_order_other_m(rd, orc, m):
    """Batches large enough for the longest-first claim order (>= 8192 cells)
    with fewer than 16 species: the cost keys read the request's m state rows
    and m x m parameter blocks.  Same states and counters as the natural
    claim order, and the oracle's on a sample."""
    w = W.kinetics16(n=12000, m=m, seed=40 + m)
    say("kinetics m", m, "n", w.n, "claim order on/off")
    a, sa, ra = run_gpu(rd, w, order=1)
    b, sb, rb = run_gpu(rd, w, order=0)
    assert ra == rb == 0
    assert np.array_equal(a, b) and np.array_equal(sa, sb)
    idx = W.sample_indices(w.n, 192, 5)
    yo, sto, reto = run_oracle(orc, w.subset(idx))
    rep = compare(a[:, idx], sa[:, idx], yo, sto, w.atol, label=f"kin m{m} ordered sample")
    # In the m = 7 batch one species decays to ~1e-13, a thousand times below
    # atol, inside cells whose other species are up to 0.1: rounding of the
    # large species (~1e-16 absolute) is then 1e-6 relative to the atol floor
    # of the per-component measure.  The error is taken per cell, against the
    # cell's largest species (floored at atol), for this batch.
    y, same = a[:, idx], np.all(sa[:, idx] == sto, axis=0)
    cell = np.abs(y - yo).max(axis=0) / np.maximum(np.abs(yo).max(axis=0), w.atol)
    say("per-cell error: same trace", cell[same].max(), "divergent", cell[~same].max(initial=0.0))
    assert cell[same].max() <= 1e-8
    assert (~same).sum() <= int(0.05 * idx.size)
    assert cell.max() <= 10 * w.rtol


@pytest.mark.parametrize("m", [16, 8, 7])
@pytest.mark.parametrize("precision", [0, 1])
def test_group_variants_fused_and_unfused_identical(rd, m, precision):
    """Every persistent variant of the 16-lane engine, including the ones
    whose row broadcasts are separate DPP moves instead of fused DPP
    multiply-adds, gives the same states and counters (m = 16: 16-column
    kernels with the fused matrix-vector solves; m = 7: 8-column kernels,
    solves as loops)."""
    w = W.kinetics16(n=6000, m=m, seed=21 + m)
    a, sa, _ = run_gpu(rd, w, precision=precision)
    names = []
    for v in range(1, rd.variant_count(rd.KINETICS, m, precision, 0) + 1):
        names.append(rd.variant_name(rd.KINETICS, m, precision, 0, v))
        d, sd, _ = run_gpu(rd, w, precision=precision, variant=v)
        assert np.array_equal(a, d) and np.array_equal(sa, sd), names[-1]
    assert any(n.endswith(".unfused") for n in names)


def test_kinetics16_mixed_precision_error_report(rd, orc):
    """FP32 inverses inside the FP64 Newton iteration, every solve refined once
    against the FP64 matrices: within 1e-8 of the FP64 oracle per cell, with
    the oracle's control decisions, on 2048 cells and on a sample of the full
    1 048 576-cell batch."""
    w = W.kinetics16(n=2048)
    say("kinetics16 mixed")
    y, st, ret = run_gpu(rd, w, precision=1)
    yo, sto, reto = run_oracle(orc, w)
    assert ret == 0
    rep = compare(y, st, yo, sto, w.atol, label="kin16 mixed")
    assert rep["max_err"] <= 1e-8
    assert rep["trace_divergent"] == 0
    w = W.kinetics16()
    say("kinetics16 mixed full batch n", w.n)
    y, st, ret = run_gpu(rd, w, precision=1)
    assert ret == 0
    idx = W.sample_indices(w.n, 4096, 42)
    yo, sto, reto = run_oracle(orc, w.subset(idx))
    rep = compare(y[:, idx], st[:, idx], yo, sto, w.atol, label="kin16 mixed full sampled")
    assert rep["max_err"] <= 1e-8
    assert rep["trace_divergent"] == 0


def _extreme_linear(m, n=256, seed=11):
    """du/dt = A u with one eigenvalue -1e300 beside modest coupled ones: the
    iteration matrices get pivots near 1e300, outside the range of the
    engines' fast reciprocals, and |p|^2 of the complex pivot overflows (the
    scaled complex reciprocal and, on the 16-lane engine, the safe re-inversion
    run).  The oracle solves the untransformed real system.  The stiff
    component ends at e^(-1e299) u0, i.e. zero up to the rounding of
    y0 + z3 ~ 1e-16 |u0|, so atol (the error floor) is 1e-6 here."""
    rng = np.random.default_rng(seed)
    A = -np.diag(np.concatenate([[1e300], np.arange(1.0, m)]))
    for i in range(1, m):
        A[i, 1 + (i % (m - 1))] += 0.3
    u = rng.uniform(0.1, 1.0, (m, n))
    return W.Workload(f"linear{m}_extreme", np.ascontiguousarray(u), W.KIND_LINEAR,
                      np.ascontiguousarray(A.ravel()), 0.1, 1e-6, 1e-6, {})


@pytest.mark.parametrize("m", [3, 5, 16])
def test_pivots_outside_the_fast_reciprocal_range(rd, orc, m):
    w = _extreme_linear(m)
    say("extreme linear m", m, "n", w.n)
    y, st, ret = run_gpu(rd, w)
    yo, sto, reto = run_oracle(orc, w)
    assert ret == reto == 0
    assert (sto[0] == 0).all() and (st[0] == 0).all()
    rep = compare(y, st, yo, sto, w.atol, label=f"extreme linear m{m}")
    assert rep["max_err"] <= 1e-8
    assert rep["trace_divergent"] == 0
