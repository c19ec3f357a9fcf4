"""Host-side pieces of the measurement (CPU, no GPU): the FLOP accounting
behind the roofline fraction, and the bench's per-cell histogram."""
import numpy as np
import pytest

import bench
from paper_1506_04651_amd import roofline as R


class Counter:
    """A number that counts the arithmetic done with it (FMA not used)."""
    ops = 0

    def __init__(self, v):
        self.v = v

    def _op(self, o, f):
        Counter.ops += 1
        return Counter(f(self.v, o.v if isinstance(o, Counter) else o))

    def __add__(self, o): return self._op(o, lambda a, b: a + b)
    def __sub__(self, o): return self._op(o, lambda a, b: a - b)
    def __mul__(self, o): return self._op(o, lambda a, b: a * b)
    def __truediv__(self, o): return self._op(o, lambda a, b: a / b)


def counted_lu_solve(m):
    """Textbook LU without pivoting and one forward/back substitution on
    counted numbers; returns (factor ops, solve ops)."""
    rng = np.random.default_rng(m)
    a = [[Counter(float(x)) for x in row] for row in rng.normal(size=(m, m)) + m * np.eye(m)]
    Counter.ops = 0
    for k in range(m):
        inv = Counter(1.0) / a[k][k]                  # reciprocal of the pivot
        for i in range(k + 1, m):
            lik = a[i][k] * inv
            a[i][k] = lik
            for j in range(k + 1, m):
                a[i][j] = a[i][j] - lik * a[k][j]
        a[k][k] = inv
    fac = Counter.ops
    b = [Counter(1.0) for _ in range(m)]
    Counter.ops = 0
    for i in range(1, m):
        for j in range(i):
            b[i] = b[i] - a[i][j] * b[j]
    for i in range(m - 1, -1, -1):
        s = b[i]
        for j in range(i + 1, m):
            s = s - a[i][j] * b[j]
        b[i] = s * a[i][i]
    return fac, Counter.ops


@pytest.mark.parametrize("m", [1, 2, 3, 4, 7, 16])
def test_real_lu_and_solve_flop_counts(m):
    """The closed forms of the roofline's real LU and solve counts equal the
    operations of a counted textbook LU (multiply-subtract = 2 FLOPs, the
    reciprocal of each pivot = 1)."""
    fac, sol = counted_lu_solve(m)
    assert R._lu_real(m) == fac
    assert R._solve_real(m) == sol


def cmul(a, b):
    """(a0 + i a1)(b0 + i b1) on counted parts: 4 multiplies, 2 adds."""
    return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])


def csub(a, b):
    return (a[0] - b[0], a[1] - b[1])


def counted_complex_lu_solve(m):
    """Complex LU with the pivot magnitudes |z|^2 of the candidates of each
    column (as partial pivoting computes them) and the pivot's reciprocal
    1/(p_r + i p_i) = (p_r - i p_i)/(p_r^2 + p_i^2); then one solve with the
    stored reciprocals.  Returns (factor ops, solve ops)."""
    rng = np.random.default_rng(100 + m)
    re = rng.normal(size=(m, m)) + m * np.eye(m)
    im = rng.normal(size=(m, m))
    a = [[(Counter(float(re[i, j])), Counter(float(im[i, j]))) for j in range(m)] for i in range(m)]
    Counter.ops = 0
    for k in range(m):
        for i in range(k, m):                       # pivot magnitudes of the candidates
            _ = a[i][k][0] * a[i][k][0] + a[i][k][1] * a[i][k][1]
        pr, pi = a[k][k]
        rn = Counter(1.0) / (pr * pr + pi * pi)
        ii = pi * rn
        inv = (pr * rn, Counter(-ii.v))             # a sign flip, not an operation
        for i in range(k + 1, m):
            lik = cmul(a[i][k], inv)
            a[i][k] = lik
            for j in range(k + 1, m):
                a[i][j] = csub(a[i][j], cmul(lik, a[k][j]))
        a[k][k] = inv
    fac = Counter.ops
    b = [(Counter(1.0), Counter(0.5)) for _ in range(m)]
    Counter.ops = 0
    for i in range(1, m):
        for j in range(i):
            b[i] = csub(b[i], cmul(a[i][j], b[j]))
    for i in range(m - 1, -1, -1):
        s = b[i]
        for j in range(i + 1, m):
            s = csub(s, cmul(a[i][j], b[j]))
        b[i] = cmul(s, a[i][i])
    return fac, Counter.ops


@pytest.mark.parametrize("m", [1, 2, 3, 4, 7, 16])
def test_complex_lu_and_solve_flop_counts(m):
    """The roofline's complex LU and solve counts equal the operations of a
    counted complex LU (the sign flip of the reciprocal's imaginary part is
    not arithmetic and is not counted)."""
    fac, sol = counted_complex_lu_solve(m)
    assert R._lu_cplx(m) == fac
    assert R._solve_cplx(m) == sol


def test_algorithmic_flops_is_linear_in_the_counters():
    ev = R.event_flops(R.KIND_OREGONATOR, 3)
    st = np.zeros((9, 2), dtype=np.int64)
    st[1:, 0] = [3, 2, 1, 20, 2, 4, 9, 7]
    st[1:, 1] = [6, 4, 2, 40, 4, 8, 18, 14]
    a = R.algorithmic_flops(st[:, :1], R.KIND_OREGONATOR, 3)
    b = R.algorithmic_flops(st, R.KIND_OREGONATOR, 3)
    assert a > 0 and b == pytest.approx(3 * a)
    assert set(ev) and all(v >= 0 for v in ev.values())


def test_step_histogram():
    n = np.array([1, 1, 2, 3, 4, 7, 8, 15, 16, 45, 600])
    h = bench.step_histogram(n)
    assert sum(h["cells"]) == n.size
    assert h["cells"][:4] == [2, 2, 2, 2] and h["max"] == 600
    assert h["p50"] == 7.0


def test_reference_flops_by_hand():
    """The reference per-event counts applied to known counters: one cell
    with nstep 10, nfev 40, njac 3, ndec 6, nnewt 12 gives
    40 f + 3 J + 6 factor + 12 Newton + 10 (estimate + step)."""
    st = np.zeros((9, 1), dtype=np.int64)
    st[1, 0], st[4, 0], st[5, 0], st[6, 0], st[8, 0] = 10, 40, 3, 6, 12
    ref = R.reference_counts(R.KIND_OREGONATOR, 3)
    assert R.reference_flops(st, ref) == 40 * 12 + 3 * 10 + 6 * 100 + 12 * 255 + 10 * (45 + 100)
    # FP32 share of the mixed path: factorizations, the Newton solves, the
    # estimate's solve
    assert R.reference_fp32_flops(st, R.KIND_OREGONATOR, 3) == 6 * 100 + 12 * 90 + 10 * 18


def test_reference_counts_by_nonzeros():
    K = np.zeros((16, 16))
    G = np.zeros((16, 16))
    K[0, 1] = K[1, 0] = K[0, 0] = 1.0      # 3 nonzeros
    G[2, 3] = 1.0                           # 1 nonzero
    ref = R.reference_counts(R.KIND_KINETICS, 16, K, G)
    assert ref["f"] == 2 * 3 + 2 * 1 + 2 * 16
    assert ref["jac"] == 4 * 1 + 256
    dense = R.reference_counts(R.KIND_KINETICS, 16)
    assert dense["f"] == 4 * 256 + 32 and dense["jac"] == 3 * 256
    assert R.reference_counts(R.KIND_NAGUMO, 1) is None


def test_blended_bound_and_mixed_counts():
    # 78.6 TFLOP of FP64 and 157.3 TFLOP of FP32 take one second each
    assert R.blended_bound_s(78.6e12, 157.3e12) == pytest.approx(2.0)
    # the mixed kernels add one refinement per solve: more FLOPs per Newton
    # iteration and estimate, nothing else changes
    a, b = R.event_flops(R.KIND_OREGONATOR, 3), R.event_flops(R.KIND_OREGONATOR, 3, mixed=True)
    assert b["newton"] > a["newton"] and b["estimate"] > a["estimate"]
    assert {k: a[k] for k in ("f", "jac", "factor", "step")} == \
        {k: b[k] for k in ("f", "jac", "factor", "step")}
