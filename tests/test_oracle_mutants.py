"""Mutation check of the oracle's pins (CPU, no GPU).

The pins in test_oracle_pins.py are meant to catch a dropped term, a wrong
sign or index, or a transposed operand anywhere in the oracle.  This test
plants such mistakes, one at a time, in a copy of the oracle's source,
compiles each copy with the oracle's own build flags, binds it in place of
the oracle, and runs the pins against it: every planted mistake must make at
least one pin fail.  The unmodified source goes through the same pipeline and
must pass every pin, so a failure is the planted mistake's doing.

Not planted: the step-size controller's constants, the Newton stopping
tolerance, the Newton start values and the pivot choice.  They steer which
steps and iterations are taken, not what a step computes, and the paper does
not fix them; the pins see them only through accuracy, which such changes
keep (a planted change of the stopping tolerance passes every pin: parity
unpinned, and the GPU path is compared with the oracle step by step
instead).
"""
import concurrent.futures as cf
import os

import numpy as np
import pytest

import oracle
from oracle.build import SRC, compile_oracle
from tests import test_oracle_pins as P

# (name, text in radau5_oracle.cpp, replacement)
MUTANTS = [
    ("A13 sign", "R.A[0][2] = (double)((-2.0L + 3.0L * r6) / 225.0L);",
     "R.A[0][2] = (double)((2.0L + 3.0L * r6) / 225.0L);"),
    ("A31 term dropped", "R.A[2][0] = (double)((16.0L - r6) / 36.0L);",
     "R.A[2][0] = (double)((16.0L) / 36.0L);"),
    ("node c1 sign", "R.c[0] = (double)((4.0L - r6) / 10.0L);",
     "R.c[0] = (double)((4.0L + r6) / 10.0L);"),
    ("gamma wrong root", "R.gamma_hat = (double)(3.0L + c13 * c13 - c13);",
     "R.gamma_hat = (double)(3.0L - c13 * c13 + c13);"),
    ("d2 sign", "R.d[1] = (double)((-13.0L + 7.0L * r6) / 3.0L);",
     "R.d[1] = (double)((13.0L + 7.0L * r6) / 3.0L);"),
    ("Newton residual drops -Z", "rhs[(size_t)i * m + r] = -Z[(size_t)i * m + r] + h * s;",
     "rhs[(size_t)i * m + r] = h * s;"),
    ("stage sum with A transposed", "s += RK.A[i][j] * F[(size_t)j * m + r];",
     "s += RK.A[j][i] * F[(size_t)j * m + r];"),
    ("Newton matrix with J transposed", "double v = -h * RK.A[i][j] * J[r * m + s];",
     "double v = -h * RK.A[i][j] * J[s * m + r];"),
    ("Newton matrix with A transposed", "double v = -h * RK.A[i][j] * J[r * m + s];",
     "double v = -h * RK.A[j][i] * J[r * m + s];"),
    ("Newton matrix sign", "double v = -h * RK.A[i][j] * J[r * m + s];",
     "double v = h * RK.A[i][j] * J[r * m + s];"),
    ("E1 sign of J", "E1[r * m + s] = (r == s ? RK.gamma_hat / h : 0.0) - J[r * m + s];",
     "E1[r * m + s] = (r == s ? RK.gamma_hat / h : 0.0) + J[r * m + s];"),
    ("estimate drops f", "e[r] = fbase[r] + dz / h;", "e[r] = dz / h;"),
    ("estimate index", "RK.d[1] * Z[m + r]", "RK.d[1] * Z[r]"),
    ("update from stage 2", "y1[r] = y[r] + Z[(size_t)2 * m + r];",
     "y1[r] = y[r] + Z[(size_t)1 * m + r];"),
    ("scale ignores |y|", "sc[r] = T.atol + T.rtol * std::fabs(y0[r]);",
     "sc[r] = T.atol + T.rtol;"),
    ("back substitution multiplies", "b[i] = s / lu[(size_t)i * n + i];",
     "b[i] = s * lu[(size_t)i * n + i];"),
    ("forward substitution index", "for (int j = 0; j < i; ++j) s -= lu[(size_t)i * n + j] * b[j];",
     "for (int j = 0; j < i; ++j) s -= lu[(size_t)j * n + i] * b[j];"),
    ("Oregonator f2 sign", "out[1] = (q * a - a * b + b * (1.0 - b)) / eps;",
     "out[1] = (q * a + a * b + b * (1.0 - b)) / eps;"),
    ("Oregonator J21 sign", "J[3] = (q - b) / eps;", "J[3] = (q + b) / eps;"),
    ("kinetics loss transposed", "loss += G[i * m + j] * y[j];",
     "loss += G[j * m + i] * y[j];"),
    ("Robertson f3 index", "out[2] = k3 * y[1] * y[1];", "out[2] = k3 * y[1] * y[2];"),
]

# the pins, each a call on the bound oracle module
PINS = [
    ("p1 constants", lambda o: P.test_p1_constants_match_collocation_definition(o)),
    ("p2 R(-50)", lambda o: P.test_p2_stability_function_real(o, -50.0)),
    ("p2 R(0.3)", lambda o: P.test_p2_stability_function_real(o, 0.3)),
    ("p2 R(-1+10i)", lambda o: P.test_p2_stability_function_complex(o, -1.0, 10.0)),
    ("p3 order", lambda o: P.test_p3_order_five(o, complex(-1, 0), [2, 4, 8, 16])),
    ("p4 degree 5", lambda o: P.test_p4_degree5_solution_exact(o, 0)),
    ("p4 estimate", lambda o: P.test_p4_error_estimate_matches_definition(o)),
    ("p5 Robertson", lambda o: P.test_p5_robertson_invariant(o, 40.0)),
    ("p6 expm", lambda o: P.test_p6_linear_kinetics_expm(o)),
    ("p7 rest state", lambda o: P.test_p7_oregonator_steady_state(o, 2e-3, (1.29574132, 0.00851737))),
    ("p9 models", lambda o: P.test_p9_models_against_finite_differences(o)),
    ("p10 Newton", lambda o: P.test_p10_linear_newton_exact_in_one_iteration(o)),
    ("p8 brute force", lambda o: P.test_p8_brute_force_oregonator(o, "2d", 6)),
]


def _apply(src, old, new):
    assert src.count(old) == 1, f"mutation site not unique: {old!r}"
    return src.replace(old, new)


@pytest.fixture(scope="module")
def builds(tmp_path_factory):
    d = tmp_path_factory.mktemp("oracle_mutants")
    with open(SRC) as fh:
        base = fh.read()
    jobs = [("unmodified", base)] + [(name, _apply(base, old, new)) for name, old, new in MUTANTS]

    def build(item):
        k, (name, text) = item
        src = os.path.join(d, f"m{k}.cpp")
        with open(src, "w") as fh:
            fh.write(text)
        return name, compile_oracle(src, os.path.join(d, f"libm{k}.so"))

    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        return dict(ex.map(build, enumerate(jobs)))


def _run_pins(libpath, stop_at_first=True):
    """Names of the pins that fail with the oracle at libpath bound in (the
    first one only, unless stop_at_first is false)."""
    import ctypes
    saved = oracle._lib
    oracle._lib = oracle.bind(ctypes.CDLL(libpath))
    failed = []
    try:
        with np.errstate(all="ignore"):
            for name, pin in PINS:
                try:
                    pin(oracle)
                except Exception:  # an assertion, or the oracle refusing the call
                    failed.append(name)
                    if stop_at_first:
                        break
    finally:
        oracle._lib = saved
    return failed


def test_unmodified_source_passes_every_pin(builds):
    assert _run_pins(builds["unmodified"], stop_at_first=False) == []


@pytest.mark.parametrize("name", [m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(builds, name):
    failed = _run_pins(builds[name])
    print(f"{name}: caught by {failed}")
    assert failed, f"no pin catches the planted mistake '{name}'"
