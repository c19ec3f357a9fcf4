"""Mutation check of the oracle's pins (CPU, no GPU).

The pins (test_oracle_pins.py, test_oracle_mra.py, test_oracle_diffusion.py)
are meant to catch a dropped term, a wrong sign or index, or a transposed
operand anywhere in the oracle.  This test plants such mistakes, one at a
time, in a copy of an oracle source: the C++ Radau5 oracle (compiled with the
oracle's own build flags and bound in place of the oracle), the
multiresolution and the diffusion oracles (imported under another name and
put in place of the module the pins call).  Every planted mistake must make
at least one pin fail.  The unmodified sources go through the same pipelines
and must pass every pin, so a failure is the planted mistake's doing.

Not planted: the step-size controller's constants, the Newton stopping
tolerance and the pivot choice.  They steer which
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
from paper_1506_04651_amd import workloads as W
from tests import test_oracle_fd_bytecode as PF
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
    # the extensions: forward-difference Jacobian, bytecode model, warm start
    ("FD increment without sqrt",
     "const double dj = std::sqrt(2.220446049250313e-16 * std::max(1e-5, std::fabs(y[j])));",
     "const double dj = 2.220446049250313e-16 * std::max(1e-5, std::fabs(y[j]));"),
    ("FD column transposed", "J[i * m + j] = (fp[i] - fy[i]) / dj;",
     "J[j * m + i] = (fp[i] - fy[i]) / dj;"),
    ("bytecode SUB operands", "case RDO_BC_SUB: r[d] = r[a] - r[b]; break;",
     "case RDO_BC_SUB: r[d] = r[b] - r[a]; break;"),
    ("bytecode POW operands", "case RDO_BC_POW: r[d] = std::pow(r[a], r[b]); break;",
     "case RDO_BC_POW: r[d] = std::pow(r[b], r[a]); break;"),
    ("bytecode writes constants", "            if (d < m + C) return false;\n            written[d] = true;",
     "            written[d] = true;"),
    # Newton start values: the collocation cubic of the last accepted step
    ("start values node", "const double sn[4] = {-1.0, RK.c[0] - 1.0, RK.c[1] - 1.0, 0.0};",
     "const double sn[4] = {-1.0, RK.c[0], RK.c[1] - 1.0, 0.0};"),
    ("start values v1 sign", "const double v1 = zold[0 * m + r] - z3;",
     "const double v1 = zold[0 * m + r] + z3;"),
    ("start values step ratio", "const double s = RK.c[i] * h / h_old;",
     "const double s = RK.c[i] * h_old / h;"),
    ("warm start ignored", "integrate_(y, dt, st, h_pre, h_io && *h_io > 0.0 ? *h_io : 0.0);",
     "integrate_(y, dt, st, h_pre, 0.0);"),
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
    ("FD vs analytic", lambda o: PF.test_fd_jacobian_matches_analytic(o, "oregonator")),
    ("FD increment", lambda o: PF.test_fd_increment(o, 2e-5)),
    ("bytecode random programs", lambda o: PF.test_bytecode_random_programs(o, 3)),
    ("bytecode like built-in", lambda o: PF.test_bytecode_integrates_like_builtin(
        o, lambda: W.robertson_program(), 5, [0.04, 1e4, 3e7], 3)),
    ("bytecode rejects", lambda o: PF.test_bytecode_invalid_programs_rejected(
        o, np.array([2, 1, 2.0, W.BC_ADD, 1, 0, 0, W.BC_OUT, 0, 1, 0], dtype=float), 1)),
    ("warm start equals h0", lambda o: PF.test_warm_start_equals_h0(o)),
    ("p11 start values", lambda o: P.test_p11_start_values_reproduce_a_cubic(o, 2.5)),
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


# ---------------------------------------------------------------------------
# The Python oracles: multiresolution (oracle/mra.py) and diffusion
# (oracle/diffusion.py).  A mutated copy is imported under another name and
# put in place of the module the pins call.
# ---------------------------------------------------------------------------
PY_MUTANTS = {
    "mra": [
        ("projection weight", "levels[j - 1] = s * (1.0 / nc)", "levels[j - 1] = s * (1.0 / (nc - 1))"),
        ("prediction sign", "sgn = [np.where(s == 0, 0.125, -0.125) for s in sub]",
         "sgn = [np.where(s == 0, -0.125, 0.125) for s in sub]"),
        ("prediction y difference", "        return rows[0] + sgn[1] * (rows[-1] - rows[1])",
         "        return rows[0] + sgn[1] * (rows[1] - rows[-1])"),
        ("prediction 3D z weight", "    return planes[0] + sgn[2] * (planes[-1] - planes[1])",
         "    return planes[0] + sgn[1] * (planes[-1] - planes[1])"),
        ("edge reflection", "c = np.where(c < 0, 0, np.where(c >= N, N - 1, c))",
         "c = np.where(c < 0, 1, np.where(c >= N, N - 1, c))"),
        ("detail sign", "out[j] = levels[j] - predict(levels[j - 1], d, j - 1, k)",
         "out[j] = levels[j] + predict(levels[j - 1], d, j - 1, k)"),
        ("detail norm mean", "return acc * (1.0 / m)", "return acc"),
        ("threshold exponent", "eps_j2 = (eps * eps) * np.ldexp(1.0, d * (j - J))",
         "eps_j2 = (eps * eps) * np.ldexp(1.0, (j - J))"),
        ("children test any", "R[j - 1] |= sig.reshape(-1, nc).any(axis=1)",
         "R[j - 1] |= sig.reshape(-1, nc).all(axis=1)"),
        ("grading neighbourhood", "nb = [coords[a] + off[a] - 1 for a in range(d)]",
         "nb = [coords[a] + off[a] for a in range(d)]"),
        ("Morton bit order", "out |= ((np.asarray(c, dtype=np.int64) >> b) & 1) << (d * b + (d - 1 - a))",
         "out |= ((np.asarray(c, dtype=np.int64) >> b) & 1) << (d * b + a)"),
        ("key level field", "lev = np.uint64(j << KEY_LEVEL_SHIFT)", "lev = np.uint64(j << (KEY_LEVEL_SHIFT + 1))"),
        ("tree parent average", "tree_val[j - 1][:, par] = s * (1.0 / nc)",
         "tree_val[j - 1][:, par] = s * (1.0 / (nc + 1))"),
    ],
    "diffusion": [
        ("Chebyshev second derivative", "d2T[j + 1] = 4 * dT[j] + 2 * x * d2T[j] - d2T[j - 1]",
         "d2T[j + 1] = 2 * dT[j] + 2 * x * d2T[j] - d2T[j - 1]"),
        ("w1 inverted", "w1 = dT[s] / d2T[s]", "w1 = d2T[s] / dT[s]"),
        ("nu sign", "nu[j] = -b[j] / b[j - 2]", "nu[j] = b[j] / b[j - 2]"),
        ("gamma index", "gamt[j] = -a[j - 1] * mut[j]", "gamt[j] = -a[j] * mut[j]"),
        ("Laplacian flux sign", "out[tuple(hi)] -= fwd", "out[tuple(hi)] += fwd"),
        ("Laplacian scale", "return (out / (h * h)).ravel()", "return (out / h).ravel()"),
        ("first stage weight", 'y_prev = y0 + c["mut"][1] * dt * F0', "y_prev = y0 + dt * F0"),
        ("stage uses Y0 twice", 'c["nu"][j] * y_prev2 + c["mut"][j] * dt * Fj',
         'c["nu"][j] * y0 + c["mut"][j] * dt * Fj'),
        ("damping", "w0 = 1.0 + eps / (s * s)", "w0 = 1.0 + eps / s"),
    ],
}


def _py_pins(kind, orc):
    from tests import test_oracle_diffusion as PD
    from tests import test_oracle_mra as PM
    if kind == "mra":
        return PM, "M", [
            ("Morton order", lambda: PM.test_morton_order_and_round_trip(2, 3)),
            ("Morton order 3D", lambda: PM.test_morton_order_and_round_trip(3, 2)),
            ("quadratic prediction 2D", lambda: PM.test_prediction_exact_for_quadratics(2)),
            ("quadratic prediction 3D", lambda: PM.test_prediction_exact_for_quadratics(3)),
            ("projection", lambda: PM.test_projection_is_the_average_of_covered_cells(2, 5)),
            ("leaf set", lambda: PM.test_leaf_set_properties(2, 6, 1e-3)),
            ("leaf set 3D", lambda: PM.test_leaf_set_properties(3, 4, 1e-3)),
            ("reconstruction", lambda: PM.test_reconstruction(2, 6)),
            ("adapt idempotent", lambda: PM.test_adapt_without_refinement_is_idempotent(2, 6, 1e-3)),
            ("1D prediction golden", lambda: PM.test_prediction_matches_the_paper_1d_operator()),
            ("thresholds golden", lambda: PM.test_thresholds_match_the_paper()),
            ("edge prediction golden", lambda: PM.test_prediction_at_the_domain_edges()),
            ("species mean", lambda: PM.test_thresholds_average_over_species()),
            ("grading isolated 2D", lambda: PM.test_grading_around_an_isolated_cell(2, 6)),
            ("grading isolated 3D", lambda: PM.test_grading_around_an_isolated_cell(3, 4)),
        ]
    return PD, "D", [
        ("stability polynomial", lambda: PD.test_rkc_stability_polynomial(5)),
        ("second order", lambda: PD.test_rkc_second_order(4)),
        ("stage rule", lambda: PD.test_rkc_stage_rule_is_stable(400.0)),
        ("Laplacian", lambda: PD.test_laplacian_constants_mass_and_modes((16, 12))),
        ("step on a mode", lambda: PD.test_diffusion_step_on_a_mode_and_mass()),
        ("Strang order", lambda: PD.test_strang_second_order_self_convergence(orc)),
    ]


def _run_py_pins(kind, text, orc, tmp_dir, stop_at_first=True):
    import importlib.util
    path = os.path.join(tmp_dir, f"mut_{kind}_{abs(hash(text))}.py")
    with open(path, "w") as fh:
        fh.write(text)
    spec = importlib.util.spec_from_file_location(f"oracle_mut_{kind}", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    pins_mod, attr, pins = _py_pins(kind, orc)
    saved = getattr(pins_mod, attr)
    setattr(pins_mod, attr, mod)
    failed = []
    try:
        with np.errstate(all="ignore"):
            for name, pin in pins:
                try:
                    pin()
                except Exception:
                    failed.append(name)
                    if stop_at_first:
                        break
    finally:
        setattr(pins_mod, attr, saved)
    return failed


def _py_source(kind):
    with open(os.path.join(os.path.dirname(SRC), f"{kind}.py")) as fh:
        return fh.read()


@pytest.mark.parametrize("kind", ["mra", "diffusion"])
def test_unmodified_python_oracle_passes_every_pin(orc, tmp_path, kind):
    assert _run_py_pins(kind, _py_source(kind), orc, tmp_path, stop_at_first=False) == []


@pytest.mark.parametrize("kind,name", [(k, m[0]) for k in PY_MUTANTS for m in PY_MUTANTS[k]])
def test_planted_mistake_in_python_oracle_fails_a_pin(orc, tmp_path, kind, name):
    old, new = next((o, n) for nm, o, n in PY_MUTANTS[kind] if nm == name)
    failed = _run_py_pins(kind, _apply(_py_source(kind), old, new), orc, tmp_path)
    print(f"{kind} / {name}: caught by {failed}")
    assert failed, f"no pin catches the planted mistake '{name}' in oracle/{kind}.py"
