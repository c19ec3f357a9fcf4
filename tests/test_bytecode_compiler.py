"""Expression-to-register-program compiler of the bytecode model (CPU).

Compiled programs are evaluated by the oracle's interpreter and compared with
the expressions evaluated directly by Python in FP64 (same operation order,
so bitwise equal where only + - * / are involved)."""
import numpy as np
import pytest

from paper_1506_04651_amd import bytecode as B
from paper_1506_04651_amd import workloads as W

OREG_EXPRS = ["(-q*a - a*b + f*c)/mu", "(q*a - a*b + b*(1.0 - b))/eps", "b - c"]


def oreg_consts():
    eps, mu, f, q = W.OREG_PARAMS
    return {"q": q, "f": f, "mu": mu, "eps": eps}


def test_oregonator_bitwise_equal_to_closed_form(orc):
    prog = B.compile_model(OREG_EXPRS, ["a", "b", "c"], oreg_consts())
    rng = np.random.default_rng(0)
    for y in rng.uniform(1e-6, 1.0, (50, 3)):
        f_prog, _ = orc.model_eval(orc.BYTECODE, prog, y, m=3)
        f_ref, _ = orc.model_eval(orc.OREGONATOR, W.OREG_PARAMS, y)
        assert np.array_equal(f_prog, f_ref)


def test_transcendentals_and_powers(orc):
    exprs = ["exp(-k*x) * y**2 - log(1 + x)", "x**0.5 + y/(1 + x*x)"]
    prog = B.compile_model(exprs, ["x", "y"], {"k": 1.3})
    rng = np.random.default_rng(1)
    for x, y in rng.uniform(0.1, 3.0, (40, 2)):
        f, _ = orc.model_eval(orc.BYTECODE, prog, np.array([x, y]), m=2)
        k = 1.3
        want = [np.exp(-k * x) * y ** 2 - np.log(1 + x), x ** 0.5 + y / (1 + x * x)]
        assert np.allclose(f, want, rtol=1e-14, atol=0)


def test_long_expression_fits_registers(orc):
    """60 terms, repeated products shared: live ranges fit in the registers."""
    consts = {f"c{i}": 1.0 + i / 8 for i in range(4)}
    terms = [f"c{i % 4}*u{i % 4}*u{(i // 4) % 4}" for i in range(60)]
    prog = B.compile_model([" + ".join(terms), "u0", "u1 - u2", "u3"],
                           ["u0", "u1", "u2", "u3"], consts)
    y = np.array([0.3, 0.7, 1.1, 0.9])
    f, _ = orc.model_eval(orc.BYTECODE, prog, y, m=4)
    want = None
    for i in range(60):
        t = consts[f"c{i % 4}"] * y[i % 4] * y[(i // 4) % 4]
        want = t if want is None else want + t
    assert f[0] == want and f[1] == y[0] and f[2] == y[1] - y[2] and f[3] == y[3]


@pytest.mark.parametrize("exprs,species,consts", [
    (["z"], ["a"], {}),                        # unknown name
    (["a if a else a"], ["a"], {}),            # unsupported syntax
    (["sin(a)"], ["a"], {}),                   # unknown function
    (["a"] * 17, [f"s{i}" for i in range(17)], {}),  # m > 16
    (["a", "b"], ["a"], {}),                   # count mismatch
    (["a"], ["a"], {"a": 1.0}),                # name clash
])
def test_compile_errors(exprs, species, consts):
    with pytest.raises(B.CompileError):
        B.compile_model(exprs, species, consts)
