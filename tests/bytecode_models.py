"""Register programs of kinetics models for the bytecode tests (test
infrastructure: model construction only, no integrator arithmetic)."""
import numpy as np


def sparse_kinetics(m, seed):
    """A sparse kinetics model small enough for the register file: a
    column-conserving chain K (K[i+1, i] = k_i, K[i, i] = -k_i, rates
    10^U(-1, 3)) and a few loss terms G[i, j] = 10^U(-2, 1)."""
    rng = np.random.default_rng(seed)
    K = np.zeros((m, m))
    for i in range(m - 1):
        k = 10.0 ** rng.uniform(-1, 3)
        K[i + 1, i] = k
        K[i, i] = -k
    G = np.zeros((m, m))
    for _ in range(m // 2):
        i, j = (int(v) for v in rng.integers(0, m, 2))
        G[i, j] = 10.0 ** rng.uniform(-2, 1)
    return K, G


def kinetics_program(K, G):
    """The kinetics right-hand side f_i = sum_j K_ij u_j - u_i sum_k G_ik u_k
    as a register program, the nonzero terms summed in index order (the zero
    terms of the dense sums add exact zeros), compiled from expressions.  A
    negative entry -c is written as the subtraction of c u_j, which rounds
    identically and lets the chain's two entries of a rate share a constant."""
    from paper_1506_04651_amd import bytecode as B
    m = K.shape[0]
    names = [f"u{i}" for i in range(m)]
    consts, exprs = {}, []

    def cname(v):
        key = f"c{len(consts)}"
        for k, x in consts.items():
            if x == v:
                return k
        consts[key] = v
        return key

    def total(terms):
        out = ""
        for v, j in terms:
            t = f"{cname(abs(v))}*u{j}"
            out = (t if v > 0 else f"-({t})") if not out else (
                f"{out} + {t}" if v > 0 else f"{out} - {t}")
        return out

    for i in range(m):
        lin = total([(K[i, j], j) for j in range(m) if K[i, j] != 0.0])
        loss = total([(G[i, j], j) for j in range(m) if G[i, j] != 0.0])
        e = f"({lin})" if lin else "0.0"
        if loss:
            e = f"{e} - u{i}*({loss})"
        exprs.append(e)
    return B.compile_model(exprs, names, consts)
