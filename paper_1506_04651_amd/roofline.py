"""Algorithmic FLOP accounting for the reaction-step kernels.

The work of one cell-integration is data dependent (the number of steps,
Newton iterations, Jacobians and factorizations differs per cell, paper
Appendix A), so FLOPs are counted from the per-cell counters the kernels
return, times the FLOPs each counted event performs in the kernels as
written.  Conventions: add, sub, mul, div and sqrt = 1 FLOP, fused multiply-add
= 2; comparisons, selects and integer work = 0.  Pivot magnitudes |z|^2 of
the complex LU are counted.

Counter rows: 0 status, 1 nstep, 2 naccept, 3 nreject, 4 nfev, 5 njac,
6 ndec, 7 nsol, 8 nnewt.
"""
from __future__ import annotations

import numpy as np

KIND_OREGONATOR, KIND_KINETICS, KIND_NAGUMO, KIND_LINEAR, KIND_ROBERTSON = 1, 2, 3, 4, 5

# MI355X published peaks (vector ALU; packed-FP32 issue is not used by these
# kernels, so FP32 vector work runs at the FP64 vector rate)
PEAK_FP64_VECTOR_TFLOPS = 78.6
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0


def _lu_real(m):
    return sum(1 + (m - k - 1) + 2 * (m - k - 1) ** 2 for k in range(m))


def _lu_cplx(m):
    return sum(3 * (m - k) + 6 + 6 * (m - k - 1) + 8 * (m - k - 1) ** 2 for k in range(m))


def _solve_real(m):
    return 2 * m * m - m


def _solve_cplx(m):
    return 8 * m * m - 2 * m


def model_costs(kind: int, m: int):
    """(C_f, C_J): FLOPs of one right-hand side and one Jacobian evaluation."""
    if kind == KIND_OREGONATOR:
        return 14, 10
    if kind == KIND_ROBERTSON:
        return 11, 8
    if kind == KIND_NAGUMO:
        return 4, 4
    if kind == KIND_LINEAR:
        return 2 * m * m, 0
    if kind == KIND_KINETICS:
        return 4 * m * m + 2 * m, 4 * m * m + m
    raise ValueError(kind)


def event_flops(kind: int, m: int) -> dict:
    """FLOPs per counted event for the kernels as written."""
    cf, cj = model_costs(kind, m)
    newton = (3 * m + 4 + 15 * m + 10 * m + _solve_real(m) + _solve_cplx(m) + 3 * m + 11 * m
              + 3 * m + 9 * m + 12)
    estimate = 7 * m + 1 + _solve_real(m) + 3 * m + 2
    factor = 7 + 2 * m + _lu_real(m) + _lu_cplx(m)
    step = 3 * m + 2 + (41 + 17 * m) + 15 * m + m + 20
    return {"f": cf, "jac": cj, "factor": factor, "newton": newton,
            "estimate": estimate, "step": step}


def algorithmic_flops(stats: np.ndarray, kind: int, m: int) -> float:
    """Total algorithmic FLOPs of a launch from its [9, n] counters."""
    e = event_flops(kind, m)
    s = np.asarray(stats, dtype=np.int64)
    nstep, nfev, njac, ndec, nsol, nnewt = (s[1].sum(), s[4].sum(), s[5].sum(), s[6].sum(),
                                            s[7].sum(), s[8].sum())
    return float(nfev * e["f"] + njac * e["jac"] + ndec * e["factor"] + nnewt * e["newton"]
                 + (nsol - nnewt) * e["estimate"] + nstep * e["step"])


def bytes_per_cell(m: int, with_stats: bool = False) -> int:
    """Algorithmic HBM bytes of one cell-integration: the state read and
    written once (plus the counters if requested)."""
    return 2 * 8 * m + (9 * 4 if with_stats else 0)
