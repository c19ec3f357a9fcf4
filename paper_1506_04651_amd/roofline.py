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


def _refine_real(m, cj_mv):
    """One refinement step of a real solve: residual b - g x + J x (J x costs
    cj_mv), then the correction solve and the update."""
    return cj_mv + 3 * m + _solve_real(m) + m


def _refine_cplx(m, cj_mv):
    """One refinement step of the complex solve: two real J products, the
    residual of both parts (6 FLOPs each), the complex correction solve and
    the update."""
    return 2 * cj_mv + 6 * m + _solve_cplx(m) + 2 * m


def jacobian_product_cost(kind: int, m: int) -> int:
    """FLOPs of one product J x as the kernels form it in the refinement."""
    if kind == KIND_KINETICS:
        return 4 * m * m + 3 * m    # (K x) and (G x), then - uJ (G x) - gJ x
    return 2 * m * m                 # J from the LDS column (or K for linear models)


def event_flops(kind: int, m: int, mixed: bool = False) -> dict:
    """FLOPs per counted event for the kernels as written.  mixed: the
    mixed-precision kernels, which refine every solve once against the FP64
    matrices (the FP32 part is reported separately by event_flops_split)."""
    cf, cj = model_costs(kind, m)
    newton = (3 * m + 4 + 15 * m + 10 * m + _solve_real(m) + _solve_cplx(m) + 3 * m + 11 * m
              + 3 * m + 9 * m + 12)
    estimate = 7 * m + 1 + _solve_real(m) + 3 * m + 2
    if mixed:
        jm = jacobian_product_cost(kind, m)
        newton += _refine_real(m, jm) + _refine_cplx(m, jm)
        estimate += _refine_real(m, jm)
    factor = 7 + 2 * m + _lu_real(m) + _lu_cplx(m)
    step = 3 * m + 2 + (41 + 17 * m) + 15 * m + m + 20
    return {"f": cf, "jac": cj, "factor": factor, "newton": newton,
            "estimate": estimate, "step": step}


def fp32_event_flops(m: int) -> dict:
    """The FP32 share of each counted event in the mixed kernels: the
    factorizations and the triangular solves (two per solve with refinement)."""
    return {"factor": _lu_real(m) + _lu_cplx(m),
            "newton": 2 * (_solve_real(m) + _solve_cplx(m)),
            "estimate": 2 * _solve_real(m)}


def _totals(stats):
    s = np.asarray(stats, dtype=np.int64)
    return {"nstep": int(s[1].sum()), "nfev": int(s[4].sum()), "njac": int(s[5].sum()),
            "ndec": int(s[6].sum()), "nsol": int(s[7].sum()), "nnewt": int(s[8].sum())}


def algorithmic_flops(stats: np.ndarray, kind: int, m: int, mixed: bool = False) -> float:
    """Total FLOPs of a launch from its [9, n] counters, kernels as written."""
    e = event_flops(kind, m, mixed)
    t = _totals(stats)
    return float(t["nfev"] * e["f"] + t["njac"] * e["jac"] + t["ndec"] * e["factor"]
                 + t["nnewt"] * e["newton"] + (t["nsol"] - t["nnewt"]) * e["estimate"]
                 + t["nstep"] * e["step"])


def fp32_flops(stats: np.ndarray, m: int) -> float:
    """FP32 FLOPs of a mixed-precision launch (kernels as written)."""
    e = fp32_event_flops(m)
    t = _totals(stats)
    return float(t["ndec"] * e["factor"] + t["nnewt"] * e["newton"]
                 + (t["nsol"] - t["nnewt"]) * e["estimate"])


# Reference per-event counts of the method, fixed before the kernels were
# written (textbook operation counts of each part of a Radau5 step; FMA = 2):
# f evaluation per nfev, Jacobian per njac, forming E1, E2 and their LU per
# ndec, one Newton iteration without f (T^-1 F, residual, real + complex
# solves 2 m^2 + 8 m^2, T, update, norm) per nnewt, the error estimate and the
# step bookkeeping (controller, start-value extrapolation) per nstep.  For the
# m = 16 kinetics model f and J are given dense and by the nonzeros of K, G.
REFERENCE_COUNTS = {
    (KIND_OREGONATOR, 3): {"f": 12, "jac": 10, "factor": 100, "newton": 255,
                           "estimate": 45, "step": 100},
    (KIND_KINETICS, 16): {"f": 4 * 16 * 16 + 2 * 16, "jac": 3 * 16 * 16, "factor": 13700,
                          "newton": 3450, "estimate": 660, "step": 420},
}
# their FP32 share in the mixed path: the factorizations and the solves
REFERENCE_FP32 = {
    (KIND_OREGONATOR, 3): {"factor": 100, "newton": 2 * 9 + 8 * 9, "estimate": 2 * 9},
    (KIND_KINETICS, 16): {"factor": 13700, "newton": 2 * 256 + 8 * 256, "estimate": 2 * 256},
}


def reference_counts(kind: int, m: int, K=None, G=None) -> dict | None:
    """The reference per-event counts for (kind, m); for kinetics with K, G
    given, f and J counted by nonzeros (f: 2 nnz(K) + 2 nnz(G) + 2 m,
    J: 4 nnz(G) + m^2) instead of dense."""
    ref = REFERENCE_COUNTS.get((kind, m))
    if ref is None:
        return None
    ref = dict(ref)
    if kind == KIND_KINETICS and K is not None and G is not None:
        nk, ng = int(np.count_nonzero(K)), int(np.count_nonzero(G))
        ref["f"] = 2 * nk + 2 * ng + 2 * m
        ref["jac"] = 4 * ng + m * m
    return ref


def reference_flops(stats: np.ndarray, ref: dict) -> float:
    """Total FLOPs of a launch from its counters and reference per-event
    counts (error estimate and bookkeeping per step attempt)."""
    t = _totals(stats)
    return float(t["nfev"] * ref["f"] + t["njac"] * ref["jac"] + t["ndec"] * ref["factor"]
                 + t["nnewt"] * ref["newton"] + t["nstep"] * (ref["estimate"] + ref["step"]))


def reference_fp32_flops(stats: np.ndarray, kind: int, m: int) -> float:
    """FP32 part of reference_flops for the mixed path."""
    r = REFERENCE_FP32[(kind, m)]
    t = _totals(stats)
    return float(t["ndec"] * r["factor"] + t["nnewt"] * r["newton"] + t["nstep"] * r["estimate"])


def blended_bound_s(f64: float, f32: float) -> float:
    """Shortest time the vector ALUs need for f64 FP64 and f32 FP32 FLOPs at
    the published peaks (FP32 at the packed-FMA rate)."""
    return f64 / (PEAK_FP64_VECTOR_TFLOPS * 1e12) + f32 / (PEAK_FP32_VECTOR_TFLOPS * 1e12)


def bytes_per_cell(m: int, with_stats: bool = False) -> int:
    """Algorithmic HBM bytes of one cell-integration: the state read and
    written once (plus the counters if requested)."""
    return 2 * 8 * m + (9 * 4 if with_stats else 0)
