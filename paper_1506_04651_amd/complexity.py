"""Per-node computational complexity of a reaction step (paper Appendix A).

The paper measures the work of the reaction step on a grid node as the number
of right-hand-side evaluations Radau5 performs there during one R_{dt/2}
step, counting an analytic Jacobian as the f evaluations it costs (three for
BZ), and reports which share of the reaction time falls on nodes of low
complexity (for BZ on a 1024^2 grid: 87 % of the time on nodes with
complexity below 17).  Time is taken proportional to complexity.

From the per-cell counters of a reaction step (rows of ``stats``):
``complexity = nfev + jac_evals * njac``, where ``jac_evals`` is the cost of
one analytic Jacobian in f evaluations (0 when the Jacobian was taken by
finite differences: those evaluations are already in nfev).

CLI (runs the GPU reaction step on the paper-constant BZ field):
    python -m paper_1506_04651_amd.complexity --side 1024
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

NFEV, NJAC = 4, 5  # rows of the stats array


def complexity(stats, jac_evals: int = 3) -> np.ndarray:
    """Per-cell complexity from the [9, n] counters."""
    st = np.asarray(stats)
    return st[NFEV].astype(np.int64) + int(jac_evals) * st[NJAC].astype(np.int64)


def time_share_below(cplx, threshold: int) -> float:
    """Share of the total work (sum of complexities) spent on cells whose
    complexity is below ``threshold``."""
    c = np.asarray(cplx, dtype=np.int64)
    tot = c.sum()
    return float(c[c < threshold].sum() / tot) if tot else 0.0


def histogram(cplx, max_bin: int | None = None) -> dict:
    """Cell count per complexity value."""
    c = np.asarray(cplx, dtype=np.int64)
    hi = int(c.max()) if max_bin is None else int(max_bin)
    counts = np.bincount(np.minimum(c, hi), minlength=hi + 1)
    return {int(k): int(v) for k, v in enumerate(counts) if v}


def summary(cplx, thresholds=(17,)) -> dict:
    c = np.asarray(cplx, dtype=np.int64)
    out = {"cells": int(c.size), "min": int(c.min()), "median": float(np.median(c)),
           "mean": float(c.mean()), "max": int(c.max()),
           "cell_share_at_min": float((c == c.min()).mean())}
    for t in thresholds:
        out[f"time_share_below_{t}"] = time_share_below(c, t)
        out[f"cell_share_below_{t}"] = float((c < t).mean())
    return out


def main():
    import torch

    from . import api
    from . import workloads as W
    ap = argparse.ArgumentParser(description="complexity histogram of one reaction step")
    ap.add_argument("--side", type=int, default=1024)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--relax", type=float, default=0.05,
                    help="reaction-only time integrated first, to put the synthetic "
                         "states on the slow manifold (0: none)")
    args = ap.parse_args()
    w = W.oregonator_2d_paper(side=args.side)
    prec = 0 if args.precision == "fp64" else 1
    u = torch.tensor(w.states, dtype=torch.float64, device="cuda")
    if args.relax > 0:
        api.reaction_step(u, args.relax, w.rtol, w.atol, w.kind, w.params, precision=prec)
    st = torch.zeros((9, w.n), dtype=torch.int32, device="cuda")
    nfail = api.reaction_step(u, w.dt, w.rtol, w.atol, w.kind, w.params, stats=st,
                              precision=prec)
    c = complexity(st.cpu().numpy(), jac_evals=3)
    out = {"workload": w.name, "failed": int(nfail), **summary(c), "histogram": histogram(c, 64)}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
