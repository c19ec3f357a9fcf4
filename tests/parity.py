"""Shared helpers for the GPU parity tests (test code, no method arithmetic)."""
import sys

import numpy as np

# counters compared for trace identity (status excluded: compared separately)
TRACE_ROWS = slice(1, 9)


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def cell_rel_err(y, ref, atol):
    """Per cell: max_i |y_i - ref_i| / max(|ref_i|, atol)."""
    return np.max(np.abs(y - ref) / np.maximum(np.abs(ref), atol), axis=0)


def compare(y_gpu, st_gpu, y_ora, st_ora, atol, tol=1e-8, label=""):
    """Parity report: per-cell relative error, trace identity of the counters.
    Returns a dict of statistics."""
    err = cell_rel_err(y_gpu, y_ora, atol)
    same = np.all(st_gpu[TRACE_ROWS] == st_ora[TRACE_ROWS], axis=0) & (st_gpu[0] == st_ora[0])
    rep = {
        "label": label, "n": int(err.size),
        "max_err": float(err.max()) if err.size else 0.0,
        "p99_err": float(np.percentile(err, 99)) if err.size else 0.0,
        "p50_err": float(np.median(err)) if err.size else 0.0,
        "frac_within_tol": float(np.mean(err <= tol)) if err.size else 1.0,
        "trace_divergent": int((~same).sum()),
        "max_err_same_trace": float(err[same].max()) if same.any() else 0.0,
        "max_err_divergent": float(err[~same].max()) if (~same).any() else 0.0,
    }
    print("[parity]", rep, file=sys.stderr, flush=True)
    return rep
