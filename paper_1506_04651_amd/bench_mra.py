"""Measure the multiresolution operations (leaf set of a field, reconstruction,
adaptation of a leaf set) on the paper's BZ setting and on a 3D front.

Each operation is one synchronous call of the C ABI (rd_mra_leaves with the
capacity of the whole fine grid, so the leaves are written in the same pass;
rd_mra_reconstruct; rd_mra_adapt), timed on the host around the call, median
of --reps calls.  Algorithmic HBM bytes of a pass, a lower bound: the input
read once and the output written once -- leaf set: m N 8 read + n_leaves
(8 + 8 m) written; reconstruction: n_leaves (8 + 8 m) read + m N 8 written;
adaptation: n_leaves (8 + 8 m) read + n_out (8 + 8 m) written -- over the
8 TB/s HBM3E peak.  The whole pyramid (4/3 of the finest level) is written
and read again by the per-level kernels, so the fraction understates how
close the kernels run to the bandwidth they actually move.

Fields: the 2D BZ spiral field with the paper's constants (q = 0.02) on a
2^J x 2^J grid, threshold 1e-2 with per-species scales max|u_i| (the
generator's 1e-3 noise sits above smaller thresholds); in 3D a seeded
spherical tanh front (width 0.02) in three species on 2^J cells per side,
threshold 1e-3.  After the leaf set, the adaptation runs on the leaf values
perturbed by a seeded 1 % multiplicative change (a stand-in for a reaction
step).

CLI:  python -m paper_1506_04651_amd.bench_mra [--dim 2] [--levels 10] [--reps 10]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0


def front_3d(J: int, seed: int = 0) -> np.ndarray:
    N = 1 << J
    x = (np.arange(N) + 0.5) / N
    rng = np.random.default_rng(seed)
    c = rng.uniform(0.35, 0.65, 3)
    z, y, xx = np.meshgrid(x, x, x, indexing="ij")  # x fastest
    r = np.sqrt((xx - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    u = np.tanh((r - 0.25) / 0.02)
    return np.vstack([u.ravel(), (0.5 * u * u + 0.1 * xx).ravel(), np.cos(3 * z + 1.0).ravel()])


def main():
    import torch

    from . import _lib, api
    from . import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--dim", type=int, default=2, choices=[2, 3])
    ap.add_argument("--levels", type=int, default=10)
    ap.add_argument("--reps", type=int, default=10)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    d, J = args.dim, args.levels
    if d * J > 30:
        raise SystemExit("dim * levels must be <= 30")
    if d == 2:
        w = W.oregonator_2d_paper(side=1 << J)
        states, eps = w.states, 1e-2
        field = f"bz_q0.02_{1 << J}x{1 << J}"
    else:
        states, eps = front_3d(J), 1e-3
        field = f"front_{1 << J}^3"
    m, N = states.shape
    scale = np.max(np.abs(states), axis=1)
    lib = _lib.load()
    fine = torch.tensor(states, dtype=torch.float64, device="cuda")
    p, keep = api._mra_params(d, J, eps, scale, m, False)
    pr, keep_r = api._mra_params(d, J, eps, scale, m, True)
    sh = api._stream_handle(None)
    keys = torch.empty(N, dtype=torch.int64, device="cuda")
    vals = torch.empty(m * N, dtype=torch.float64, device="cuda")
    okeys = torch.empty(N, dtype=torch.int64, device="cuda")
    ovals = torch.empty(m * N, dtype=torch.float64, device="cuda")
    rec = torch.empty((m, N), dtype=torch.float64, device="cuda")
    counts = (ctypes.c_int64 * (J + 1))()
    ocounts = (ctypes.c_int64 * (J + 1))()
    P = ctypes.c_void_p

    def leaves():
        return api._check(lib.rd_mra_leaves(P(fine.data_ptr()), m, ctypes.byref(p), P(keys.data_ptr()),
                                            P(vals.data_ptr()), N, counts, sh))

    def reconstruct(n):
        return api._check(lib.rd_mra_reconstruct(P(keys.data_ptr()), P(vals.data_ptr()), n, m,
                                                 ctypes.byref(p), P(rec.data_ptr()), sh))

    def adapt(n):
        return api._check(lib.rd_mra_adapt(P(keys.data_ptr()), P(vals.data_ptr()), n, m,
                                           ctypes.byref(pr), P(okeys.data_ptr()), P(ovals.data_ptr()),
                                           N, ocounts, sh))

    def timed(fn, *a):
        fn(*a)  # warm-up: workspace
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.reps):
            t0 = time.perf_counter()
            r = fn(*a)
            ts.append((time.perf_counter() - t0) * 1e3)
        ts.sort()
        return r, ts[len(ts) // 2]

    n, t_leaves = timed(leaves)
    _, t_rec = timed(reconstruct, n)
    # perturb the leaf values (a stand-in for a reaction step), then adapt
    g = torch.Generator(device="cuda").manual_seed(5)
    v = vals[: m * n].view(m, n)
    v.mul_(1.0 + 0.01 * torch.rand((m, n), generator=g, dtype=torch.float64, device="cuda"))
    nout, t_adapt = timed(adapt, n)
    del keep, keep_r
    leaf_b = 8 + 8 * m
    b_leaves = m * N * 8 + n * leaf_b
    b_rec = n * leaf_b + m * N * 8
    b_adapt = n * leaf_b + nout * leaf_b

    def gbs(b, ms):
        return b / (ms * 1e-3) / 1e9

    out = {"workload": field, "dim": d, "levels": J, "m": m, "fine_cells": N, "eps": eps,
           "leaves": n, "compression": 1.0 - n / N, "leaves_per_level": list(counts),
           "adapted_leaves": nout,
           "leaves_ms": t_leaves, "reconstruct_ms": t_rec, "adapt_ms": t_adapt,
           "algorithmic_bytes": {"leaves": b_leaves, "reconstruct": b_rec, "adapt": b_adapt},
           "achieved_GBps": {"leaves": gbs(b_leaves, t_leaves), "reconstruct": gbs(b_rec, t_rec),
                             "adapt": gbs(b_adapt, t_adapt)},
           "hbm_peak_GBps": HBM_PEAK_GBS,
           "timing": "host wall around one synchronous call, median of %d" % args.reps}
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
