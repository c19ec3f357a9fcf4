"""Measure the diffusion step (RKC stage kernels, HBM bound) and the Strang
step R_{dt/2} D_dt R_{dt/2} on the paper-constant BZ field.

The diffusion step's algorithmic HBM traffic per RKC step of s stages is
m n (24 + 40 (s - 1)) bytes: the first stage reads Y0 and writes F0 = A Y0
and Y1; each later stage reads Y0, F0, Y_{j-1} and Y_{j-2} and writes Y_j
(stencil neighbours of Y_{j-1} counted once).  Achieved bandwidth = those
bytes / measured time, against the 8 TB/s HBM3E peak.

CLI:  python -m paper_1506_04651_amd.bench_strang [--side 1024] [--dim 2]
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

HBM_PEAK_GBS = 8000.0
BZ_DIFF = [2.5e-3, 2.5e-3, 1.5e-3]


def diffusion_bytes(m: int, n: int, s: int) -> int:
    return m * n * (24 + 40 * (s - 1))


def main():
    import torch

    from . import api
    from . import workloads as W
    ap = argparse.ArgumentParser()
    ap.add_argument("--side", type=int, default=1024)
    ap.add_argument("--dim", type=int, default=2, choices=[2, 3])
    ap.add_argument("--dt", type=float, default=1e-3)
    ap.add_argument("--reps", type=int, default=10)
    ap.add_argument("--strang-steps", type=int, default=5)
    args = ap.parse_args()
    torch.cuda.set_device(0)
    if args.dim == 2:
        w = W.oregonator_2d_paper(side=args.side, dt=args.dt)
        shape = (args.side, args.side)
        states = w.states
    else:
        side = args.side
        rng = np.random.default_rng(7)
        n = side ** 3
        states = np.vstack([rng.uniform(0, 0.1, n), rng.uniform(0, 1, n), rng.uniform(0, 0.2, n)])
        w = W.oregonator_2d_paper(side=64, dt=args.dt)
        shape = (side, side, side)
    h = 1.0 / args.side
    m, n = states.shape
    u0 = torch.tensor(states, dtype=torch.float64, device="cuda")
    u = u0.clone()
    stream = torch.cuda.current_stream()
    s = api.diffusion_step(u, shape, h, BZ_DIFF, args.dt)          # warm-up, workspace
    ms = []
    for _ in range(args.reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        api.diffusion_step(u, shape, h, BZ_DIFF, args.dt)
        b.record(stream)
        b.synchronize()
        ms.append(a.elapsed_time(b))
    ms.sort()
    dms = ms[len(ms) // 2]
    nbytes = diffusion_bytes(m, n, s)
    out = {"workload": f"bz_{'x'.join(map(str, shape))}", "cells": n, "m": m, "dt": args.dt,
           "rkc_stages": s, "diffusion_ms": dms,
           "diffusion_stage_ms": dms / s,
           "algorithmic_bytes": nbytes,
           "achieved_GBps": nbytes / (dms * 1e-3) / 1e9,
           "hbm_peak_GBps": HBM_PEAK_GBS}
    out["hbm_frac"] = out["achieved_GBps"] / HBM_PEAK_GBS
    if args.dim == 2 and args.strang_steps > 0:
        u = u0.clone()
        times = {"R1": [], "D": [], "R2": []}
        for _ in range(args.strang_steps):
            for key, fn in (("R1", lambda: api.reaction_step(u, args.dt / 2, w.rtol, w.atol, w.kind,
                                                              w.params)),
                            ("D", lambda: api.diffusion_step(u, shape, h, BZ_DIFF, args.dt)),
                            ("R2", lambda: api.reaction_step(u, args.dt / 2, w.rtol, w.atol, w.kind,
                                                              w.params))):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                fn()
                b.record(stream)
                b.synchronize()
                times[key].append(a.elapsed_time(b))
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        api.strang_step(u, shape, h, BZ_DIFF, args.dt, w.rtol, w.atol, w.kind, w.params)
        b.record(stream)
        b.synchronize()
        out["strang_ms"] = a.elapsed_time(b)
        # whole split steps on a side stream, eager and replayed from one
        # recorded graph, alternating (the field keeps evolving)
        side = torch.cuda.Stream()
        tt = {"eager": [], "graph": []}
        for k in range(2 * args.strang_steps + 2):
            mode = "graph" if k % 2 else "eager"
            with torch.cuda.stream(side):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(side)
                api.strang_step(u, shape, h, BZ_DIFF, args.dt, w.rtol, w.atol, w.kind, w.params,
                                stream=side, use_graph=(mode == "graph"))
                b.record(side)
            b.synchronize()
            if k >= 2:
                tt[mode].append(a.elapsed_time(b))
        out["strang_ms_median"] = {k: float(np.median(v)) for k, v in tt.items()}
        out["strang_breakdown_ms_median"] = {k: float(np.median(v)) for k, v in times.items()}
        tot = sum(out["strang_breakdown_ms_median"].values())
        out["reaction_share"] = (out["strang_breakdown_ms_median"]["R1"] +
                                 out["strang_breakdown_ms_median"]["R2"]) / tot
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
