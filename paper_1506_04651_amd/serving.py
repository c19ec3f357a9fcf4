"""Serving harness: an open-loop replay of a Poisson stream of reaction-step
requests through an rd_session (continuous batching by HBM budget).

Each request takes a batch of cells from one of three device-resident pools
(the 512^2 BZ spiral field, the BZ scroll-wave field and the m = 16 kinetics
field), a splitting step dt, and that generator's tolerances.  Requests are
submitted at their arrival times (optionally compressed), completions are
polled, and per-request latency (submit -> done, session clock) is reported
with p50 / p99 and the aggregate cell-integration rate.

CLI:  python -m paper_1506_04651_amd.serving --requests 2000 --budget-gib 2
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import api
from . import workloads as W
from ._lib import MIXED, PERSISTENT


def make_pools(small: bool = False, given=None):
    """Device-resident cell pools.  small=True uses reduced 3D / m=16 pools
    (for tests); the full pools are the benchmark's 2D, 3D and m=16 fields.
    given: already generated workloads to reuse, by pool name."""
    import torch
    given = given or {}
    o2 = given.get("oreg2d") or W.oregonator_2d()
    o3 = given.get("oreg3d") or (W.oregonator_3d(side=64, n_total=64 ** 3, check=False)
                                 if small else W.oregonator_3d())
    k16 = given.get("kin16") or (W.kinetics16(n=1 << 16) if small else W.kinetics16())
    pools = {}
    for name, w in (("oreg2d", o2), ("oreg3d", o3), ("kin16", k16)):
        pools[name] = {"w": w, "states": torch.tensor(w.states, dtype=torch.float64, device="cuda")}
    return pools


def gather(pool, idx):
    import torch
    t = torch.as_tensor(idx, device="cuda", dtype=torch.int64)
    return pool["states"].index_select(1, t).contiguous()


def replay(session: api.Session, requests, pools, time_scale: float = 1.0, keep_outputs=False,
           log=None):
    """Submit every request at t_arrival * time_scale (open loop), poll
    completions; returns a list of per-request dicts."""
    import torch
    # inputs prepared ahead (device gathers), so the timed loop only submits
    inputs = []
    for r in requests:
        p = pools[r.pool]
        inputs.append(gather(p, r.idx))
    torch.cuda.synchronize()
    recs = [None] * len(requests)
    pending = {}
    t0 = time.perf_counter()
    i = 0
    while i < len(requests) or pending:
        now = time.perf_counter() - t0
        while i < len(requests) and requests[i].t_arrival * time_scale <= now:
            r = requests[i]
            w = pools[r.pool]["w"]
            rid = session.submit(inputs[i], r.dt, w.rtol, w.atol, w.kind, w.params)
            pending[rid] = i
            i += 1
        done = []
        for rid, j in pending.items():
            info = session.poll(rid)
            if info is not None:
                done.append(rid)
                recs[j] = {"n": int(info.n_cells), "pool": requests[j].pool, "dt": requests[j].dt,
                           "latency_ms": (info.t_done_ns - info.t_submit_ns) * 1e-6,
                           "queue_ms": (info.t_admit_ns - info.t_submit_ns) * 1e-6,
                           "failed": int(info.n_failed), "status": int(info.status),
                           "batch": int(info.batch_id), "stream": int(info.stream),
                           "deferred": int(info.deferred),
                           "t_submit_ns": int(info.t_submit_ns),
                           "t_admit_ns": int(info.t_admit_ns), "t_done_ns": int(info.t_done_ns),
                           "kernel_start_ms": float(info.kernel_start_ms),
                           "kernel_end_ms": float(info.kernel_end_ms)}
                if not keep_outputs:
                    inputs[j] = None
        for rid in done:
            del pending[rid]
        if log and done:
            log(f"done {sum(r is not None for r in recs)}/{len(requests)}")
        if i < len(requests):
            nxt = requests[i].t_arrival * time_scale - (time.perf_counter() - t0)
            if nxt > 0 and not done:
                time.sleep(min(nxt, 5e-4))
        elif pending and not done:
            time.sleep(2e-4)
    wall = time.perf_counter() - t0
    return recs, wall, (inputs if keep_outputs else None)


def max_concurrent_kernels(recs):
    """Largest number of requests whose reaction-step kernels were running on
    the device at the same instant (device timestamps of the session)."""
    ev = []
    for r in recs:
        if r["kernel_start_ms"] >= 0.0 and r["kernel_end_ms"] > r["kernel_start_ms"]:
            ev.append((r["kernel_start_ms"], 1))
            ev.append((r["kernel_end_ms"], -1))
    best = cur = 0
    for _, d in sorted(ev, key=lambda e: (e[0], e[1])):
        cur += d
        best = max(best, cur)
    return best


def summarize(recs, wall):
    lat = np.array([r["latency_ms"] for r in recs])
    cells = sum(r["n"] for r in recs)
    out = {"requests": len(recs), "cells": cells, "wall_s": wall,
           "cell_integrations_per_s": cells / wall,
           "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
           "max_ms": float(lat.max()), "mean_queue_ms": float(np.mean([r["queue_ms"] for r in recs])),
           "failed_cells": int(sum(r["failed"] for r in recs)),
           "deferred_requests": int(sum(1 for r in recs if r["deferred"] > 0)),
           "max_concurrent_kernels": max_concurrent_kernels(recs),
           "errors": int(sum(1 for r in recs if r["status"] != 0))}
    for pool in sorted({r["pool"] for r in recs}):
        sel = [r for r in recs if r["pool"] == pool]
        pl = np.array([r["latency_ms"] for r in sel])
        out[f"{pool}_p50_ms"] = float(np.percentile(pl, 50))
        out[f"{pool}_p99_ms"] = float(np.percentile(pl, 99))
    return out


def main():
    import torch
    ap = argparse.ArgumentParser(description="replay a Poisson stream of reaction-step requests")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--budget-gib", type=float, default=2.0)
    ap.add_argument("--time-scale", type=float, default=1.0,
                    help="multiply arrival times (0.1 = 10x compressed)")
    ap.add_argument("--streams", type=int, default=4)
    ap.add_argument("--precision", default="mixed", choices=["fp64", "mixed"])
    ap.add_argument("--small-pools", action="store_true")
    args = ap.parse_args()
    torch.cuda.set_device(0)
    print("[serving] building pools", file=sys.stderr, flush=True)
    pools = make_pools(small=args.small_pools)
    sizes = {k: v["w"].n for k, v in pools.items()}
    reqs = W.serving_stream(args.requests, pool_sizes=sizes)
    prec = MIXED if args.precision == "mixed" else 0
    budget = int(args.budget_gib * (1 << 30))
    with api.Session(budget, n_streams=args.streams, precision=prec, schedule=PERSISTENT) as s:
        recs, wall, _ = replay(s, reqs, pools, args.time_scale,
                               log=lambda m: None)
    out = summarize(recs, wall)
    out.update({"budget_bytes": budget, "time_scale": args.time_scale, "streams": args.streams,
                "precision": args.precision, "offered_cells_per_s":
                sum(len(r.idx) for r in reqs) / (reqs[-1].t_arrival * args.time_scale)})
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
