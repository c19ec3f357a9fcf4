"""Autotuner for the reaction-step kernels.

The library compiles several variants of each kernel: work-group size, the
waves-per-SIMD target the register allocator is held to (higher occupancy at
the price of spills), how many lanes must wait before the step-end block runs
(batching), how many lanes must be idle before a wave claims new cells (claim
rounds), whether the step parameters are staged in LDS or kept in scalar
registers, the layout of the per-lane LDS slots (lane columns or lane rows),
the wave issue priorities of the persistent schedule and, for the 16-lane
kernels, fused or separate broadcasts and 8 or 16 matrix columns per lane;
for the kinetics and linear models with m <= 4 also the number of lanes per
cell (one lane, 64 cells per wave, or a 16-lane group, 4 cells per wave).
Variants of one engine compute the same per-cell arithmetic and must give
bitwise the same states; a variant with another number of lanes per cell
runs other arithmetic (Gauss-Jordan inverses instead of LU) and is accepted
when every cell has the same counters (the same control decisions) and its
states agree to 1e-10 relative (floored at atol).  Which one is fastest depends on the model, m, the
precision and on the distribution of per-cell cost in the batch, so the choice
is measured: every
variant is timed on the caller's own batch (HIP events on the launch stream),
the fastest becomes the library default for (kind, m, precision, schedule),
and the result is cached in a JSON file keyed by device name.

CLI:  python -m paper_1506_04651_amd.autotune --workload oregonator_2d
"""
from __future__ import annotations

import argparse
import json
import os
import sys

from . import api
from ._lib import FP64, MIXED, ONE_LAUNCH, PERSISTENT

DEFAULT_CACHE = os.environ.get("RD_AUTOTUNE_CACHE",
                               os.path.join(os.path.expanduser("~"), ".cache", "rd_autotune.json"))


def _device_name():
    import torch
    return torch.cuda.get_device_name(0)


def _launch_ms(u, states0, dt, rtol, atol, kind, params, precision, schedule, variant):
    """Milliseconds of one step of one variant on a fresh copy of the states."""
    import torch
    stream = torch.cuda.current_stream()
    u.copy_(states0)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    api.reaction_step(u, dt, rtol, atol, kind, params, precision=precision,
                      schedule=schedule, variant=variant, async_=True)
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b)


def time_variant(states0, dt, rtol, atol, kind, params, precision, schedule, variant, reps=3):
    """Median milliseconds of `reps` launches of one variant (after one warm-up)."""
    import torch
    u = torch.empty_like(states0)
    times = [_launch_ms(u, states0, dt, rtol, atol, kind, params, precision, schedule, variant)
             for _ in range(reps + 1)][1:]
    times.sort()
    return times[len(times) // 2], u


def tune(states0, dt, rtol, atol, kind, params, precision=FP64, schedule=PERSISTENT, reps=3,
         apply=True, verbose=False):
    """Time every variant; make the fastest the default.  Returns
    {"best": v, "ms": {v: ms}, "names": {v: name}}.  Variants whose output
    differs bitwise from variant 1's are rejected (they must run the same
    per-cell arithmetic)."""
    import torch
    m, n = int(states0.shape[0]), int(states0.shape[1])
    nv = api.variant_count(kind, m, precision, schedule)
    res = {"ms": {}, "names": {}, "rejected": [], "lanes": {}}
    # correctness first: one launch of each variant with counters, compared
    # with variant 1
    ref = ref_st = None
    lanes1 = api.variant_lanes(kind, m, precision, schedule, 1)
    u = torch.empty_like(states0)
    st = torch.zeros((9, n), dtype=torch.int32, device=states0.device)
    ok = []
    for v in range(1, nv + 1):
        name = api.variant_name(kind, m, precision, schedule, v)
        if name is None:
            continue
        u.copy_(states0)
        api.reaction_step(u, dt, rtol, atol, kind, params, stats=st, precision=precision,
                          schedule=schedule, variant=v)
        lanes = api.variant_lanes(kind, m, precision, schedule, v)
        if ref is None:
            ref, ref_st = u.clone(), st.clone()
            same = True
        elif lanes == lanes1:
            same = torch.equal(u, ref) and torch.equal(st, ref_st)
        else:
            rel = (u - ref).abs() / torch.clamp(ref.abs(), min=max(atol, 1e-300))
            same = torch.equal(st, ref_st) and float(rel.max()) <= 1e-10
        if not same:
            res["rejected"].append(v)
            if verbose:
                print(f"  variant {v} {name}: output differs from variant 1, rejected",
                      file=sys.stderr)
            continue
        ok.append(v)
        res["names"][v] = name
        res["lanes"][v] = lanes
    # then `reps` rounds over all variants, so that clock and cache drift
    # falls on every variant alike; the median per variant
    times = {v: [] for v in ok}
    for _ in range(reps):
        for v in ok:
            times[v].append(_launch_ms(u, states0, dt, rtol, atol, kind, params, precision,
                                       schedule, v))
    for v in ok:
        t = sorted(times[v])
        res["ms"][v] = t[len(t) // 2]
        if verbose:
            print(f"  variant {v:2d} {res['names'][v]:45s} {res['ms'][v]:8.3f} ms",
                  file=sys.stderr, flush=True)
    best = min(res["ms"], key=res["ms"].get)
    res["best"] = best
    if apply:
        api.set_default_variant(kind, m, precision, schedule, best)
    return res


def save(results: dict, path: str = DEFAULT_CACHE):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    try:
        with open(path) as fh:
            cache = json.load(fh)
    except (OSError, ValueError):
        cache = {}
    cache.setdefault(_device_name(), {}).update(results)
    with open(path, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)


def apply_cache(path: str = DEFAULT_CACHE) -> int:
    """Set the cached best variants for this device as defaults; returns how many."""
    try:
        with open(path) as fh:
            cache = json.load(fh)
    except (OSError, ValueError):
        return 0
    n = 0
    for key, rec in cache.get(_device_name(), {}).items():
        kind, m, prec, sched = (int(x) for x in key.split(":")[:4])
        api.set_default_variant(kind, m, prec, sched, int(rec["best"]))
        n += 1
    return n


def main():
    import torch

    from . import workloads as W
    ap = argparse.ArgumentParser(description="time every kernel variant on a workload")
    ap.add_argument("--workload", default="oregonator_2d", choices=sorted(W.CONFIGS))
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--cache", default=DEFAULT_CACHE)
    args = ap.parse_args()
    w = W.CONFIGS[args.workload]()
    u0 = torch.tensor(w.states, dtype=torch.float64, device="cuda")
    out = {}
    for prec in (FP64, MIXED):
        for sched in (PERSISTENT, ONE_LAUNCH):
            print(f"{w.name} precision {prec} schedule {sched}", file=sys.stderr, flush=True)
            r = tune(u0, w.dt, w.rtol, w.atol, w.kind, w.params, prec, sched, args.reps,
                     verbose=True)
            out[f"{w.kind}:{w.m}:{prec}:{sched}:{w.name}"] = {"best": r["best"], "ms": r["ms"],
                                                              "names": r["names"]}
    save(out, args.cache)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
