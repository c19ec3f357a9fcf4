#!/usr/bin/env python3
"""Benchmark of the Radau5 reaction substep on one MI355X.

One "step" is one reaction substep over a whole synthetic leaf set: the
states are restored from a resident copy (a device-to-device copy of
2*8*m bytes per cell) and every cell is integrated over dt with Radau5 by the
HIP kernels.  Default workload: the 160^3 BZ/Oregonator scroll-wave leaf set
(4 194 304 cells, m = 3, dt = 1/64, rtol = 1e-5, atol = 1e-8), FP64,
persistent work-stealing kernel.  Beside it, in the same JSON line: the
one-launch schedule and the mixed-precision path on the same cells (error
against the FP64 result), the m = 16 kinetics batch (1 048 576 cells) in FP64
and mixed precision, and a replay of the Poisson request stream through a
serving session (p50 / p99 latency, aggregate rate).

Roofline: the FLOPs of a launch are counted from its per-cell counters with
the reference per-event counts (roofline.REFERENCE_COUNTS; also with the
counts of the kernels as written), divided by the main kernel's average
duration from the library's HIP events on the launch stream.

Prints ONE JSON line.  --gpus N with N > 1 exits: the reaction step needs no
communication, and the benchmark runs on one GPU.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Radau5 cell-integrations/s per split step, FP64 vs mixed; p50/p99 latency"

WORKLOADS = {
    "oregonator_2d": "BZ/Oregonator 512x512 spiral field, 262144 cells, m=3, dt=1/64",
    "oregonator_1d": "BZ/Oregonator 1D fronts, 4096 cells, m=3, dt=1/256",
    "oregonator_3d": "BZ/Oregonator 160^3 scroll wave, 4194304 cells, m=3, dt=1/64",
    "kinetics16": "synthetic stiff kinetics, 1048576 cells, m=16, dt=1e-2",
}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def make_workload(name):
    from paper_1506_04651_amd import workloads as W
    return {"oregonator_2d": W.oregonator_2d, "oregonator_1d": W.oregonator_1d,
            "oregonator_3d": W.oregonator_3d, "kinetics16": W.kinetics16}[name]()


def time_path(rd, torch, w, u0, steps, warmup, **opts):
    """Time `steps` reaction substeps; returns dict with wall and per-launch times."""
    u = torch.empty_like(u0)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        u.copy_(u0)
        rd.reaction_step(u, w.dt, w.rtol, w.atol, w.kind, w.params, async_=True, **opts)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        u.copy_(u0)
        ev[i][0].record(stream)
        rd.reaction_step(u, w.dt, w.rtol, w.atol, w.kind, w.params, async_=True, **opts)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = sorted(a.elapsed_time(b) for a, b in ev)
    import numpy as np
    return {"wall_s": wall, "launch_ms": ms, "avg_launch_ms": float(np.mean(ms)),
            "p50_ms": float(np.percentile(ms, 50)), "p99_ms": float(np.percentile(ms, 99)),
            "value": w.n * steps / wall, "out": u}


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def step_histogram(nstep):
    """Per-cell step counts (attempts) of one launch: octave bins and
    percentiles."""
    import numpy as np
    edges = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1 << 30]
    counts, _ = np.histogram(nstep, bins=edges)
    return {"bin_lo": edges[:-1], "cells": [int(c) for c in counts],
            "p50": float(np.percentile(nstep, 50)), "p90": float(np.percentile(nstep, 90)),
            "p99": float(np.percentile(nstep, 99)), "max": int(nstep.max())}


def kernel_source_sha():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1506_04651_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h", ".cpp")):
            with open(os.path.join(csrc, f), "rb") as fh:
                h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_name, workload):
    """HBM bytes per launch from a committed rocprofv3 PMC summary, if it was
    taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = rec.get(f"{kernel_name}@{workload}")
    if not ent or ent.get("kernel_source_sha") != kernel_source_sha():
        return None
    return ent.get("hbm_bytes_per_launch")


def kernel_times(rd, torch, w, u0, steps, **opts):
    """Durations of the main kernel (the library's HIP events around it on the
    launch stream) over `steps` launches, each awaited before the next."""
    u = torch.empty_like(u0)
    kms = []
    for _ in range(steps):
        u.copy_(u0)
        rd.reaction_step(u, w.dt, w.rtol, w.atol, w.kind, w.params, async_=True, **opts)
        kms.append(rd.last_kernel_ms())
    return kms


def counter_pass(rd, torch, w, u0, **opts):
    """One launch with per-cell counters (identical in every launch: the
    integration is deterministic); returns (states, counters, failed)."""
    st = torch.zeros((9, w.n), dtype=torch.int32, device="cuda")
    u = u0.clone()
    nfail = rd.reaction_step(u, w.dt, w.rtol, w.atol, w.kind, w.params, stats=st, **opts)
    return u.cpu().numpy(), st.cpu().numpy(), int(nfail)


def roofline_block(roofline, w, stats, kernel_ms, mixed):
    """Algorithmic FLOP/s of the dominant kernel against the vector peak (FP64;
    for the mixed path the blended FP64 + FP32 bound)."""
    K = w.info.get("K")
    G = w.info.get("G")
    ref = roofline.reference_counts(w.kind, w.m)
    t = kernel_ms * 1e-3
    out = {"bound": "alu", "unit": "TFLOP/s", "avg_kernel_ms": kernel_ms}
    written = roofline.algorithmic_flops(stats, w.kind, w.m, mixed)
    if ref is not None:
        flops = roofline.reference_flops(stats, ref)
        out["flops_per_launch"] = flops
        out["counts"] = "reference per-event counts"
        if K is not None:
            refn = roofline.reference_counts(w.kind, w.m, K, G)
            out["flops_per_launch_nnz"] = roofline.reference_flops(stats, refn)
    else:
        flops = written
        out["flops_per_launch"] = flops
        out["counts"] = "kernels as written"
    out["flops_per_launch_as_written"] = written
    out["achieved"] = flops / t / 1e12
    if mixed and ref is not None:
        f32 = roofline.reference_fp32_flops(stats, w.kind, w.m)
        bound = roofline.blended_bound_s(flops - f32, f32)
        out["peak"] = flops / bound / 1e12
        out["peak_kind"] = "blended FP64 78.6 + FP32 157.3 TFLOP/s over the FP64/FP32 split"
        out["frac"] = bound / t
    else:
        out["peak"] = roofline.PEAK_FP64_VECTOR_TFLOPS
        out["peak_kind"] = "FP64 vector"
        out["frac"] = out["achieved"] / roofline.PEAK_FP64_VECTOR_TFLOPS
    out["frac_as_written"] = written / t / 1e12 / roofline.PEAK_FP64_VECTOR_TFLOPS
    if "flops_per_launch_nnz" in out:
        out["frac_nnz"] = out["flops_per_launch_nnz"] / t / 1e12 / roofline.PEAK_FP64_VECTOR_TFLOPS
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="oregonator_3d", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--schedule", default="persistent", choices=["persistent", "onelaunch"])
    ap.add_argument("--variant", type=int, default=0)
    ap.add_argument("--graph", action="store_true", help="replay a captured hipGraph per step")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip every side measurement (schedules, precisions, m = 16, serving)")
    ap.add_argument("--no-kinetics", action="store_true", help="skip the m = 16 side measurement")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving replay")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="time every compiled kernel variant first and run the fastest (the "
                         "default runs the library's default variant, which the committed "
                         "profiles cover)")
    ap.add_argument("--no-autotune", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the reaction step has no "
              "cross-cell communication, so more GPUs would each run their own persistent kernel "
              "on a contiguous, cost-balanced range of the Morton-ordered cells.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1506_04651_amd as rd
    from paper_1506_04651_amd import roofline

    rd.load()
    torch.cuda.set_device(0)
    log("workload", args.workload)
    w = make_workload(args.workload)
    prec = rd.FP64 if args.precision == "fp64" else rd.MIXED
    sched = rd.PERSISTENT if args.schedule == "persistent" else rd.ONE_LAUNCH
    opts = dict(precision=prec, schedule=sched, variant=args.variant, use_graph=args.graph)
    u0 = torch.tensor(w.states, dtype=torch.float64, device="cuda")

    tuning = {}
    if args.autotune and not args.no_autotune and args.variant == 0:
        from paper_1506_04651_amd import autotune
        for p in (rd.FP64, rd.MIXED):
            log("autotune precision", p)
            r = autotune.tune(u0, w.dt, w.rtol, w.atol, w.kind, w.params, p, sched,
                              reps=7 if w.m <= 4 else 2)
            tuning[f"precision{p}"] = {r["names"][v]: round(ms, 4) for v, ms in r["ms"].items()}

    log("counter pass")
    ref_out, stats, nfail = counter_pass(rd, torch, w, u0, **opts)

    log("timed run", args.precision, args.schedule, "steps", args.steps)
    main_run = time_path(rd, torch, w, u0, args.steps, args.warmup, **opts)
    out_main = main_run.pop("out").cpu().numpy()
    if not np.array_equal(out_main, ref_out):
        raise SystemExit("timed launches did not reproduce the counter pass bitwise")
    # the main kernel's duration over as many launches as the timed region
    kernel_ms = float(np.mean(kernel_times(rd, torch, w, u0, args.steps, **opts)))
    kname = rd.variant_name(w.kind, w.m, prec, sched, args.variant) or "?"
    roof = roofline_block(roofline, w, stats, kernel_ms, prec == rd.MIXED)
    traffic = measured_traffic(kname, args.workload)
    roof["traffic"] = traffic
    roof["traffic_source"] = ("rocprofv3 FETCH_SIZE + WRITE_SIZE of this kernel on these sources, "
                              "scaled by a device-to-device copy" if traffic else None)
    roof["avg_step_ms_events"] = main_run["avg_launch_ms"]
    roof["frac_of_step_time"] = roof["frac"] * kernel_ms / main_run["avg_launch_ms"]
    roof["algorithmic_bytes_per_launch"] = w.n * roofline.bytes_per_cell(w.m)
    roof["hbm_gbs_algorithmic"] = roof["algorithmic_bytes_per_launch"] / (kernel_ms * 1e-3) / 1e9

    compare = {}
    if not args.no_compare:
        for label, o in [("fp64_onelaunch", dict(precision=rd.FP64, schedule=rd.ONE_LAUNCH)),
                         ("fp64_persistent", dict(precision=rd.FP64, schedule=rd.PERSISTENT)),
                         ("mixed_persistent", dict(precision=rd.MIXED, schedule=rd.PERSISTENT)),
                         ("mixed_onelaunch", dict(precision=rd.MIXED, schedule=rd.ONE_LAUNCH))]:
            if o["precision"] == prec and o["schedule"] == sched:
                continue
            log("side run", label)
            r = time_path(rd, torch, w, u0, max(5, args.steps // 2), 1, **o)
            out = r.pop("out").cpu().numpy()
            err = np.max(np.abs(out - ref_out) / np.maximum(np.abs(ref_out), w.atol), axis=0)
            kms = float(np.mean(kernel_times(rd, torch, w, u0, 5, **o)))
            ent = {"value": r["value"], "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"],
                   "kernel_ms": kms,
                   "kernel": rd.variant_name(w.kind, w.m, o["precision"], o["schedule"], 0),
                   "max_rel_diff_vs_main": float(err.max()),
                   "frac_within_1e-8_of_main": float(np.mean(err <= 1e-8))}
            if o["precision"] == rd.MIXED:
                _, st_m, _ = counter_pass(rd, torch, w, u0, **o)
                rb = roofline_block(roofline, w, st_m, kms, True)
                ent["roofline_frac"] = rb["frac"]
                ent["counters_equal_main"] = bool(np.array_equal(st_m, stats))
            compare[label] = ent

        if not args.no_kinetics and args.workload != "kinetics16":
            log("side workload kinetics16")
            wk = make_workload("kinetics16")
            k0 = torch.tensor(wk.states, dtype=torch.float64, device="cuda")
            kref, kst, kfail = counter_pass(rd, torch, wk, k0, precision=rd.FP64)
            ent = {"workload": wk.name, "n_cells": wk.n, "m": wk.m, "dt": wk.dt,
                   "rtol": wk.rtol, "atol": wk.atol, "failed_cells": kfail}
            for label, p in (("fp64_persistent", rd.FP64), ("mixed_persistent", rd.MIXED)):
                r = time_path(rd, torch, wk, k0, 3, 1, precision=p)
                out = r.pop("out").cpu().numpy()
                kms = float(np.mean(kernel_times(rd, torch, wk, k0, 3, precision=p)))
                st_p = kst if p == rd.FP64 else counter_pass(rd, torch, wk, k0, precision=p)[1]
                rb = roofline_block(roofline, wk, st_p, kms, p == rd.MIXED)
                err = np.max(np.abs(out - kref) / np.maximum(np.abs(kref), wk.atol), axis=0)
                ent[label] = {"value": r["value"], "p50_ms": r["p50_ms"], "p99_ms": r["p99_ms"],
                              "kernel_ms": kms,
                              "kernel": rd.variant_name(wk.kind, wk.m, p, rd.PERSISTENT, 0),
                              "roofline_frac": rb["frac"],
                              "roofline_frac_nnz": rb.get("frac_nnz"),
                              "roofline_frac_as_written": rb["frac_as_written"],
                              "max_rel_diff_vs_fp64": float(err.max())}
            compare["kinetics16"] = ent
            del k0

        if not args.no_serving:
            log("serving replay,", args.serving_requests, "requests")
            from paper_1506_04651_amd import serving
            from paper_1506_04651_amd import workloads as W
            given = {"oreg3d": w} if args.workload == "oregonator_3d" else {}
            pools = serving.make_pools(given=given)
            sizes = {k: v["w"].n for k, v in pools.items()}
            reqs = W.serving_stream(args.serving_requests, pool_sizes=sizes)
            budget = 2 << 30
            # the stream at its nominal rate (200 requests/s, above the
            # device's capacity for it: latency is mostly queueing), then
            # with the arrival times stretched 2.5x (below capacity)
            for label, scale in (("serving", 1.0), ("serving_stretched_2.5x", 2.5)):
                with rd.Session(budget, n_streams=4, precision=rd.MIXED) as sess:
                    recs, wall, _ = serving.replay(sess, reqs, pools, scale)
                summ = serving.summarize(recs, wall)
                summ.update({"budget_bytes": budget, "precision": "mixed", "streams": 4,
                             "time_scale": scale,
                             "offered_cells_per_s": sum(len(r.idx) for r in reqs)
                             / (reqs[-1].t_arrival * scale)})
                compare[label] = summ
            del pools

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        from paper_1506_04651_amd import workloads as W
        ns = min(w.n, 262144 if w.m <= 4 else 2048)
        idx = W.sample_indices(w.n, ns, 77) if ns < w.n else slice(None)
        s = w.subset(idx) if ns < w.n else w
        nth = os.cpu_count() or 1
        log("cpu baseline: oracle on", s.n, "cells,", nth, "threads")
        # whole passes over the sample until about 10 s of wall time have run
        passes, el = 0, 0.0
        while passes == 0 or el < 10.0:
            t0 = time.perf_counter()
            oracle.reaction_step(s.states, s.dt, s.rtol, s.atol, s.kind, s.params, nthreads=nth)
            el += time.perf_counter() - t0
            passes += 1
        cpu = {"value": passes * s.n / el, "unit": "cell-integrations/s", "cores": nth,
               "kind": "oracle",
               "sample": (f"all {s.n} cells of {w.name}" if ns == w.n else
                          f"{s.n} cells of {w.name} (seeded sample)") +
                         f", {passes} passes, {el:.1f} s"}
        # one host core, on a smaller seeded sample, about 2 s
        n1 = min(w.n, 16384 if w.m <= 4 else 64)
        s1 = w.subset(W.sample_indices(w.n, n1, 78)) if n1 < w.n else w
        passes, el = 0, 0.0
        while passes == 0 or el < 2.0:
            t0 = time.perf_counter()
            oracle.reaction_step(s1.states, s1.dt, s1.rtol, s1.atol, s1.kind, s1.params, nthreads=1)
            el += time.perf_counter() - t0
            passes += 1
        cpu["one_core"] = {"value": passes * s1.n / el,
                           "sample": f"{s1.n} cells (seeded sample), {passes} passes, {el:.1f} s"}
        cpu["cpu_model"] = host_cpu_model()

    line = {
        "metric": METRIC,
        "value": main_run["value"],
        "unit": "cell-integrations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["wall_s"] * 1e3 / args.steps,
        "p50_ms": main_run["p50_ms"],
        "p99_ms": main_run["p99_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == rd.FP64 else "f64+f32lu",
        "data": "synthetic",
        "config": {"workload": w.name, "n_cells": w.n, "m": w.m, "dt": w.dt, "rtol": w.rtol,
                   "atol": w.atol, "precision": args.precision, "schedule": args.schedule,
                   "kernel": kname, "graph": bool(args.graph),
                   "failed_cells": int(nfail)},
        "roofline": roof,
        "cpu_baseline": cpu,
        "compare": compare,
        "autotune_ms": tuning,
        "counters_mean": {k: float(stats[i].mean()) for i, k in enumerate(rd.STAT_NAMES)},
        "nstep_hist": step_histogram(stats[1]),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
