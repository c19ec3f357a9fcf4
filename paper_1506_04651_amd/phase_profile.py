"""Where a persistent reaction-step kernel spends its time, phase by phase.

Runs a workload through the diagnostic copy of the library built with
RD_PHASE_PROFILE (`python -m paper_1506_04651_amd.build --phase-profile`,
which writes librd_phase.so beside librd.so and leaves librd.so alone).  In
that build every wave of the persistent kernels accumulates, per phase, the
shader-clock cycles from the phase's start to its end, the lanes active and
the number of times the phase ran (rd_phase.h).  Printed per phase: its
share of the waves' time in the kernel, how often it ran per wave, the mean
active lanes, and cycles per run.  The cycles are wall time of the wave
(including time it waits for memory or for issue while its SIMD runs other
waves), so shares describe where waves are, not which unit is busy; the
counting itself adds a few percent to the kernel time.

Phases: newton (one simplified-Newton iteration of the iterating lanes),
finish (error estimate and step control), start (Jacobian, factorization,
Newton start values; factor is the factorization inside it), claim (the
scheduling loop's claim, load and store of cells).

CLI:  python -m paper_1506_04651_amd.phase_profile --workload oregonator_3d [--precision mixed]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import os

PHASES = ["newton", "finish", "start", "factor", "claim", "kernel"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="oregonator_3d")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--launches", type=int, default=3)
    args = ap.parse_args()
    from . import _lib
    from . import build as B
    if not os.path.exists(B.PHASE_LIB):
        raise SystemExit(f"{B.PHASE_LIB} is not built: run "
                         "`python -m paper_1506_04651_amd.build --phase-profile`")
    _lib.LIB_PATH = B.PHASE_LIB
    import torch

    from . import api
    from . import workloads as W
    lib = _lib.load()
    readers = [getattr(ctypes.CDLL(B.PHASE_LIB), n) for n in ("rd_phase_read_small",
                                                               "rd_phase_read_group")]
    n_words = 3 * len(PHASES)
    buf = (ctypes.c_ulonglong * n_words)()
    w = W.CONFIGS[args.workload]()
    prec = 1 if args.precision == "mixed" else 0
    u0 = torch.tensor(w.states, dtype=torch.float64, device="cuda")
    u = u0.clone()
    api.reaction_step(u, w.dt, w.rtol, w.atol, w.kind, w.params, precision=prec)  # warm-up
    torch.cuda.synchronize()
    for r in readers:
        r(buf, 1)
    ms = []
    for _ in range(args.launches):
        u = u0.clone()
        torch.cuda.synchronize()
        api.reaction_step(u, w.dt, w.rtol, w.atol, w.kind, w.params, precision=prec)
        torch.cuda.synchronize()
        ms.append(api.last_kernel_ms())
    tot = [0] * n_words
    for r in readers:
        if r(buf, 0) != 0:
            raise SystemExit("reading the phase counters failed")
        tot = [a + b for a, b in zip(tot, buf)]
    kernel = tot[PHASES.index("kernel")]
    n_waves = tot[2 * len(PHASES) + PHASES.index("kernel")]
    out = {"workload": w.name, "precision": args.precision,
           "kernel": api.variant_name(w.kind, w.m, prec, api.PERSISTENT, 0),
           "kernel_ms": sorted(ms)[len(ms) // 2], "waves": n_waves, "phases": {}}
    for i, name in enumerate(PHASES[:-1]):
        cyc, lanes, runs = tot[i], tot[len(PHASES) + i], tot[2 * len(PHASES) + i]
        out["phases"][name] = {
            "share_of_wave_time": cyc / kernel if kernel else 0.0,
            "runs_per_wave": runs / n_waves if n_waves else 0.0,
            "mean_active_lanes": lanes / runs if runs else 0.0,
            "cycles_per_run": cyc / runs if runs else 0.0,
        }
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
