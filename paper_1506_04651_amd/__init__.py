"""Batched Radau5 reaction substep for MI355X (gfx950).

Every cell of an adaptive-grid leaf set integrates its own stiff system
du/dt = f(u) over one splitting substep with Radau5 (Descombes et al. §2.1,
§1 footnote; Hairer & Wanner, Solving ODEs II, §IV.8), in hand-written HIP
kernels behind the C ABI of ``include/rd.h``.  PyTorch supplies device memory
and streams only.

    import torch, paper_1506_04651_amd as rd
    u = torch.tensor(states, dtype=torch.float64, device="cuda")   # [m, n]
    nfail = rd.reaction_step(u, dt, rtol, atol, rd.OREGONATOR, params)
"""
from ._lib import (BYTECODE, FP64, JAC_ANALYTIC, JAC_FD, KINETICS, LINEAR, MIXED, NAGUMO,
                   ONE_LAUNCH, OREGONATOR, PERSISTENT, ROBERTSON, STAT_NAMES, NSTATS, load,
                   last_error)
from .api import (RdError, Session, diffusion_step, last_kernel_ms, mra_adapt, mra_leaves,
                  mra_reconstruct, persistent_grid, reaction_step, request_bytes,
                  set_default_variant, strang_step, variant_count, variant_lanes,
                  variant_name)

__all__ = ["FP64", "MIXED", "PERSISTENT", "ONE_LAUNCH", "OREGONATOR", "KINETICS",
           "NAGUMO", "LINEAR", "ROBERTSON", "BYTECODE", "JAC_ANALYTIC", "JAC_FD",
           "STAT_NAMES", "NSTATS", "load",
           "last_error", "RdError", "Session", "reaction_step", "diffusion_step",
           "strang_step", "mra_leaves", "mra_reconstruct", "mra_adapt", "last_kernel_ms",
           "persistent_grid", "request_bytes", "variant_count", "variant_name",
           "variant_lanes", "set_default_variant"]
