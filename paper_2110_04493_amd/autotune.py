"""Autotuner for the product-path thresholds of one workload.

The squaring product runs either on scalar rows (Gustavson, bitmap-rank
accumulator) or on 16 x 16 tiles on the FP64 matrix cores, chosen per step
from the tile fill of the iterate (``tile_min_fill``), and the matrix may be
reordered for fuller tiles (``reorder``).  The best setting depends on the
matrix family, so this module times the forward pass (and optionally the
adjoint) on the caller's own matrix for a small grid of settings and returns
the fastest as ``api.Options``.  Every candidate runs on the GPU through the
same library; nothing here computes any part of the method.
"""
from __future__ import annotations

import itertools
import time
from dataclasses import replace

import torch

from . import api

FILLS = (0.0, 0.1, 0.2, 0.35, 0.5, 2.0)
REORDERS = (0, 1)


def _time_once(plan: api.Plan, crow, col, val, eps, with_adjoint: bool):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rp, ci, v = plan.expm(crow, col, val, eps)
    if with_adjoint:
        plan.backward(torch.ones_like(v), val.numel())   # adjoint of sum(E)
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def autotune(crow: torch.Tensor, col: torch.Tensor, val: torch.Tensor, eps: float, *,
             base: api.Options | None = None, fills=FILLS, reorders=REORDERS,
             with_adjoint: bool = False, repeats: int = 2, verbose: bool = False):
    """Returns (best Options, {(tile_min_fill, reorder): seconds}).

    Each setting runs once untimed, then ``repeats`` timed passes (the
    minimum counts).  With ``with_adjoint`` the adjoint of sum(E) is timed
    too (the plan keeps checkpoints)."""
    base = base or api.Options()
    if with_adjoint:
        base = replace(base, keep_checkpoints=True)
    times = {}
    for fill, ro in itertools.product(fills, reorders):
        opts = replace(base, tile_min_fill=float(fill), reorder=int(ro))
        plan = api.Plan(val.device, opts)
        try:
            _time_once(plan, crow, col, val, eps, with_adjoint)
            best = min(_time_once(plan, crow, col, val, eps, with_adjoint)
                       for _ in range(repeats))
        finally:
            plan.close()
        times[(fill, ro)] = best
        if verbose:
            print(f"[autotune] tile_min_fill={fill} reorder={ro}: {best * 1e3:.2f} ms", flush=True)
    (fill, ro), _ = min(times.items(), key=lambda kv: kv[1])
    return replace(base, tile_min_fill=float(fill), reorder=int(ro)), times
