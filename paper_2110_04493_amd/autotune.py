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


# ---------------------------------------------------------------- cached choices
# The tuned thresholds of a workload family are kept in a JSON file (path in
# $EXPM_TUNE_CACHE, default ~/.cache/paper_2110_04493_amd/tune.json), keyed by
# the GPU architecture and a shape bucket: powers of two of n, of the stored
# entries per row and of ||H||_1 (of the sums over instances, plus the
# instance count, for batches).  A bucket is tuned once, on the first input
# that falls in it; later inputs of the bucket reuse the choice.

import json
import math
import os


def cache_path() -> str:
    return os.environ.get("EXPM_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_2110_04493_amd", "tune.json")


def _arch(device) -> str:
    return torch.cuda.get_device_properties(device).gcnArchName.split(":")[0]


def _b2(x: float) -> int:
    return int(math.floor(math.log2(x))) if x > 0 else -1


def _norm1(crow, col, val) -> float:
    n = crow.numel() - 1
    cs = torch.zeros(n, dtype=torch.float64, device=val.device)
    cs.index_add_(0, col.long(), val.abs())
    return float(cs.max()) if n else 0.0


def shape_key(mats, device) -> str:
    """Architecture and shape bucket of one matrix or of a batch."""
    n = sum(m[0].numel() - 1 for m in mats)
    nnz = sum(m[2].numel() for m in mats)
    norm = sum(_norm1(*m) for m in mats)
    kind = "single" if len(mats) == 1 else f"batch{_b2(len(mats))}"
    return f"{_arch(device)}/{kind}/n{_b2(n)}/r{_b2(nnz / max(n, 1))}/h{_b2(norm)}"


def _load(path: str) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(path: str, key: str, entry: dict) -> None:
    data = _load(path)
    data[key] = entry
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + f".tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuned_options(crow, col, val, eps: float, *, base: api.Options | None = None,
                  with_adjoint: bool = False, fills=FILLS, reorders=REORDERS):
    """Options for one matrix from the cache, tuning its bucket on a miss.
    Returns (Options, cached: bool)."""
    base = base or api.Options()
    key = shape_key([(crow, col, val)], val.device) + ("/adj" if with_adjoint else "")
    path = cache_path()
    hit = _load(path).get(key)
    if hit is not None:
        return replace(base, tile_min_fill=float(hit["tile_min_fill"]),
                       reorder=int(hit["reorder"])), True
    opts, times = autotune(crow, col, val, eps, base=base, fills=fills, reorders=reorders,
                           with_adjoint=with_adjoint)
    _store(path, key, {"tile_min_fill": opts.tile_min_fill, "reorder": opts.reorder,
                       "seconds": min(times.values())})
    return opts, False


def autotune_batched(mats, eps, *, base: api.Options | None = None, fills=FILLS,
                     repeats: int = 2, verbose: bool = False):
    """The batched path's tile threshold: times expm_sparse_batched on the
    caller's instances for each candidate fill.  Returns (best Options,
    {tile_min_fill: seconds})."""
    base = base or api.Options()
    times = {}
    for fill in fills:
        plan = api.Plan(mats[0][2].device, replace(base, tile_min_fill=float(fill)))
        try:
            def once():
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                outs = plan.expm_batched(mats, eps)
                torch.cuda.synchronize()
                del outs
                return time.perf_counter() - t0
            once()
            times[fill] = min(once() for _ in range(repeats))
        finally:
            plan.close()
        if verbose:
            print(f"[autotune batched] tile_min_fill={fill}: {times[fill] * 1e3:.2f} ms",
                  flush=True)
    fill = min(times, key=times.get)
    return replace(base, tile_min_fill=float(fill)), times


def tuned_batched_options(mats, eps, *, base: api.Options | None = None, fills=FILLS):
    """Options for a batch from the cache, tuning its bucket on a miss.
    Returns (Options, cached: bool)."""
    base = base or api.Options()
    key = shape_key(mats, mats[0][2].device)
    path = cache_path()
    hit = _load(path).get(key)
    if hit is not None:
        return replace(base, tile_min_fill=float(hit["tile_min_fill"])), True
    opts, times = autotune_batched(mats, eps, base=base, fills=fills)
    _store(path, key, {"tile_min_fill": opts.tile_min_fill, "seconds": min(times.values())})
    return opts, False
