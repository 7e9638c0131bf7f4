"""Benchmark: filtered precise-integration expm, forward + adjoint, on one GPU.

One step = one pass of the whole hot path on the 2D heat-conduction
workload (300 x 300 five-point grid, n = 90,000, lognormal(0, 0.5)
conductances, H = -tau L with ||H||_1 = 50, eps_tol = 1e-12): planning,
Taylor seed, N filtered squarings, E = I + T_N, then the adjoint of
L = sum(G .* E) (G: 2% dense, N(0,1), a counter-based synthetic matrix).
Inputs are resident on the device before timing starts.

Prints one JSON line.  `value` is the wall time of one step in seconds
(lower is better).  `roofline` covers the dominant kernel, the tile product
of the squarings: its launches are timed with HIP events on the library's
stream inside the timed steps (profile mode 2: event pairs only, read after
each call), and its algorithmic flops per launch come from untimed passes
after them, on a plan of their own, with the full profile (profile mode 1,
which counts the partial products of every step and waits for the device
after each step; the per-step table and phase times come from the second of
those passes).  The bound of each roofline object is the roof that the
kernel's arithmetic intensity (algorithmic flops per algorithmic byte) meets
first.  `adjoint` is the same for the adjoint tile step.  `other_workloads`
holds short measurements of the differentiation, large-grid, batched and
E R configurations.  `cpu_baseline` times the CPU oracle, forward +
adjoint, on the benchmark's own workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "expm wall time + squaring-SpGEMM HBM GB/s (% roofline) at n=90k; fwd+adjoint"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6      # MI355X FP64 vector (and FP64 matrix) peak
RIDGE = PEAK_FP64_TFLOPS * 1e12 / (PEAK_HBM_GBS * 1e9)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--side", type=int, default=300, help="grid side (300 -> n = 90,000)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-side", type=int, default=0,
                    help="time the oracle on a smaller grid of the same family instead of the "
                         "benchmark's own workload (0: the full workload, the default)")
    ap.add_argument("--cpu-runs", type=int, default=1,
                    help="oracle runs for the CPU baseline (the median is reported)")
    ap.add_argument("--cpu-only", action="store_true",
                    help="only time the CPU oracle (the cpu_baseline measurement, with the "
                         "thread count OMP_NUM_THREADS gives it) and print it as one JSON line; "
                         "the GPU is not used")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the lines of the other workloads (differentiation, large grid, "
                         "batched, E R) that follow the headline line")
    ap.add_argument("--forward-only", action="store_true")
    ap.add_argument("--workload", choices=["grid", "batched", "grad", "complex"], default="grid",
                    help="grid: the headline 2D heat-conduction workload (default); batched: "
                         "many uneven instances of the batched family in one call, timed "
                         "against a per-matrix loop; grad: the differentiation workload "
                         "(200 x 200 grid, forward + adjoint), timed against a forward-only "
                         "loop; complex: the complex entry point on the Schroedinger "
                         "propagator of the --side grid")
    ap.add_argument("--count", type=int, default=64, help="batched: number of instances")
    ap.add_argument("--nmin", type=int, default=500, help="batched: smallest n")
    ap.add_argument("--nmax", type=int, default=2000, help="batched: largest n")
    ap.add_argument("--wave-gb", type=float, default=0.0,
                    help="batched: run the instances in waves whose dense-output estimate "
                         "(60 n^2 bytes each: E, the iterates and the candidate as if dense) "
                         "stays within this many GB, each wave's outputs counted and freed "
                         "before the next (0: one call for all)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device copy of BYTES bytes three times (the "
                         "reference kernel for scaling HBM counter readings) and exit")
    return ap.parse_args()


# the tile kernels and the locality ordering that shapes their tiles
TILE_SOURCES = ("paper_2110_04493_amd/csrc/bsr.hip", "paper_2110_04493_amd/csrc/bsr_common.hpp",
                "paper_2110_04493_amd/csrc/reorder.hip")
TRAFFIC_FILE = "profiles/k_bsr_numeric_panel_grid300_traffic.md"


def kernel_source_digest() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in TILE_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(flop_per_launch: float):
    """HBM bytes per launch of the tile product from the committed counter
    summary, or None when it is absent, the kernel source has changed since
    the counters were taken, or the launches do different work (the summary's
    algorithmic flops per launch differ from this run's by more than 1%)."""
    path = os.path.join(ROOT, TRAFFIC_FILE)
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                kv[k.strip()] = v.strip().strip("`")
    if kv.get("kernel_source_sha256") != kernel_source_digest():
        return None
    try:
        ref = float(kv["algorithmic_flop_per_launch"])
        if abs(ref - flop_per_launch) > 0.01 * ref:
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def copy_calibration(nbytes: int):
    """A plain copy kernel of known size: torch's elementwise kernel for
    dst = src * 1 reads and writes nbytes each."""
    import torch
    n = nbytes // 8
    src = torch.rand(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 8, "launches": 3}), flush=True)


def kernel_roofline(flops: float, nbytes: float, ms: float) -> dict:
    """Roofline of one launch from its algorithmic flops and bytes: the
    bound is the roof its arithmetic intensity (flops per algorithmic byte)
    meets first, the achieved rate is in that roof's unit, and frac is
    achieved / peak, i.e. the launch's time at that roof over its measured
    time."""
    intensity = flops / nbytes if nbytes else float("inf")
    if intensity >= RIDGE:
        ach = flops / (ms * 1e9)
        out = {"bound": "mfma", "achieved": round(ach, 3), "peak": PEAK_FP64_TFLOPS,
               "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64_TFLOPS, 4)}
    else:
        ach = nbytes / (ms * 1e6)
        out = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS,
               "unit": "GB/s", "frac": round(ach / PEAK_HBM_GBS, 4)}
    out["flop_per_byte"] = round(intensity, 2)
    return out


def adjoint_roofline(tl: dict, pstats: dict, steps: int) -> dict:
    """The adjoint tile step (its two kernels under one event pair per step)
    against its roofline: launch times from the timed steps; algorithmic
    flops and bytes per launch from the profiled pass (2 per partial
    product of G T^T and T^T G landing in the mask plus 2 per mask entry;
    G and T read once, the masked output written once)."""
    if not tl["adj_launches"] or not pstats.get("adj_tile_launches"):
        return {"kernel": "k_bsr_adjoint", "launches": tl["adj_launches"]}
    avg_ms = tl["adj_ms"] / tl["adj_launches"]
    fl = pstats["adj_tile_flops"] / pstats["adj_tile_launches"]
    by = pstats["adj_tile_bytes"] / pstats["adj_tile_launches"]
    out = kernel_roofline(fl, by, avg_ms)
    out.update({"kernel": "k_bsr_adjoint", "launches": tl["adj_launches"],
                "avg_launch_ms": round(avg_ms, 4), "ms_per_step": round(tl["adj_ms"] / steps, 3),
                "algorithmic_flop_per_launch": round(fl),
                "algorithmic_bytes_per_launch": round(by)})
    return out


def numeric_roofline(stats: dict, n: int):
    """Algorithmic work of the numeric SpGEMM pass over all squaring steps.
    Per step i: flops = 2 * (partial products of T*T) + 2 * nnz(T_{i-1})
    (the 2T term), or, for a symmetric T on tiles (only the upper triangle
    formed), (fma + nnz) + (nnz + n), as the library counts it; bytes =
    12 * nnz(T_{i-1}) + 8 * (n + 1) (input CSR read once) + 12 * cand_i
    (candidate CSR written once)."""
    fl = by = t = 0.0
    per = []
    sym = bool(stats.get("symmetric", 0))
    for i in range(stats["N"]):
        fma, nin, cand = stats["sq_fma"][i], stats["sq_in"][i], stats["sq_cand"][i]
        if sym and stats["sq_tiles"][i]:
            f = float(fma + nin) + float(nin + n)
        else:
            f = 2.0 * fma + 2.0 * nin
        b = 12.0 * nin + 8.0 * (n + 1) + 12.0 * cand
        ms = stats["t_num_ms"][i]
        fl += f
        by += b
        t += ms
        per.append({"step": i + 1, "ms": round(ms, 4), "gbps": round(b / (ms * 1e6), 1),
                    "tflops": round(f / (ms * 1e9), 3), "cand": cand,
                    "path": "tiles" if stats["sq_tiles"][i] else "rows",
                    "tile_slots": 256 * stats["sq_tiles"][i],
                    "kept": stats["sq_kept"][i], "filter_iters": stats["sq_iters"][i]})
    return fl, by, t, per


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on exactly one GPU; --gpus N > 1 is not "
                                   "supported (see the multi-GPU design notes)"}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.cpu_only:
        from paper_2110_04493_amd import workloads as W
        H, _ = W.config2(args.side)
        print(json.dumps({"cpu_baseline": cpu_baseline(args, H.n)}), flush=True)
        return
    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "grad":
        bench_grad(args)
        return
    if args.workload == "complex":
        c = complex_numbers(args.side, args.warmup, args.steps)
        sec = c["forward_s"]
        print(json.dumps({"metric": "complex expm wall time (forward)", "value": sec,
                          "unit": "s", "n_gpus": 1, "steps": args.steps,
                          "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 3),
                          "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
                          "dtype": "c128", "data": "synthetic",
                          "config": {"workload": c["workload"], "parallelism": "single GPU"},
                          "roofline": c["squaring_numeric"], "detail": c}), flush=True)
        return
    import torch
    from paper_2110_04493_amd import api, workloads as W

    torch.cuda.set_device(0)
    H, eps = W.config2(args.side)
    n = H.n
    crow = torch.from_numpy(H.rowptr).cuda()
    col = torch.from_numpy(H.col).cuda()
    val = torch.from_numpy(H.val).cuda()
    dE = None

    def step(plan):
        nonlocal dE
        rp, ci, v = plan.expm(crow, col, val, eps)
        if not args.forward_only:
            if dE is None or dE.numel() != v.numel():
                # synthetic loss weights on E's support (built once, outside timing)
                rows = np.repeat(np.arange(n), np.diff(rp.cpu().numpy()))
                g = W.loss_weights(rows, ci.cpu().numpy(), n, density=0.02)
                dE = torch.from_numpy(g).cuda()
            plan.backward(dE, val.numel())
        return v.numel()

    # The timed steps run with the tile kernel timers only; untimed passes
    # with the full profile (phase timers and the algorithmic work of every
    # squaring step, which needs a wait after each step) follow on a plan of
    # their own.  The warmup calls also let the plan's workspace reach its
    # steady size (buffers that trade roles grow over the first calls).
    plan = api.Plan("cuda", api.Options(keep_checkpoints=not args.forward_only, profile=2))
    for _ in range(args.warmup):
        step(plan)
    torch.cuda.synchronize()
    times, fwd_ms, bwd_ms, stats = [], [], [], None
    tl = {"launches": 0, "ms": 0.0, "adj_launches": 0, "adj_ms": 0.0}
    t_all0 = time.perf_counter()
    for _ in range(args.steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nnz_e = step(plan)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        stats = plan.stats()
        fwd_ms.append(stats["t_total_ms"])
        bwd_ms.append(stats["t_backward_ms"] if not args.forward_only else 0.0)
        tl["launches"] += stats["tile_launches"]
        tl["ms"] += stats["tile_ms"]
        tl["adj_launches"] += stats["adj_tile_launches"]
        tl["adj_ms"] += stats["adj_tile_ms"]
    t_all = time.perf_counter() - t_all0
    plan.close()
    sec = t_all / args.steps
    pplan = api.Plan("cuda", api.Options(keep_checkpoints=not args.forward_only, profile=1))
    for _ in range(2):   # the first call also grows the plan's workspace
        step(pplan)
    torch.cuda.synchronize()
    pstats = pplan.stats()
    pplan.close()

    fl, by, tnum, per = numeric_roofline(pstats, n)
    tflops = fl / (tnum * 1e9)
    gbps = by / (tnum * 1e6)
    if tl["launches"]:
        # dominant kernel: the tile squaring product on FP64 matrix cores.
        # Launch durations from the timed steps; the algorithmic work of the
        # same launches (same input, same path) from the profiled pass.
        if pstats["tile_launches"] * args.steps != tl["launches"]:
            print("warning: the profiled pass launched the tile product "
                  f"{pstats['tile_launches']} times, a timed step "
                  f"{tl['launches'] / args.steps}", file=sys.stderr)
        avg_ms = tl["ms"] / tl["launches"]
        fl_launch = pstats["tile_flops"] / pstats["tile_launches"]
        by_launch = pstats["tile_bytes"] / pstats["tile_launches"]
        roof = kernel_roofline(fl_launch, by_launch, avg_ms)
        roof.update({"traffic": measured_traffic(fl_launch), "kernel": "k_bsr_numeric_panel",
                     "launches": tl["launches"], "avg_launch_ms": round(avg_ms, 4),
                     "algorithmic_flop_per_launch": round(fl_launch),
                     "algorithmic_bytes_per_launch": round(by_launch)})
    else:
        bound = "alu" if fl / by > RIDGE else "hbm"
        if bound == "alu":
            roof = {"bound": "alu", "achieved": round(tflops, 3), "peak": PEAK_FP64_TFLOPS,
                    "unit": "TFLOP/s", "frac": round(tflops / PEAK_FP64_TFLOPS, 4)}
        else:
            roof = {"bound": "hbm", "achieved": round(gbps, 1), "peak": PEAK_HBM_GBS,
                    "unit": "GB/s", "frac": round(gbps / PEAK_HBM_GBS, 4)}
        roof.update({"traffic": None, "kernel": "k_numeric"})
    t_bound = max(by / (PEAK_HBM_GBS * 1e9), fl / (PEAK_FP64_TFLOPS * 1e12)) * 1e3
    out = {
        "metric": METRIC, "value": round(sec, 5), "unit": "s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 3),
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"2D 5-point grid Laplacian {args.side}x{args.side} (n={n}), "
                               "lognormal(0,0.5) conductances, H=-tau*L with ||H||_1=50, "
                               "eps_tol=1e-12; forward expm"
                               + ("" if args.forward_only else
                                  " + adjoint of sum(G.*E), G 2% N(0,1)"),
                   "n": n, "nnz_h": int(H.nnz), "nnz_e": int(nnz_e), "M": stats["M"],
                   "N": stats["N"], "parallelism": "single GPU"},
        "forward_ms": round(float(np.median(fwd_ms)), 3),
        "adjoint_ms": round(float(np.median(bwd_ms)), 3),
        "roofline": roof,
        "adjoint": adjoint_roofline(tl, pstats, args.steps),
        "squaring_spgemm": {"kernel": "numeric pass (k_numeric rows / k_bsr_numeric tiles)",
                            "source": "untimed pass with per-step phase timers",
                            "ms": round(tnum, 3),
                            "algorithmic_GB": round(by / 1e9, 3),
                            "algorithmic_GFLOP": round(fl / 1e9, 2),
                            "hbm_gbps": round(gbps, 1), "hbm_frac": round(gbps / PEAK_HBM_GBS, 4),
                            "fp64_tflops": round(tflops, 3),
                            "roofline_frac": round(t_bound / tnum, 4),
                            "per_step": per},
        "phase_ms": {"source": "untimed pass with per-step phase timers",
                     "symbolic": round(sum(pstats["t_sym_ms"]), 3),
                     "numeric": round(tnum, 3),
                     "filter": round(sum(pstats["t_filter_ms"]), 3),
                     "taylor": round(pstats["t_taylor_ms"], 3)},
    }
    if not args.no_extras:
        out["other_workloads"] = other_workloads(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args, n)
    print(json.dumps(out), flush=True)


def _sync_time(fn):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0, out


def bench_batched(args):
    """Instances j = 0 .. count-1 of the batched family (even j: unit grid,
    tau ~ U[1, 20]; odd j: random adjacency, beta ~ U[0.1, 1]; eps 1e-12),
    n ~ U[nmin, nmax].  One expm_sparse_batched call against a loop of
    expm_sparse calls on the same plan options, both on resident inputs."""
    import torch
    from paper_2110_04493_amd import api, workloads as W
    torch.cuda.set_device(0)
    inst = [W.config4_instance(j, nmin=args.nmin, nmax=args.nmax) for j in range(args.count)]
    dev = [tuple(torch.from_numpy(a).cuda() for a in (H.rowptr, H.col, H.val)) for H, _ in inst]
    eps = [e for _, e in inst]
    # waves: instances in index order, each wave within the dense-output budget
    waves = [list(range(len(inst)))]
    if args.wave_gb > 0:
        waves, cur, used = [], [], 0.0
        for j, (H, _) in enumerate(inst):
            need = 60.0 * H.n * H.n / 1e9
            if cur and used + need > args.wave_gb:
                waves.append(cur)
                cur, used = [], 0.0
            cur.append(j)
            used += need
        if cur:
            waves.append(cur)
    plan = api.Plan("cuda", api.Options())

    def run_batched():
        nnz = 0
        for k, wv in enumerate(waves):
            outs = plan.expm_batched([dev[j] for j in wv], [eps[j] for j in wv])
            nnz += sum(int(o[2].numel()) for o in outs)
            del outs
            if len(waves) > 1:
                print(f"batched: wave {k + 1} of {len(waves)} done ({len(wv)} instances)",
                      file=sys.stderr, flush=True)
            if len(waves) > 1:
                # the outputs' memory goes back to the device for the
                # library's workspace of the next wave
                torch.cuda.empty_cache()
        return nnz

    def run_loop():
        nnz = 0
        for j, (d, e) in enumerate(zip(dev, eps)):
            out = plan.expm(*d, e)
            nnz += int(out[2].numel())
            del out
            if len(waves) > 1 and (j + 1) % 16 == 0:
                torch.cuda.synchronize()
                print(f"loop: {j + 1} of {len(dev)} instances done", file=sys.stderr, flush=True)
        return nnz

    tb, tl = [], []
    for it in range(args.warmup + args.steps):
        t_b, nnz_b = _sync_time(run_batched)
        t_l, nnz_l = _sync_time(run_loop)
        print(f"batched pass {it}: {t_b:.3f} s, loop {t_l:.3f} s", file=sys.stderr, flush=True)
        if it >= args.warmup:
            tb.append(t_b)
            tl.append(t_l)
    plan.close()
    assert nnz_b == nnz_l
    sec = float(np.median(tb))
    out = {"metric": "batched expm wall time (one call) vs per-matrix loop",
           "value": round(sec, 5), "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 3), "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"{args.count} instances of the batched family, n in "
                                  f"[{args.nmin}, {args.nmax}], half unit grids (tau in [1, 20]), "
                                  "half random adjacency (beta in [0.1, 1]), eps 1e-12",
                      "count": args.count, "sum_n": int(sum(H.n for H, _ in inst)),
                      "nnz_e_total": nnz_b, "waves": len(waves),
                      "parallelism": "single GPU"},
           "loop_s": round(float(np.median(tl)), 5),
           "speedup_vs_loop": round(float(np.median(tl)) / sec, 3)}
    print(json.dumps(out), flush=True)


def bench_grad(args):
    """The differentiation workload: 200 x 200 grid, lognormal(0, 0.5)
    conductances, H = -5 L / ||L||_1, eps 1e-12, loss sum(G .* E) with G 2%
    N(0, 1); forward + adjoint against the forward alone."""
    import torch
    from paper_2110_04493_amd import api, workloads as W
    torch.cuda.set_device(0)
    H, eps = W.config5(200)
    crow, col, val = (torch.from_numpy(a).cuda() for a in (H.rowptr, H.col, H.val))
    plan = api.Plan("cuda", api.Options(keep_checkpoints=True))
    rp, ci, v = plan.expm(crow, col, val, eps)
    rows = np.repeat(np.arange(H.n), np.diff(rp.cpu().numpy()))
    dE = torch.from_numpy(W.loss_weights(rows, ci.cpu().numpy(), H.n, density=0.02)).cuda()
    tf, tfb = [], []
    for it in range(args.warmup + args.steps):
        t1, _ = _sync_time(lambda: plan.expm(crow, col, val, eps))
        t2, _ = _sync_time(lambda: plan.backward(dE, val.numel()))
        if it >= args.warmup:
            tf.append(t1)
            tfb.append(t1 + t2)
    st = plan.stats()
    plan.close()
    sec = float(np.median(tfb))
    out = {"metric": "expm forward + adjoint wall time (differentiation workload)",
           "value": round(sec, 5), "unit": "s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(sec * 1e3, 3), "higher_is_better": False,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "2D 5-point grid 200x200 (n=40000), lognormal(0,0.5), "
                                  "H=-5L/||L||_1, eps 1e-12, loss sum(G.*E), G 2% N(0,1)",
                      "n": H.n, "nnz_e": int(st["nnz_e"]), "M": st["M"], "N": st["N"],
                      "parallelism": "single GPU"},
           "forward_s": round(float(np.median(tf)), 5),
           "adjoint_over_forward": round(sec / float(np.median(tf)) - 1.0, 3)}
    print(json.dumps(out), flush=True)


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(args, n_full):
    """The oracle, as it stands, on the host cores: forward + adjoint of the
    same workload (the full 300 x 300 grid by default; --cpu-sample-side
    picks a smaller grid of the same family, reported as measured, not
    scaled), the median of --cpu-runs runs, wall time of the oracle calls
    only (input generation and the loss weights excluded)."""
    import oracle
    from paper_2110_04493_amd import workloads as W
    side = args.cpu_sample_side or args.side
    H, eps = W.config2(side)
    times, fwd = [], []
    for r in range(max(args.cpu_runs, 1)):
        print(f"cpu_baseline: oracle run {r + 1} on the {side}x{side} grid", file=sys.stderr,
              flush=True)
        t0 = time.perf_counter()
        run = oracle.Run(H.rowptr, H.col, H.val, eps, keep=not args.forward_only)
        res = run.result()
        t1 = time.perf_counter()
        print(f"cpu_baseline: forward {t1 - t0:.1f} s", file=sys.stderr, flush=True)
        tb = 0.0
        if not args.forward_only:
            rows = np.repeat(np.arange(H.n), np.diff(res.rowptr))
            g = W.loss_weights(rows, res.col, H.n, density=0.02)
            t2 = time.perf_counter()
            run.backward(g)
            tb = time.perf_counter() - t2
            print(f"cpu_baseline: adjoint {tb:.1f} s", file=sys.stderr, flush=True)
        run.close()
        times.append(t1 - t0 + tb)
        fwd.append(t1 - t0)
    full = H.n == n_full
    return {"value": round(float(np.median(times)), 3), "unit": "s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": (f"oracle forward{'' if args.forward_only else ' + adjoint'} on "
                       + ("the benchmark's own workload" if full else
                          f"the {side}x{side} grid of the same family (n={H.n}; not scaled)")
                       + f", M={res.stats['M']}, N={res.stats['N']}, median of {len(times)} "
                       f"run(s), forward {np.median(fwd):.2f} s"),
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def other_workloads(args) -> dict:
    """Short measurements of the other configurations, after the headline:
    the differentiation workload (200 x 200 grid, forward + adjoint), the
    action E R of the headline E with R = rand(n, 1000) (section 5.3), the
    checkpoint placements, the large unit grid (1448 x 1448, one forward on
    a fresh plan: time, nnz(E), peak device memory), a complex H, and a
    batch of uneven instances against a per-matrix loop."""
    import torch
    from paper_2110_04493_amd import api, workloads as W
    out = {}
    print("other workloads: differentiation", file=sys.stderr, flush=True)
    out["differentiation"] = grad_numbers(3, 5)
    print("other workloads: action E R", file=sys.stderr, flush=True)
    out["action"] = action_numbers(args.side, 1000)
    print("other workloads: checkpoint placements", file=sys.stderr, flush=True)
    out["checkpoints"] = checkpoint_numbers(args.side)
    print("other workloads: large grid", file=sys.stderr, flush=True)
    out["large_grid"] = large_grid_numbers()
    print("other workloads: complex H", file=sys.stderr, flush=True)
    out["complex"] = complex_numbers(args.side, 1, 3)
    print("other workloads: batched", file=sys.stderr, flush=True)
    out["batched"] = batched_numbers(64, 500, 2000, 1, 3)
    print("other workloads: batched at the stated size range", file=sys.stderr, flush=True)
    out["batched_stated_range"] = batched_numbers(8, 500, 20000, 1, 1)
    return out


def complex_numbers(side: int, warmup: int, steps: int) -> dict:
    """The complex entry point on the discrete Schroedinger propagator
    H = -i t (L + V) of a side x side unit grid (t = 1, V ~ U[0, 1]): median
    forward time on a warm plan, and the sizes."""
    import torch
    from paper_2110_04493_amd import api, workloads as W
    H = W.schrodinger_grid(side, 1.0, vmax=1.0, seed=7000)
    dev = (torch.from_numpy(H.rowptr).cuda(), torch.from_numpy(H.col).cuda(),
           torch.from_numpy(H.val).cuda())
    plan = api.Plan("cuda")
    ts = []
    nnz = 0
    for it in range(warmup + steps):
        t, (rp, ci, v) = _sync_time(lambda: plan.expm_z(*dev, 1e-12))
        nnz = int(v.numel())
        del rp, ci, v
        if it >= warmup:
            ts.append(t)
    st = plan.stats()
    plan.close()
    # the squaring products' numeric pass (k_numeric_z) from an untimed pass
    # with per-step phase timers: 8 flops per complex partial product of
    # T T and 4 per stored entry of T (the 2T term); 20 bytes (value and
    # column) per stored entry of T read once, 8 (n + 1) for its row
    # pointer and 20 per candidate written once
    pplan = api.Plan("cuda", api.Options(profile=1))
    for _ in range(2):
        out = pplan.expm_z(*dev, 1e-12)
        del out
    torch.cuda.synchronize()
    ps = pplan.stats()
    pplan.close()
    n = side * side
    fl = sum(8.0 * f + 4.0 * k for f, k in zip(ps["sq_fma"], ps["sq_in"]))
    by = sum(20.0 * k + 8.0 * (n + 1) + 20.0 * c for k, c in zip(ps["sq_in"], ps["sq_cand"]))
    ms = sum(ps["t_num_ms"])
    bound = "alu" if fl / by > RIDGE else "hbm"
    if bound == "alu":
        ach = fl / (ms * 1e9)
        roof = {"bound": "alu", "achieved": round(ach, 3), "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64_TFLOPS, 4)}
    else:
        ach = by / (ms * 1e6)
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": round(ach / PEAK_HBM_GBS, 4)}
    roof.update({"kernel": "k_numeric_z (numeric pass of the squarings)", "ms": round(ms, 3),
                 "algorithmic_flop": fl, "algorithmic_bytes": by,
                 "flop_per_byte": round(fl / by, 2)})
    return {"workload": f"H = -i t (L + V), {side}x{side} unit grid (n={n}), t=1, "
                        "V ~ U[0,1], eps 1e-12, complex128, scalar-row path",
            "forward_s": round(float(np.median(ts)), 5), "M": st["M"], "N": st["N"],
            "normal": st["normal"], "nnz_e": nnz, "squaring_numeric": roof,
            "phase_ms": {"symbolic": round(sum(ps["t_sym_ms"]), 3), "numeric": round(ms, 3),
                         "filter": round(sum(ps["t_filter_ms"]), 3),
                         "taylor": round(ps["t_taylor_ms"], 3)}}


def checkpoint_numbers(side: int) -> dict:
    """The headline step (forward + adjoint) under four checkpoint
    placements: the default (every iterate while they fit a memory budget),
    the last ceil(sqrt(N)) iterates, every ceil(sqrt(N))-th iterate counted
    back from T_{N-1}, and every iterate;
    median step time of 4 steps after 2 warmup steps, and the device memory
    the plan holds by then (free memory before and after)."""
    import math
    import torch
    from paper_2110_04493_amd import api, workloads as W
    H, eps = W.config2(side)
    torch.cuda.empty_cache()
    dev = [torch.from_numpy(a).cuda() for a in (H.rowptr, H.col, H.val)]
    out = {}
    dE = None
    for name, interval in (("default", 0), ("last_sqrtN", -1), ("every_sqrtN", -2), ("all", 1)):
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        if interval == -2:
            probe = api.Plan("cuda")
            N = probe.analyze(*dev, eps)["N"]
            probe.close()
            interval = max(1, math.ceil(math.sqrt(N)))
        plan = api.Plan("cuda", api.Options(keep_checkpoints=True, checkpoint_interval=interval))
        ts = []
        for it in range(6):
            if dE is None:
                rp, ci, v = plan.expm(*dev, eps)
                rows = np.repeat(np.arange(H.n), np.diff(rp.cpu().numpy()))
                dE = torch.from_numpy(W.loss_weights(rows, ci.cpu().numpy(), H.n,
                                                     density=0.02)).cuda()
                plan.backward(dE, H.nnz)
                continue
            t, _ = _sync_time(lambda: (plan.expm(*dev, eps), plan.backward(dE, H.nnz)))
            if it >= 2:
                ts.append(t)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        plan.close()
        torch.cuda.empty_cache()
        out[name] = {"checkpoint_interval": interval, "step_s": round(float(np.median(ts)), 5),
                     "device_memory_gb": round((free0 - free1) / 1e9, 1)}
    return out


def grad_numbers(warmup: int, steps: int) -> dict:
    import torch
    from paper_2110_04493_amd import api, workloads as W
    H, eps = W.config5(200)
    crow, col, val = (torch.from_numpy(a).cuda() for a in (H.rowptr, H.col, H.val))
    plan = api.Plan("cuda", api.Options(keep_checkpoints=True))
    rp, ci, v = plan.expm(crow, col, val, eps)
    rows = np.repeat(np.arange(H.n), np.diff(rp.cpu().numpy()))
    dE = torch.from_numpy(W.loss_weights(rows, ci.cpu().numpy(), H.n, density=0.02)).cuda()
    tf, tfb = [], []
    for it in range(warmup + steps):
        t1, _ = _sync_time(lambda: plan.expm(crow, col, val, eps))
        t2, _ = _sync_time(lambda: plan.backward(dE, val.numel()))
        if it >= warmup:
            tf.append(t1)
            tfb.append(t1 + t2)
    st = plan.stats()
    plan.close()
    return {"workload": "200x200 grid (n=40000), lognormal(0,0.5), H=-5L/||L||_1, eps 1e-12, "
                        "loss sum(G.*E), G 2% N(0,1)",
            "fwd_adjoint_s": round(float(np.median(tfb)), 5),
            "forward_s": round(float(np.median(tf)), 5), "M": st["M"], "N": st["N"],
            "nnz_e": int(st["nnz_e"]), "steps": steps}


def action_numbers(side: int, m: int) -> dict:
    """Y = E R for the headline workload's E and R = rand(n, m): the time of
    one expm_spmm call (tile assembly of E plus the product) from HIP events
    on the product's stream; algorithmic flops 2 nnz(E) m,
    algorithmic bytes 12 nnz(E) + 8 (n + 1) + 16 n m (E read once, R read
    once, Y written once)."""
    import torch
    from paper_2110_04493_amd import api, workloads as W
    H, eps = W.config2(side)
    dev = [torch.from_numpy(a).cuda() for a in (H.rowptr, H.col, H.val)]
    plan = api.Plan("cuda")
    rp, ci, v = plan.expm(*dev, eps)
    R = torch.rand((H.n, m), dtype=torch.float64, device="cuda")
    Y = plan.spmm(rp, ci, v, R)   # warmup
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 3
    ms = []
    for _ in range(reps):
        with torch.cuda.stream(plan.stream):
            ev0.record(plan.stream)
            Y = plan.spmm(rp, ci, v, R)
            ev1.record(plan.stream)
        ev1.synchronize()
        ms.append(ev0.elapsed_time(ev1))
    nnz = int(v.numel())
    plan.close()
    t = float(np.median(ms))
    fl = 2.0 * nnz * m
    by = 12.0 * nnz + 8.0 * (H.n + 1) + 16.0 * H.n * m
    roof = kernel_roofline(fl, by, t)
    roof.update({"kernel": "k_spmm_tiles (E's 16x16 tiles built in the same call)",
                 "ms": round(t, 3), "algorithmic_flop": fl, "algorithmic_bytes": by})
    return {"workload": f"E of the {side}x{side} grid (nnz {nnz}) times rand(n, {m})",
            "roofline": roof}


def large_grid_numbers() -> dict:
    import torch
    from paper_2110_04493_amd import api, workloads as W
    H, eps = W.config3(1448)
    torch.cuda.empty_cache()
    dev = [torch.from_numpy(a).cuda() for a in (H.rowptr, H.col, H.val)]
    torch.cuda.synchronize()
    plan = api.Plan("cuda")
    t, (rp, ci, v) = _sync_time(lambda: plan.expm(*dev, eps))
    st = plan.stats()
    nnz = int(v.numel())
    del rp, ci, v
    t_warm, out = _sync_time(lambda: plan.expm(*dev, eps))
    del out
    plan.close()
    torch.cuda.empty_cache()
    return {"workload": "1448x1448 unit grid (n=2096704), H=-0.5L, eps 1e-10, one forward on a "
                        "fresh plan (allocation included), then one on the warm plan",
            "forward_s": round(t, 4), "forward_warm_s": round(t_warm, 4),
            "M": st["M"], "N": st["N"], "nnz_e": nnz,
            "library_workspace_peak_gib": round(st["peak_workspace_bytes"] / 2 ** 30, 2)}


def batched_numbers(count: int, nmin: int, nmax: int, warmup: int, steps: int) -> dict:
    import torch
    from paper_2110_04493_amd import api, workloads as W
    inst = [W.config4_instance(j, nmin=nmin, nmax=nmax) for j in range(count)]
    dev = [tuple(torch.from_numpy(a).cuda() for a in (H.rowptr, H.col, H.val)) for H, _ in inst]
    eps = [e for _, e in inst]
    plan = api.Plan("cuda", api.Options())
    tb, tl = [], []
    for it in range(warmup + steps):
        t_b, outs = _sync_time(lambda: plan.expm_batched(dev, eps))
        del outs
        t_l, outs = _sync_time(lambda: [plan.expm(*d, e) for d, e in zip(dev, eps)])
        del outs
        if it >= warmup:
            tb.append(t_b)
            tl.append(t_l)
    plan.close()
    return {"workload": f"{count} instances of the batched family, n in [{nmin}, {nmax}] "
                        "(half unit grids, tau in [1, 20]; half random adjacency, beta in "
                        "[0.1, 1]), eps 1e-12",
            "batched_s": round(float(np.median(tb)), 5),
            "loop_s": round(float(np.median(tl)), 5),
            "speedup_vs_loop": round(float(np.median(tl)) / float(np.median(tb)), 3)}


if __name__ == "__main__":
    main()
