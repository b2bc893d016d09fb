#!/usr/bin/env python3
"""Benchmark: exact plan evaluations per second on the paper-scale warehouse.

One step = one call of the exact evaluator (``wo_eval_plans``) over one batch
of synthetic candidate plans already resident in HBM: 4,096 plans on the
400-aisle, 200,000-location warehouse with 4,000 orders (~10,000 items) and
capacity 30.  Prints one JSON line.

The roofline object reports the evaluation kernel against the plain integer
VALU roof; its algorithmic work per plan is 8 ops per pick + 4 per order +
12 per tour (tour counts come from a host-side next-fit count, reporting
only).  The cpu_baseline object times the CPU oracle on a bounded sample of
the same plans, on the host's cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 64 lanes x 2.4 GHz, one 32-bit integer op per lane per clock
INT_VALU_PEAK_OPS = 256 * 64 * 2.4e9
HBM_PEAK_BYTES = 8.0e12


def tour_counts(inst, seq: np.ndarray) -> np.ndarray:
    """Next-fit tour count per plan (reporting only: sizes the op count)."""
    lens = np.diff(inst.order_offsets).astype(np.int32)
    cnt = lens[seq.astype(np.int64)]
    load = np.zeros(seq.shape[0], dtype=np.int32)
    tours = np.zeros(seq.shape[0], dtype=np.int64)
    Q = inst.capacity
    for i in range(seq.shape[1]):
        c = cnt[:, i]
        new = (load + c > Q) | (i == 0)
        tours += new
        load = np.where(new, c, load + c)
    return tours


def algorithmic_ops(inst, seq: np.ndarray) -> float:
    T = tour_counts(inst, seq)
    n = seq.shape[0]
    return float(8 * inst.n_items * n + 4 * inst.n_orders * n + 12 * T.sum())


def cpu_baseline(inst, Z, S, min_wall_s: float = 1.5):
    import oracle
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    n = Z.shape[0]
    done, reps = 0, 0
    t0 = time.perf_counter()
    while True:
        oracle.eval_plans(inst, Z, S, n_threads=cores)
        done += n
        reps += 1
        el = time.perf_counter() - t0
        if el >= min_wall_s:
            break
    return {"value": done / el, "unit": "plans/s", "cores": cores, "kind": "oracle",
            "sample": "%d passes over the same %d plans (%.1f s wall, ~%.0f core-s)"
                      % (reps, n, el, el * cores)}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="paper", choices=["paper", "tiny"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported (the evaluator "
              "shards plans across GPUs with no exchange, see DESIGN.md)" % args.gpus, file=sys.stderr)
        return 2

    import torch

    import synth
    from paper_2110_13693_amd import wo

    torch.cuda.set_device(0)
    inst, Z, S = synth.workload(args.workload)
    n_plans = Z.shape[0]
    wh = wo.wo_load_warehouse([inst])
    z = torch.from_numpy(Z).cuda()
    s = torch.from_numpy(S.view(np.int16)).cuda().reshape(-1)
    dist = torch.empty(n_plans, dtype=torch.int32, device="cuda")
    thr = torch.empty(n_plans, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        wo.wo_eval_plans(wh, z, s, dist, thr, stream=stream)
    torch.cuda.synchronize()
    print("warmup done", file=sys.stderr, flush=True)

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for _ in range(args.steps):
        wo.wo_eval_plans(wh, z, s, dist, thr, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    ms_per_step = gpu_ms / args.steps
    value = n_plans * args.steps / (gpu_ms / 1e3)
    print("timed %d steps: %.4f ms/step (wall %.3f s)" % (args.steps, ms_per_step, wall),
          file=sys.stderr, flush=True)

    ops = algorithmic_ops(inst, S)
    # one launch per step: the kernel's average duration is the step time
    achieved_ops = ops / (ms_per_step / 1e3)
    roofline = {"bound": "alu", "achieved": achieved_ops / 1e12, "peak": INT_VALU_PEAK_OPS / 1e12,
                "unit": "Tops/s", "frac": achieved_ops / INT_VALU_PEAK_OPS, "traffic": None}

    out = {
        "metric": "exact plan evals/s @4k orders",
        "value": value,
        "unit": "plans/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32",
        "data": "synthetic",
        "config": {"workload": "paper-scale warehouse: 400 aisles x 2 x 250 slots, 150k SKUs in "
                               "64 categories, 4,000 orders (~10k items), capacity 30, 4,096 "
                               "plans per call" if args.workload == "paper" else "tiny warehouse",
                   "plans_per_step": n_plans, "orders": inst.n_orders, "items": inst.n_items,
                   "parallelism": "1 GPU"},
        "roofline": roofline,
    }
    d_host = dist.cpu().numpy()
    out["check"] = {"dist_min": int(d_host.min()), "dist_max": int(d_host.max())}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(inst, Z, S)
    wh.free()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
