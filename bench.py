#!/usr/bin/env python3
"""Benchmark: exact plan evaluations per second on the paper-scale warehouse.

One step = one call of the exact evaluator (``wo_eval_plans``) over one batch
of synthetic candidate plans already resident in HBM: 4,096 plans on the
400-aisle, 200,000-location warehouse with 4,000 orders (~10,000 items) and
capacity 30.  Prints one JSON line.

The roofline object reports the evaluation kernel against the plain integer
VALU roof; its algorithmic work per plan is 8 ops per pick + 4 per order +
12 per tour (tour counts come from a host-side next-fit count, reporting
only).  Its ``traffic`` is the kernel's HBM bytes per launch (FETCH_SIZE +
WRITE_SIZE, each scaled by its reading on a plain copy) from the committed
rocprofv3 summary, reported only while the kernel sources still hash to the
profiled ones.  The cpu_baseline object times the CPU oracle on a bounded sample of
the same plans, on the host's cores.
"""
from __future__ import annotations

import argparse
import dataclasses
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
# route of every tour: S-shape (the headline), return, largest gap, optimal, combined
ROUTES = {"sshape": 0, "return": 1, "largest-gap": 2, "optimal": 3, "combined": 4}
BATCHINGS = {"next-fit": 0, "first-fit": 1, "seed": 2}
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


def profiled_traffic():
    """HBM bytes per launch of the evaluation kernel, from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None when the kernel sources
    have changed since those counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "eval_plans_kernel_paper4096_hbm.md")
    try:
        fields = {}
        for line in open(path):
            if ":" in line and not line.startswith(("|", "#", "`")):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
        h = hashlib.sha256()
        for src in fields["kernel_sources"].split():
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
        if h.hexdigest() != fields["kernel_sources_sha256"]:
            return None
        return int(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads():
    """Threads the CPU baseline may use: the cores this process may run on,
    limited to the CPU share its environment declares (OMP_NUM_THREADS)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    share = os.environ.get("OMP_NUM_THREADS")
    used = min(avail, int(share)) if share and share.isdigit() and int(share) > 0 else avail
    return max(1, used), avail


def cpu_baseline(inst, Z, S, ops_per_plan: float, d_gpu, t_gpu, min_wall_s: float = 1.5):
    """The CPU oracle on the host's cores: all-threads and one-thread rates,
    the CPU roofline fraction, and the oracle's check of the GPU's results for
    the same plans (every plan of the timed call)."""
    import oracle
    cores, avail = host_threads()
    n = Z.shape[0]
    done, reps = 0, 0
    t0 = time.perf_counter()
    d_ref = t_ref = None
    while True:
        d, t = oracle.eval_plans(inst, Z, S, n_threads=cores)
        if d_ref is None:
            d_ref, t_ref = d, t
        done += n
        reps += 1
        el = time.perf_counter() - t0
        if el >= min_wall_s:
            break
    rate = done / el
    # one thread, on a bounded sample of the same plans
    m = min(n, 256)
    done1, t1 = 0, time.perf_counter()
    while True:
        oracle.eval_plans(inst, Z[:m], S[:m], n_threads=1)
        done1 += m
        el1 = time.perf_counter() - t1
        if el1 >= min_wall_s / 2:
            break
    rate1 = done1 / el1
    per_core = oracle.int_ops_per_second()
    achieved = ops_per_plan * rate
    mism_d = int(np.count_nonzero(d_ref != d_gpu))
    rel = np.abs(t_gpu.astype(np.float64) - t_ref) / np.maximum(np.abs(t_ref.astype(np.float64)), 1e-30)
    mism_t = int(np.count_nonzero(rel > 1e-6))
    return ({"value": rate, "unit": "plans/s", "cores": cores, "kind": "oracle",
             "sample": "%d passes over the same %d plans (%.1f s wall, ~%.0f core-s)" % (reps, n, el, el * cores),
             "cores_available": avail, "cpu_model": cpu_model(),
             "value_1core": rate1, "sample_1core": "%d plans, one thread (%.1f s)" % (done1, el1),
             "roofline": {"bound": "alu", "achieved": achieved / 1e9, "unit": "Gops/s",
                          "peak": cores * per_core / 1e9, "frac": achieved / (cores * per_core),
                          "peak_per_core": per_core / 1e9,
                          "note": "algorithmic ops (8/pick + 4/order + 12/tour) over cores x a measured "
                                  "scalar integer rate (8 independent add/xor chains)"}},
            {"oracle_plans_checked": n, "oracle_dist_mismatches": mism_d, "oracle_thr_mismatches": mism_t})


def search_comparison(args):
    """Plain genetic search vs surrogate-screened search at equal wall time.

    The ``--workload`` warehouse (the paper-scale one by default; ``tiny`` is
    the 12-category, 200-order one, where the one-hot input is zero-padded),
    population 16,384, tournament 4, mutation 0.02 per
    position; the screened arm proposes 65,536 children per generation and
    re-scores the best 3,277 exactly.  The surrogate is trained first on plans
    the exact evaluator scores (random slottings at the identity sequence);
    its data generation and training time are reported and counted both ways.
    Each of ``--seeds`` runs draws its own initial population, GA stream,
    training slottings and surrogate initialisation; the JSON line gives the
    median and range over the seeds of the screened/plain best-cost ratio at
    equal total wall time (training counted) and at equal search time, and of
    the time the screened arm takes to come within 0.5 % of the plain arm's
    final best, with and without its training.
    """
    import torch

    import synth
    from paper_2110_13693_amd import wo

    torch.cuda.set_device(0)
    inst = synth.WORKLOADS[args.workload]["make"](0)
    n = inst.n_orders
    P, K, keep = args.population, 65536, 3277
    wh = wo.wo_load_warehouse([inst])

    def run(sur, budget_s, max_gen, label, Z0, S0, ga_seed):
        s = wo.wo_search_create(wh, 0, Z0, S0, P, candidates=K if sur else 0, keep=keep if sur else 0,
                                seed=ga_seed)
        torch.cuda.synchronize()
        trace = [(0.0, wo.wo_search_best(s)[2])]
        t0 = time.perf_counter()
        g = 0
        while g < max_gen and (budget_s is None or time.perf_counter() - t0 < budget_s):
            wo.wo_search_step(wh, s, sur, 1)
            g += 1
            trace.append((time.perf_counter() - t0, wo.wo_search_best(s)[2]))
        best = wo.wo_search_best(s)
        s.free()
        print("%s: %d generations, %.2f s, best %d" % (label, g, trace[-1][0], best[2]),
              file=sys.stderr, flush=True)
        return trace, best

    # surrogate training pairs from the exact evaluator: random slottings
    # drawn on the device (argsort of seeded uniform keys) at the identity
    # order sequence
    def draw_slottings(gen, m):
        keys = torch.rand(m, inst.n_categories, generator=gen, device="cuda")
        z = torch.full((m, 64), 0xFF, dtype=torch.uint8, device="cuda")
        z[:, :inst.n_categories] = keys.argsort(dim=1).to(torch.uint8)
        return z

    draw_slottings(torch.Generator(device="cuda"), 4096)   # first-use set-up of these ops, untimed
    chunk = 16384
    seq_chunk = torch.arange(n, dtype=torch.int16, device="cuda").repeat(chunk)
    r_ho = np.random.default_rng([0, synth.generators.STREAM_SURROGATE_HELDOUT])
    zho = torch.from_numpy(synth.generators.random_zone_perms(r_ho, K, inst.n_categories)).cuda()
    dho = torch.empty(K, dtype=torch.int32, device="cuda")
    for c0 in range(0, K, chunk):
        wo.wo_eval_plans(wh, zho[c0:c0 + chunk], seq_chunk, dho[c0:c0 + chunk])
    torch.cuda.synchronize()
    ex = dho.cpu().numpy().astype(np.float64)

    def best_at(trace, t):
        b = trace[0][1]
        for tt, v in trace:
            if tt <= t:
                b = v
        return b

    def time_to(trace, thr):
        for t, v in trace:
            if v <= thr:
                return t
        return None

    from scipy.stats import spearmanr   # reporting only: rank correlation, average ranks for ties
    runs = []
    for i in range(args.seeds):
        rng = np.random.default_rng([i, synth.generators.STREAM_SEARCH_INIT])
        Z0 = torch.from_numpy(synth.generators.random_zone_perms(rng, P, inst.n_categories)).cuda()
        S0 = torch.from_numpy(synth.generators.random_order_perms(rng, P, n).view(np.int16)).cuda().reshape(-1)
        plain_trace, plain_best = run(None, None, args.generations, "seed %d plain" % i, Z0, S0, 11 + i)
        wall = plain_trace[-1][0]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gen = torch.Generator(device="cuda")
        gen.manual_seed(int(synth.generators.STREAM_SURROGATE_TRAIN) + 1000 * i)
        ztr = draw_slottings(gen, args.train_samples)
        dtr = torch.empty(args.train_samples, dtype=torch.int32, device="cuda")
        for c0 in range(0, args.train_samples, chunk):
            m = min(chunk, args.train_samples - c0)
            wo.wo_eval_plans(wh, ztr[c0:c0 + m], seq_chunk[:m * n], dtr[c0:c0 + m])
        torch.cuda.synchronize()
        t_data = time.perf_counter() - t0
        sur = wo.wo_sur_create(inst.n_categories, None, seed=1 + i)
        t1 = time.perf_counter()
        loss = wo.wo_sur_train(sur, ztr, dtr, epochs=args.epochs, batch=args.batch, lr=args.lr, seed=2 + i)
        t_train = time.perf_counter() - t1
        del ztr, dtr
        pho = torch.empty(K, dtype=torch.float32, device="cuda")
        wo.wo_sur_predict(sur, zho, pho)
        torch.cuda.synchronize()
        pr = pho.cpu().numpy().astype(np.float64)
        # the screened arm searches as long as the plain arm did; the trace
        # gives its best at equal search time and at equal total time (its
        # data generation and training counted)
        scr_trace, scr_best = run(sur, wall, 10 ** 9, "seed %d screened" % i, Z0, S0, 11 + i)
        sur.free()
        target = plain_best[2] * 1.005
        t_hit = time_to(scr_trace, target)
        t_prep = t_data + t_train
        runs.append({
            "seed": i, "plain_best": int(plain_best[2]), "plain_wall_s": wall,
            "plain_generations": len(plain_trace) - 1, "initial_best": int(plain_trace[0][1]),
            "screened_best_equal_search_time": int(scr_best[2]),
            "screened_best_equal_total_time": int(best_at(scr_trace, wall - t_prep)),
            "screened_generations": len(scr_trace) - 1,
            "time_to_within_0.5pct_s": t_hit,
            "time_to_within_0.5pct_incl_training_s": None if t_hit is None else t_hit + t_prep,
            "reaches_target_in_less_total_time": t_hit is not None and t_hit + t_prep < wall,
            "data_s": t_data, "train_s": t_train, "last_epoch_loss": loss,
            "heldout_rel_mae": float(np.mean(np.abs(pr - ex) / ex)),
            "heldout_spearman": float(spearmanr(pr, ex).correlation),
            "plain_best_plan": plain_best, "screened_best_plan": scr_best,
        })
    # throughput of the first seed's best plans from the evaluator itself
    r0 = runs[0]
    zb = torch.from_numpy(np.stack([r0["plain_best_plan"][0], r0["screened_best_plan"][0]])).cuda()
    sb = torch.from_numpy(np.concatenate([r0["plain_best_plan"][1], r0["screened_best_plan"][1]]).view(np.int16)).cuda()
    db = torch.empty(2, dtype=torch.int32, device="cuda")
    tb = torch.empty(2, dtype=torch.float32, device="cuda")
    wo.wo_eval_plans(wh, zb, sb, db, tb)
    torch.cuda.synchronize()
    thr_plain, thr_scr = [float(x) for x in tb.cpu().numpy()]
    for r in runs:
        del r["plain_best_plan"], r["screened_best_plan"]

    def stats(vals):
        v = np.array([x for x in vals if x is not None], dtype=np.float64)
        if v.size == 0:
            return None
        return {"median": float(np.median(v)), "min": float(v.min()), "max": float(v.max()), "n": int(v.size)}

    ratio_total = [r["screened_best_equal_total_time"] / r["plain_best"] for r in runs]
    ratio_search = [r["screened_best_equal_search_time"] / r["plain_best"] for r in runs]
    out = {
        "metric": "surrogate vs plain best cost at equal time",
        "value": float(np.median(ratio_total)),
        "unit": "screened best D / plain best D at equal total wall time (median over seeds)",
        "higher_is_better": False,
        "n_gpus": 1,
        "config": {"workload": "%s warehouse (%d categories, %d orders), population %d, %d generations of "
                               "plain search; screened: %d candidates, keep %d; %d seeds"
                               % ("paper-scale" if args.workload == "paper" else "tiny", inst.n_categories, n, P,
                                  args.generations, K, keep, args.seeds),
                   "surrogate": {"train_samples": args.train_samples, "epochs": args.epochs, "batch": args.batch,
                                 "lr": args.lr}},
        "summary": {
            "ratio_equal_total_time": stats(ratio_total),
            "ratio_equal_search_time": stats(ratio_search),
            "time_to_within_0.5pct_s": stats([r["time_to_within_0.5pct_s"] for r in runs]),
            "time_to_within_0.5pct_incl_training_s": stats([r["time_to_within_0.5pct_incl_training_s"] for r in runs]),
            "plain_wall_s": stats([r["plain_wall_s"] for r in runs]),
            "seeds_reaching_target_in_less_total_time": int(sum(r["reaches_target_in_less_total_time"] for r in runs)),
            "heldout_spearman": stats([r["heldout_spearman"] for r in runs]),
            "heldout_rel_mae": stats([r["heldout_rel_mae"] for r in runs]),
        },
        "orders_per_window_seed0": {"plain": thr_plain, "screened": thr_scr},
        "runs": runs,
    }
    wh.free()
    print(json.dumps(out), flush=True)
    return 0


def batched_bench(args):
    """Uneven instances in one launch: 512 warehouses (aisles and orders
    log-uniform) x 256 plans = 131,072 plans per call.  The launch
    configuration is autotuned first; the call is then timed eagerly and as
    a replayed graph."""
    import torch

    import synth
    from paper_2110_13693_amd import wo

    torch.cuda.set_device(0)
    per = 256
    insts = synth.make_batched_instances(512, seed=0)
    Z, S, _ = synth.generators.pack_batched_plans(insts, per, seed=0)
    offs = np.arange(len(insts) + 1, dtype=np.int64) * per
    n_plans = Z.shape[0]
    wh = wo.wo_load_warehouse(insts)
    z = torch.from_numpy(Z).cuda()
    s = torch.from_numpy(S.view(np.int16)).cuda()
    dist = torch.empty(n_plans, dtype=torch.int32, device="cuda")
    thr = torch.empty(n_plans, dtype=torch.float32, device="cuda")
    if args.no_autotune:
        best, table = wo.wo_get_eval_config(wh), []
    else:
        best, table = wo.wo_autotune_eval(wh, z, s, dist, plan_offsets=offs, reps=3)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        wo.wo_eval_plans(wh, z, s, dist, thr, plan_offsets=offs, stream=stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        wo.wo_eval_plans(wh, z, s, dist, thr, plan_offsets=offs, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    eager_ms = ev0.elapsed_time(ev1) / args.steps
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        wo.wo_eval_plans(wh, z, s, dist, thr, plan_offsets=offs, stream=side)
    stream.wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        wo.wo_eval_plans(wh, z, s, dist, thr, plan_offsets=offs, stream=torch.cuda.current_stream())
    g.replay()
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        g.replay()
    ev1.record(stream)
    torch.cuda.synchronize()
    graph_ms = ev0.elapsed_time(ev1) / args.steps
    ops = 0.0
    base = 0
    for inst in insts:
        seq = S[base:base + per * inst.n_orders].reshape(per, inst.n_orders)
        ops += algorithmic_ops(inst, seq)
        base += per * inst.n_orders
    achieved = ops / (graph_ms / 1e3)
    out = {
        "metric": "exact plan evals/s, 512 uneven instances",
        "value": n_plans / (graph_ms / 1e3),
        "unit": "plans/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": graph_ms, "eager_ms_per_step": eager_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "i32",
        "data": "synthetic",
        "config": {"workload": "512 warehouses, aisles log-uniform in [8, 400], orders log-uniform in "
                               "[50, 4000], capacity 30, 256 plans each (131,072 plans per call)",
                   "items": int(sum(i.n_items for i in insts)), "autotuned" if not args.no_autotune else "launch_config": best},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": INT_VALU_PEAK_OPS / 1e12,
                     "unit": "Tops/s", "frac": achieved / INT_VALU_PEAK_OPS, "traffic": None},
        "autotune_table": [[c["block_threads"], c["blocks_per_cu"], c["queue"], c["line_pass"],
                            c["small_orders"], round(c["ms"], 4)] for c in table],
    }
    wh.free()
    print(json.dumps(out), flush=True)
    return 0


# MFMA work of the surrogate per candidate: 2 (4096 x 1024 + 1024 x 256 + 256)
SUR_FWD_FLOP = 2.0 * (4096 * 1024 + 1024 * 256 + 256)
# one training sample: forward, input-gradient-free backward (two weight
# gradients and one activation gradient for the hidden layers)
SUR_TRAIN_FLOP = 18.35e6
BF16_PEAK_FLOPS = 2.5e15


def kmeans_bench(args):
    """K-means class-based storage on the paper-scale order history (10,006
    lines over 150,000 SKUs, 16 classes), one synchronous call per step."""
    import torch

    import synth
    from paper_2110_13693_amd import wo

    torch.cuda.set_device(0)
    inst, _, _ = synth.workload("paper", n_plans=1)
    k = 16
    skus = torch.from_numpy(np.ascontiguousarray(inst.order_skus, dtype=np.int32)).cuda()
    cat = torch.empty(inst.n_skus, dtype=torch.int32, device="cuda")
    for _ in range(args.warmup):
        wo.wo_kmeans_categories(skus, inst.n_skus, k, cat)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        used, iters = wo.wo_kmeans_categories(skus, inst.n_skus, k, cat)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    # algorithmic bytes of a call: the order lines once, the frequency of
    # every SKU written, read for the histogram and read for the label, and
    # the category written
    bytes_call = 4 * inst.n_items + 16 * inst.n_skus
    out = {"metric": "K-means class-based storage calls/s", "value": 1e3 / ms, "unit": "calls/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "i32/i64", "data": "synthetic",
           "config": {"workload": "pick frequencies of the paper-scale order history (10,006 lines over "
                                  "150,000 SKUs) clustered into %d classes" % k,
                      "classes_used": used, "assignments": iters, "parallelism": "1 GPU"},
           "roofline": {"bound": "hbm", "achieved": bytes_call / (ms / 1e3) / 1e9, "peak": HBM_PEAK_BYTES / 1e9,
                        "unit": "GB/s", "frac": bytes_call / (ms / 1e3) / HBM_PEAK_BYTES, "traffic": None}}
    if not args.no_cpu_baseline:
        from oracle import kmeans
        reps, t1 = 0, time.perf_counter()
        while time.perf_counter() - t1 < 1.5:
            kmeans.kmeans_categories(kmeans.pick_frequency(inst.n_skus, inst.order_skus), k)
            reps += 1
        dt = time.perf_counter() - t1
        out["cpu_baseline"] = {"value": reps / dt, "unit": "calls/s", "cores": 1, "kind": "oracle",
                               "sample": "%d calls on the same history (%.1f s)" % (reps, dt)}
    print(json.dumps(out), flush=True)
    return 0


def svm_bench(args):
    """Order categories (section 5, subroutine 5) on 1,048,576 synthetic typed
    orders over the paper-scale warehouse's 64 categories, 8 order types:
    features of every order, one training step on a window of 65,536 orders,
    and categories of every order.  The prediction pass reads each order's
    64 double features once: it is bound by HBM."""
    import torch

    import synth
    from paper_2110_13693_amd import wo

    torch.cuda.set_device(0)
    inst, _, _ = synth.workload("paper", n_plans=1)
    n, K, F, W = 1 << 20, 8, 64, 1 << 16
    off, skus, ty = synth.make_typed_orders(n, K, inst.sku_category, inst.n_categories, drift=0.5, seed=0)
    d_off = torch.from_numpy(off).cuda()
    d_sku = torch.from_numpy(skus).cuda()
    d_cat = torch.from_numpy(np.ascontiguousarray(inst.sku_category, np.int32)).cuda()
    d_ty = torch.from_numpy(ty).cuda()
    x = torch.empty((n, F), dtype=torch.float64, device="cuda")
    cls = torch.empty(n, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(reps):
            fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps

    feat_ms = timed(lambda: wo.wo_order_features(d_off, d_sku, d_cat, F, x), 10)
    m = wo.wo_svm_create(F, K, W, 1e-3)
    wo.wo_svm_push(m, x[n - W:], d_ty[n - W:])
    train_ms = timed(lambda: wo.wo_svm_train(m, 1), 5)
    wo.wo_svm_train(m, 100)
    pred_ms = timed(lambda: wo.wo_svm_predict(m, x, cls), 20)
    acc = float((cls[: n - W] == d_ty[: n - W]).float().mean().item())
    m.free()
    bytes_pred = n * (F * 8 + 4)
    out = {"metric": "order categories per second (SVM prediction)", "value": n / (pred_ms / 1e3),
           "unit": "orders/s", "n_gpus": 1, "steps": 20, "ms_per_step": pred_ms, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": {"workload": "1,048,576 typed orders (8 types, drifting), 64 categories of the paper-scale "
                                  "warehouse; window of 65,536 orders, lambda 1e-3",
                      "features_ms": feat_ms, "train_step_ms": train_ms,
                      "accuracy_on_older_orders_after_106_steps": acc},
           "roofline": {"bound": "hbm", "achieved": bytes_pred / (pred_ms / 1e3) / 1e9,
                        "peak": HBM_PEAK_BYTES / 1e9, "unit": "GB/s",
                        "frac": bytes_pred / (pred_ms / 1e3) / HBM_PEAK_BYTES, "traffic": None}}
    hbm_meas = wo.wo_measure_peaks(3)["hbm_read_bytes_per_s"]
    out["roofline"]["peak_measured"] = hbm_meas / 1e9
    out["roofline"]["frac_measured"] = bytes_pred / (pred_ms / 1e3) / hbm_meas
    print(json.dumps(out), flush=True)
    return 0


def aisle_bench(args):
    """Aisle-width design (section 5, Subproblem 1, Eq. (1)) for one plan of
    the paper-scale warehouse: racks 12 dm deep, cross aisles 30 dm, widths
    5 .. 404 dm (400 widths, every one evaluated exactly in one launch).  A
    call is synchronous (it returns the chosen width), so it is timed on the
    host; its CPU baseline is the oracle's sweep over a sample of widths."""
    import torch

    import synth
    from oracle import aisles as A
    from paper_2110_13693_amd import wo

    torch.cuda.set_device(0)
    inst, Z, S = synth.workload("paper", n_plans=1)
    wh = wo.wo_load_warehouse([inst])
    z = torch.from_numpy(Z).cuda()
    s = torch.from_numpy(S.view(np.int16)).cuda().reshape(-1)
    r, c, k, a0, a1 = 12, 30, 0.5, 5, 404
    for _ in range(3):
        res, dist = wo.wo_aisle_width(wh, z, s, r, c, k, a0, a1)
    torch.cuda.synchronize()
    reps = max(5, args.steps // 10)
    t0 = time.perf_counter()
    for _ in range(reps):
        res, dist = wo.wo_aisle_width(wh, z, s, r, c, k, a0, a1)
    dt = (time.perf_counter() - t0) / reps
    n_w = a1 - a0 + 1
    wh.free()
    # oracle check of sampled widths and its own rate
    sample = list(range(a0, a1 + 1, 40))
    t1 = time.perf_counter()
    ref = [A.distance_at(inst, Z[0], S[0], a + 2 * r) for a in sample]
    t_cpu = (time.perf_counter() - t1) / len(sample)
    mism = int(sum(int(dist[a - a0]) != d for a, d in zip(sample, ref)))
    out = {"metric": "aisle widths evaluated per second (Eq. (1) sweep)", "value": n_w / dt,
           "unit": "widths/s", "n_gpus": 1, "steps": reps, "ms_per_step": dt * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "i32", "data": "synthetic",
           "config": {"workload": "one plan of the paper-scale warehouse, racks 12 dm, cross aisles 30 dm, "
                                  "widths 5..404 dm, k 0.5", "result": res},
           "check": {"oracle_widths_checked": len(sample), "oracle_mismatches": mism},
           "cpu_baseline": {"value": 1.0 / t_cpu, "unit": "widths/s", "cores": 1, "kind": "oracle",
                            "sample": "%d widths of the same plan" % len(sample)}}
    print(json.dumps(out), flush=True)
    return 0


def surrogate_bench(args):
    """Surrogate throughput on the BF16 matrix cores: screening predictions
    (65,536 candidates per call) and training (batch 4,096), on random
    slottings of the 64-category paper warehouse."""
    import torch

    import synth
    from paper_2110_13693_amd import wo

    torch.cuda.set_device(0)
    rng = np.random.default_rng([0, synth.generators.STREAM_SURROGATE_TRAIN])
    K = 65536
    z = torch.from_numpy(synth.generators.random_zone_perms(rng, K, 64)).cuda()
    pred = torch.empty(K, dtype=torch.float32, device="cuda")
    sur = wo.wo_sur_create(64, None, seed=1)
    wo.wo_sur_set_scale(sur, 2.3e7, 2.0e5)
    stream = torch.cuda.current_stream()
    for _ in range(3):
        wo.wo_sur_predict(sur, z, pred, stream=stream)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = max(5, args.steps // 10)
    ev0.record(stream)
    for _ in range(reps):
        wo.wo_sur_predict(sur, z, pred, stream=stream)
    ev1.record(stream)
    torch.cuda.synchronize()
    pred_ms = ev0.elapsed_time(ev1) / reps
    n_train = 1 << 18
    zt = torch.from_numpy(synth.generators.random_zone_perms(rng, n_train, 64)).cuda()
    dt = torch.from_numpy(rng.integers(22_000_000, 24_000_000, n_train, dtype=np.int32)).cuda()
    wo.wo_sur_train(sur, zt[:8192], dt[:8192], epochs=1, batch=4096, lr=1e-4, seed=3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    wo.wo_sur_train(sur, zt, dt, epochs=1, batch=4096, lr=1e-4, seed=4)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    pred_flops = SUR_FWD_FLOP * K / (pred_ms / 1e3)
    train_flops = SUR_TRAIN_FLOP * n_train / train_s
    out = {
        "metric": "surrogate screening candidates/s",
        "value": K / (pred_ms / 1e3),
        "unit": "candidates/s",
        "n_gpus": 1, "steps": reps, "ms_per_step": pred_ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "MLP 4096-1024-256-1 on one-hot(64 x 64) slottings, 65,536 candidates "
                               "per call; training batch 4,096 over 262,144 samples"},
        "roofline": {"bound": "mfma", "achieved": pred_flops / 1e12, "peak": BF16_PEAK_FLOPS / 1e12,
                     "unit": "TFLOP/s", "frac": pred_flops / BF16_PEAK_FLOPS, "traffic": None},
        "train": {"samples_per_s": n_train / train_s, "epoch_s": train_s,
                  "achieved_tflops": train_flops / 1e12, "frac": train_flops / BF16_PEAK_FLOPS,
                  "note": "wall time of one epoch; shuffle and loss table on the device"},
    }
    sur.free()
    bf16_meas = wo.wo_measure_peaks(3)["bf16_flops_per_s"]
    out["roofline"]["peak_measured"] = bf16_meas / 1e12
    out["roofline"]["frac_measured"] = pred_flops / bf16_meas
    out["train"]["frac_measured"] = train_flops / bf16_meas
    print(json.dumps(out), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="paper", choices=["paper", "tiny"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--line-pass", type=int, default=None, choices=[0, 1, 2],
                    help="mapping of the aisle-set pass (0 instance order, 1 order per lane, 2 sequence order)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="--batched: keep the default launch configuration (for profiling the timed calls alone)")
    ap.add_argument("--autotune", action="store_true",
                    help="time every launch configuration first and keep the fastest (table in the JSON line)")
    ap.add_argument("--route", default="sshape", choices=list(ROUTES),
                    help="route of every tour (the default S-shape is the headline)")
    ap.add_argument("--batching", default="next-fit", choices=list(BATCHINGS),
                    help="order batching rule")
    ap.add_argument("--search", action="store_true",
                    help="run the plain vs surrogate-screened search comparison instead")
    ap.add_argument("--population", type=int, default=16384)
    ap.add_argument("--generations", type=int, default=200)
    ap.add_argument("--train-samples", type=int, default=1 << 20)
    ap.add_argument("--epochs", type=int, default=1, help="surrogate training epochs (search comparison)")
    ap.add_argument("--batch", type=int, default=4096, help="surrogate training batch (search comparison)")
    ap.add_argument("--lr", type=float, default=2e-3, help="surrogate learning rate (search comparison)")
    ap.add_argument("--seeds", type=int, default=5, help="independent search/surrogate seeds (search comparison)")
    ap.add_argument("--batched", action="store_true",
                    help="time the 512-instance uneven batch (autotuned, eager and graph replay) instead")
    ap.add_argument("--kmeans", action="store_true",
                    help="time K-means class-based storage on the paper-scale order history instead")
    ap.add_argument("--aisle", action="store_true",
                    help="time the aisle-width design (400 widths of one paper-scale plan) instead")
    ap.add_argument("--svm", action="store_true",
                    help="time order-category features, SVM training and prediction instead")
    ap.add_argument("--surrogate", action="store_true",
                    help="time surrogate screening and training on the matrix cores instead")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer 10 times (calibrates HBM byte counters)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print("bench.py measures one GPU only; --gpus %d is not supported (on several GPUs the "
              "evaluator would shard the plans, with no exchange between GPUs)" % args.gpus, file=sys.stderr)
        return 2

    if args.search:
        return search_comparison(args)
    if args.batched:
        return batched_bench(args)
    if args.surrogate:
        return surrogate_bench(args)
    if args.kmeans:
        return kmeans_bench(args)
    if args.svm:
        return svm_bench(args)
    if args.aisle:
        return aisle_bench(args)
    if args.copy_probe:
        import torch
        a = torch.empty(args.copy_probe << 20, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(10):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel(), "copies": 10}))
        return 0

    import torch

    import synth
    from paper_2110_13693_amd import wo

    torch.cuda.set_device(0)
    inst, Z, S = synth.workload(args.workload)
    inst = dataclasses.replace(inst, routing=ROUTES[args.route], batching=BATCHINGS[args.batching])
    n_plans = Z.shape[0]
    wh = wo.wo_load_warehouse([inst])
    z = torch.from_numpy(Z).cuda()
    s = torch.from_numpy(S.view(np.int16)).cuda().reshape(-1)
    dist = torch.empty(n_plans, dtype=torch.int32, device="cuda")
    thr = torch.empty(n_plans, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    if args.line_pass is not None:
        cfg = wo.wo_get_eval_config(wh)
        cfg["line_pass"] = args.line_pass
        wo.wo_set_eval_config(wh, **cfg)
    tuned = None
    if args.autotune:
        # every launch configuration timed on these plans; the fastest is kept
        best, table = wo.wo_autotune_eval(wh, z, s, dist, reps=5, stream=stream)
        tuned = {"best": best, "table": [[c["block_threads"], c["blocks_per_cu"], c["queue"], c["line_pass"],
                                          c["small_orders"], round(c["ms"], 4)] for c in table]}
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

    if args.batching == "next-fit":
        ops = algorithmic_ops(inst, S)
    else:
        # first fit's and seed batching's tours are not counted on the host:
        # the fewest tours possible, ceil(items / capacity), keeps the figure
        # a lower bound
        t_min = -(-inst.n_items // inst.capacity)
        ops = float((8 * inst.n_items + 4 * inst.n_orders + 12 * t_min) * S.shape[0])
        if args.batching == "seed":
            # each of the n joins (or seeds) follows a test of every order
            # not yet in a tour: n (n + 1) / 2 tests of 3 operations (fit,
            # key, minimum), a lower bound of the rule's work
            n = inst.n_orders
            ops += 3.0 * n * (n + 1) / 2 * S.shape[0]
    # one launch per step: the kernel's average duration is the step time
    achieved_ops = ops / (ms_per_step / 1e3)
    roofline = {"bound": "alu", "achieved": achieved_ops / 1e12, "peak": INT_VALU_PEAK_OPS / 1e12,
                "unit": "Tops/s", "frac": achieved_ops / INT_VALU_PEAK_OPS,
                "traffic": profiled_traffic() if (args.workload == "paper" and args.route == "sshape"
                                                  and args.batching == "next-fit"
                                                  and not args.line_pass and not args.autotune) else None}

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
                   "route": args.route, "batching": args.batching,
                   "plans_per_step": n_plans, "orders": inst.n_orders, "items": inst.n_items,
                   "parallelism": "1 GPU"},
        "roofline": roofline,
    }
    if args.line_pass is not None:
        out["config"]["line_pass"] = args.line_pass
    if tuned is not None:
        out["autotune"] = tuned
    if os.environ.get("WO_TILE_TOURS"):
        out["config"]["tile_tours_cap"] = int(os.environ["WO_TILE_TOURS"])
    # the device's own integer peak, beside the one from the unit counts
    peaks = wo.wo_measure_peaks(3)
    peak_meas = peaks["int_ops_per_s"]
    roofline["peak_measured"] = peak_meas / 1e12
    roofline["frac_measured"] = achieved_ops / peak_meas
    out["peaks_measured"] = {"int_valu_Tops": peaks["int_ops_per_s"] / 1e12,
                             "lds_read_TBps": peaks["lds_bytes_per_s"] / 1e12,
                             "hbm_read_TBps": peaks["hbm_read_bytes_per_s"] / 1e12,
                             "bf16_mfma_TFLOPs": peaks["bf16_flops_per_s"] / 1e12,
                             "l2_read_TBps": peaks["l2_read_bytes_per_s"] / 1e12}
    d_host = dist.cpu().numpy()
    t_host = thr.cpu().numpy()
    out["check"] = {"dist_min": int(d_host.min()), "dist_max": int(d_host.max())}
    if not args.no_cpu_baseline:
        base, chk = cpu_baseline(inst, Z, S, ops / n_plans, d_host, t_host)
        out["cpu_baseline"] = base
        out["check"].update(chk)
    wh.free()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
