"""Benchmarks of the batched and serving forms (used by bench.py --workload).

batch: 512 mazes (sides log-uniform in [128, 2048], Bernoulli(p), p ~ U[0.2,
       0.45], 1-8 sources, 16-512 targets; seeded).  One batched step =
       omap_batch_create + propagate (run-time L per maze) + extract paths +
       destroy.  Baseline: the plain per-maze loop (plan create + propagate +
       extract + destroy for each maze, one after another) on the same GPU.
serve: distinct maze queries (side log-uniform in [256, 8192], DFS maze with 2%
       removals or Bernoulli(0.35), 1-16 sources, 8-2048 targets; seeded),
       first all queued at once (capacity), then arriving as a Poisson process
       at 0.7 x that capacity; latency = completion - arrival, after the
       warm-up queries.  Baseline: the plain per-maze loop.
"""
from __future__ import annotations

import concurrent.futures as cf
import time

import numpy as np


def _log(*a):
    import sys
    print(*a, file=sys.stderr, flush=True)


def _gen_config4(n):
    import workloads
    params = workloads.config4_params()
    return [workloads.config4_maze(i, params) for i in range(n)]


def bench_batch(args):
    import torch
    import paper_2004_00540_amd as omap
    import workloads

    n = 512
    t0 = time.perf_counter()
    params = workloads.config4_params()
    with cf.ProcessPoolExecutor(max_workers=8) as ex:
        mazes = list(ex.map(workloads.config4_maze, range(n), [params] * n, chunksize=16))
    _log(f"generated {n} mazes in {time.perf_counter() - t0:.1f} s")
    dev = torch.device("cuda:0")
    occs = [torch.from_numpy(m.occ).to(dev) for m in mazes]
    cells = sum(m.H * m.W for m in mazes)
    n_tgt = sum(len(m.targets) for m in mazes)
    opts = dict(temporal_depth=args.depth, tile_rows=args.tile_rows, schedule=args.schedule,
                lane_columns=args.lane_columns, round_launch=args.launch)
    items = [(occs[i], m.sources, m.targets) for i, m in enumerate(mazes)]
    tuned = None
    if not args.no_tune and not any(opts.values()):
        # the tile shape and layers per visit for this workload, from the autotuner
        t0 = time.perf_counter()
        tuned = omap.tune(items, omap.USE_BATCH)
        tuned["seconds"] = round(time.perf_counter() - t0, 2)
        opts = tuned["options"]
        _log(f"autotuner: {tuned}")

    def batched(o=None):
        with omap.Batch(items, **(opts if o is None else o)) as b:
            b.propagate(sync=False)
            out = b.paths()
        return out

    def plain():
        # the plain loop runs single-maze plans with their own defaults
        res = []
        for i, m in enumerate(mazes):
            with omap.Plan(occs[i], m.sources, m.targets) as p:
                p.propagate(sync=False)
                res.append(p.paths())
        return res

    batched()
    torch.cuda.synchronize()
    reps = max(1, args.steps)
    t0 = time.perf_counter()
    for _ in range(reps):
        batched()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    t_default = None
    if tuned is not None:
        batched({})
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            batched({})
        torch.cuda.synchronize()
        t_default = (time.perf_counter() - t0) / reps
    with omap.Batch(items, **opts) as b:
        infos = b.propagate()
        b.profile(True)
        b.propagate(sync=False)
        prof = b.profile_read()
    t_plain = None
    if not getattr(args, "no_plain_loop", False):
        plain()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plain()
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
    eff = sum(m.H * m.W * (i["layers"] + 1) for m, i in zip(mazes, infos))
    # roofline of the batch's sweep kernel on its own algorithmic bytes: the
    # integer sweep 8.125 B per cell-update; the bit-sliced one 3 bits per
    # cell and layer (reached set in and out, mask) + 4 B per reached cell
    resolved = omap.resolve_options(**opts)
    bits = resolved["schedule"] == omap.SCHEDULE_BITS
    reached = sum(i["reached_cells"] for i in infos)
    alg = prof["cell_updates"] * (0.375 if bits else 8.125) + (4 * reached if bits else 0)
    k_s = prof["ms"] / 1e3
    achieved = alg / k_s / 1e9 if k_s > 0 else 0.0
    return {
        "metric": "mazes/s", "value": round(n / t_batch, 2), "unit": "mazes/s", "n_gpus": 1,
        "steps": reps, "warmup": 1, "ms_per_step": round(t_batch * 1e3, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "config4_512_mazes_loguniform_128_2048", "mazes": n, "cells": cells,
                   "targets": n_tgt, "max_layers_run_time": max(i["layers"] for i in infos)},
        "plain_loop_mazes_per_s": round(n / t_plain, 2) if t_plain else None,
        "speedup_vs_plain_loop": round(t_plain / t_batch, 2) if t_plain else None,
        "effective_gcell_updates_per_s": round(eff / t_batch / 1e9, 1),
        "paths_per_s": round(n_tgt / t_batch, 1),
        "sweep_kernel": {"kernel": f"k_bits<{resolved['temporal_depth']}>" if bits else
                         f"k_sweep<{resolved['temporal_depth']},{resolved['lane_columns']}>",
                         "launches": prof["launches"], "ms_total": round(prof["ms"], 3),
                         "avg_us": round(prof["ms"] * 1e3 / max(prof["launches"], 1), 2),
                         "cell_updates": prof["cell_updates"], "reached_cells": reached},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": 8000.0, "unit": "GB/s",
                     "frac": round(achieved / 8000.0, 4),
                     "algorithmic_bytes": "0.375 B per cell-layer + 4 B per reached cell" if bits
                     else "8.125 B per cell-update"},
        "options": resolved if tuned is None else tuned["options"],
        "options_source": ("command line or built-in defaults" if tuned is None else
                           "autotuner" if any(tuned["options"].values()) else
                           "autotuner: the built-in batch defaults won (zero fields = the defaults)"),
        "autotuner": tuned,
        "default_options_mazes_per_s": round(n / t_default, 2) if t_default else None,
    }


def _gen_query(i):
    import workloads
    return workloads.serve_query(i)


def bench_serve(args):
    """Serving form on the serving workload's recipe: distinct queries
    (query i of the seeded stream), all queued at once to measure the engine's
    capacity, then Poisson arrivals at 0.7 x that capacity, latency =
    completion - arrival over the queries after the warm-up ones.  Baseline:
    the plain per-maze loop (occupancy upload, plan create, propagate, paths
    to host, destroy) over the first queries of the same stream."""
    import torch
    import paper_2004_00540_amd as omap
    import workloads

    n_warm = args.serve_warmup
    n_req = n_warm + args.serve_requests
    t0 = time.perf_counter()
    with cf.ProcessPoolExecutor(max_workers=16) as ex:
        seq = list(ex.map(_gen_query, range(n_req), chunksize=4))
    _log(f"generated {n_req} distinct queries in {time.perf_counter() - t0:.1f} s; "
         f"mean cells {np.mean([q.H * q.W for q in seq]) / 1e6:.1f} M")
    dev = torch.device("cuda:0")
    opts = dict(temporal_depth=args.depth, tile_rows=args.tile_rows, schedule=args.schedule,
                lane_columns=args.lane_columns, round_launch=args.launch)
    tuned = None
    if not args.no_tune and not any(opts.values()):
        # options for this query mix from the autotuner, on a sample of the stream
        sample = seq[:48]
        occ_s = [torch.from_numpy(q.occ).to(dev) for q in sample]
        t0 = time.perf_counter()
        tuned = omap.tune([(o, q.sources, q.targets) for o, q in zip(occ_s, sample)], omap.USE_ENGINE)
        tuned["seconds"] = round(time.perf_counter() - t0, 2)
        opts = tuned["options"]
        _log(f"autotuner: {tuned}")
        del occ_s
        torch.cuda.empty_cache()
    free, _ = torch.cuda.mem_get_info()
    budget = int(min(args.serve_budget_gb * (1 << 30), 0.8 * free))

    def plain_one(q):
        # the plain loop runs single-maze plans with their own defaults
        occ = torch.from_numpy(q.occ).to(dev)
        with omap.Plan(occ, q.sources, q.targets) as p:
            p.propagate(sync=False)
            ln, off, cells = p.paths()
            cells.cpu()
    plain_one(seq[0])
    torch.cuda.synchronize()
    n_plain = min(n_req, args.serve_plain)
    t0 = time.perf_counter()
    for q in seq[:n_plain]:
        plain_one(q)
    torch.cuda.synchronize()
    plain_rate = n_plain / (time.perf_counter() - t0)
    _log(f"plain loop {plain_rate:.2f} mazes/s over {n_plain} queries")

    def run(arrivals, rounds, window=None):
        # window: most queries submitted and not finished at once (None: the
        # arrivals alone decide)
        eng = omap.Engine(budget, max_slots=args.serve_slots, **opts)
        done = {}
        ids = {}
        k = 0
        steps = 0
        start = time.perf_counter()
        while len(done) < len(arrivals):
            now = time.perf_counter() - start
            while k < len(arrivals) and arrivals[k] <= now and (window is None or k - len(done) < window):
                q = seq[k]
                ids[eng.submit(q.occ, q.sources, q.targets)] = k
                k += 1
            res, _ = eng.step(rounds=rounds)
            steps += 1
            now = time.perf_counter() - start
            for qid in eng.completed():
                eng.fetch(qid)
                j = ids.pop(qid)
                done[j] = now - arrivals[j]
            if res == 0 and not ids and k < len(arrivals):
                time.sleep(max(0.0, arrivals[k] - (time.perf_counter() - start)))
        total = time.perf_counter() - start
        eng.close()
        lat = np.array([done[j] for j in range(len(arrivals))])
        return total, lat, steps

    # closed loop: every query available at t = 0, kept queued two slots'
    # worth deep -> capacity
    t_closed, _, steps_closed = run(np.zeros(n_req), args.serve_rounds, window=2 * args.serve_slots)
    capacity = n_req / t_closed
    _log(f"engine capacity {capacity:.2f} mazes/s ({steps_closed} steps)")
    rate = 0.7 * capacity
    arrivals = workloads.serve_arrivals(n_req, rate)
    t_open, lat, steps_open = run(arrivals, args.serve_rounds)
    lat = lat[n_warm:]
    return {
        "metric": "mazes/s", "value": round(capacity, 2), "unit": "mazes/s", "n_gpus": 1,
        "steps": n_req, "warmup": n_warm, "ms_per_step": round(1e3 / capacity, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"serve_poisson_{args.serve_requests}_after_{n_warm}_distinct_queries_side_256_8192",
                   "arrival_rate_per_s": round(rate, 2), "budget_gb": round(budget / (1 << 30), 1),
                   "slots": args.serve_slots, "rounds_per_step": args.serve_rounds},
        "capacity_mazes_per_s": round(capacity, 2),
        "open_loop_mazes_per_s": round(n_req / t_open, 2),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)) * 1e3, 2),
                       "p99": round(float(np.percentile(lat, 99)) * 1e3, 2),
                       "mean": round(float(lat.mean()) * 1e3, 2)},
        "plain_loop_mazes_per_s": round(plain_rate, 2),
        "capacity_vs_plain_loop": round(capacity / plain_rate, 2),
        "options": opts,
        "options_source": ("command line or built-in defaults" if tuned is None else
                           "autotuner" if any(tuned["options"].values()) else
                           "autotuner: the built-in engine defaults won (zero fields = the defaults)"),
        "autotuner": tuned,
    }


# The paper's own run-time workloads (empty maps, fixed L), with the times the
# paper reports on its hardware (context only, other GPUs):
#   Table gpu_comp: 2000x2000, 2000 layers, one pass: 2.370 s (GTX 1080 Ti), 0.871 s (Titan V)
#   Sec. "Run-time": t_r(n, L) ~ 3.0751e-10 * L * n^2 s (GTX 1080 Ti), n in 500..4000
#   Sec. "Limitations": n = 26,000, L = 3,450: 692.3 s; 5,000 sources, L = 650: 147.4 s
PAPER_CASES = [
    # (name, n, L, n_sources, paper_seconds, paper_hw)
    ("gpu_comp_2000_L2000", 2000, 2000, 1, 2.370, "GTX 1080 Ti"),
    ("time_pro_1000_L1000", 1000, 1000, 1, 3.0751e-10 * 1000 * 1000 ** 2, "GTX 1080 Ti (fit)"),
    ("time_pro_2000_L4000", 2000, 4000, 1, 3.0751e-10 * 4000 * 2000 ** 2, "GTX 1080 Ti (fit)"),
    ("time_pro_4000_L8000", 4000, 8000, 1, 3.0751e-10 * 8000 * 4000 ** 2, "GTX 1080 Ti (fit)"),
    ("big_26000_L3450", 26000, 3450, 1, 692.3, "GTX 1080 Ti"),
    ("big_26000_5000src_L650", 26000, 650, 5000, 147.4, "GTX 1080 Ti"),
]


def bench_paper(args):
    """Empty n x n maps run for exactly L layers (the paper's output A_L), one
    source in the corner (the paper's worst case) or k seeded random sources;
    timed with the dense, the active and the bit-sliced schedule."""
    import torch
    import paper_2004_00540_amd as omap
    import workloads

    dev = torch.device("cuda:0")
    rows = []
    for name, n, L, k, paper_s, hw in PAPER_CASES:
        occ = torch.zeros((n, n), dtype=torch.uint8, device=dev)
        if k == 1:
            src = np.array([[0, 0]], np.int32)
        else:
            rc = workloads.below(5, 11, n * n, k)
            src = np.unique(np.stack([rc // n, rc % n], 1).astype(np.int32), axis=0)
        row = {"case": name, "n": n, "layers": L, "sources": int(len(src)),
               "paper_s": round(paper_s, 4), "paper_hw": hw}
        for sched, label in ((omap.SCHEDULE_DENSE, "dense"), (omap.SCHEDULE_ACTIVE, "active"),
                             (omap.SCHEDULE_BITS, "bits")):
            with omap.Plan(occ, src, None, schedule=sched, temporal_depth=args.depth,
                           tile_rows=args.tile_rows) as plan:
                plan.propagate(L)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                plan.propagate(L, sync=False)
                torch.cuda.synchronize()
                t = time.perf_counter() - t0
            row[f"{label}_s"] = round(t, 5)
            row[f"{label}_gcell_updates_per_s"] = round(n * n * L / t / 1e9, 1)
            row[f"{label}_speedup_vs_paper"] = round(paper_s / t, 1)
        _log(row)
        rows.append(row)
        del occ
        torch.cuda.empty_cache()
    best = rows[0]
    return {
        "metric": "Gcell-updates/s", "value": best["active_gcell_updates_per_s"], "unit": "Gcell-updates/s",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": round(best["active_s"] * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic", "config": {"workload": "paper_empty_maps_fixed_L"}, "cases": rows,
    }
