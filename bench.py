"""Benchmark of the oMAP hot path on one MI355X.

One step = the whole path for one maze: ingest (pack the occupancy, store
sources / targets), propagate with the run-time determined layer count, and
extract the path of every target.  Inputs are resident in HBM before timing.

Default workload: the 23170 x 23170 maze (Bernoulli(0.40) + 50,000 filled
rectangles, 16 sources, 4096 targets on the largest component; seeded,
synthetic).  Metric: Gcell-updates/s = cell-updates the sweep kernels execute
per step (interior cells of the visited tiles x layers per visit) / step time.
The dense equivalent of the paper's layer-by-layer network, cells x S_J / step
time with S_J = L* + 1 effective layers, is reported beside it under its own
key (the active schedule reaches the same bits while executing a small part of
that dense work).  The same line carries the batched form (512 mazes) and the
serving form (Poisson arrivals, p50 / p99 latency) and the CPU oracle on the
same inputs.

Prints one JSON line.  --workload batch | serve | paper run one form alone
(see bench_forms.py); --no-forms leaves the batched and serving forms out of
the default line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0                  # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_sweep_c3_traffic.json")
KERNEL_SOURCES = ("omap_sweep.h", "omap_sweep_split.h", "omap_sweep_variant.hip", "omap_internal.h")
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz, 32-bit ops
BYTES_PER_CELL_UPDATE = 8.125          # int32 read + int32 write + 1 mask bit
LDS_FILE = os.path.join(ROOT, "profiles", "lds_c3_23170.json")
LDS_SOURCES = KERNEL_SOURCES + ("omap_kernels.hip",)
# LDS: 256 CUs x 128 B per clock (32 banks of 4 B) x 2.4 GHz
LDS_PEAK_GBS = 256 * 128 * 2.4
# kernels whose LDS use is summarized: (part of the name in the counter files, label)
LDS_KERNELS = (("omap::k_sweep_split<", "k_sweep_split<16>"), ("omap::k_walk(", "k_walk"))
LDS_COUNTERS = ("SQ_INSTS_LDS", "SQ_LDS_IDX_ACTIVE", "SQ_LDS_BANK_CONFLICT", "SQ_WAVES")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    return model, cores


def cpu_baseline(m, gpu_step_s: float, gpu_cell_updates: int, effective_layers: int, budget_s: float = 25.0):
    """The CPU oracle on the same maze, two ways.

    Work-matched (the reported value): the oracle computes the same outputs as
    one GPU step -- the activity map (multi-source BFS and the closed form
    max(0, L+1-d), which the oracle's pins tie to the paper's layers) and the
    simple path of all targets -- over the whole maze, on one core (the oracle
    is single-threaded there).  Its rate is expressed in the metric's unit as
    the GPU step's executed cell-updates divided by the oracle's time.

    The literal network: the oracle's layers on the whole grid for a bounded
    number of layers on all host cores and on one core, extrapolated to the
    S_J layers the plain layer-by-layer method needs."""
    import oracle
    model, cores = cpu_info()
    threads = max(1, min(cores, 16))
    t0 = time.perf_counter()
    d, ecc = oracle.bfs(m.occ, m.sources)
    t_bfs = time.perf_counter() - t0
    t0 = time.perf_counter()
    A = oracle.activity_from_bfs(d, ecc)
    t_map = time.perf_counter() - t0
    del d
    t0 = time.perf_counter()
    oracle.walk(A, m.sources, m.targets)
    t_walk = time.perf_counter() - t0
    del A
    t_full = t_bfs + t_map + t_walk
    log(f"cpu oracle: bfs {t_bfs:.2f} s, map {t_map:.2f} s, walk {t_walk:.2f} s")
    # literal layers on the whole grid, bounded (a one-layer run sizes each)
    lit = {}
    for n_thr, share in ((threads, 0.7), (1, 0.3)):
        t0 = time.perf_counter()
        oracle.layers(m.occ, m.sources, 1, threads=n_thr)
        t1 = time.perf_counter() - t0
        K = int(max(1, min(64, share * budget_s / max(t1, 1e-3))))
        t0 = time.perf_counter()
        oracle.layers(m.occ, m.sources, K, threads=n_thr)
        tk = time.perf_counter() - t0
        rate = m.H * m.W * K / tk
        lit[n_thr] = (K, tk, rate)
        log(f"cpu literal layers: {K} layers on {n_thr} thread(s) in {tk:.1f} s -> {rate / 1e9:.3f} G/s")
    K, tk, rate = lit[threads]
    K1, tk1, rate1 = lit[1]
    dense = m.H * m.W * effective_layers
    return {
        "value": round(gpu_cell_updates / t_full / 1e9, 4), "unit": "Gcell-updates/s", "cores": 1,
        "kind": "oracle",
        "sample": f"whole maze: oracle multi-source BFS ({t_bfs:.2f} s) + closed-form activity map ({t_map:.2f} s) "
                  f"+ simple walk of all {len(m.targets)} targets ({t_walk:.2f} s) = {t_full:.2f} s on one core for "
                  f"the outputs of one GPU step; value = the GPU step's {gpu_cell_updates} executed cell-updates / "
                  f"that time",
        "oracle_step_s": round(t_full, 3),
        "gpu_step_speedup": round(t_full / gpu_step_s, 1),
        "cpu_model": model, "host_cores": cores,
        "literal_layers": {
            "gcell_updates_per_s_all_cores": round(rate / 1e9, 4), "threads": threads, "layers_timed": K,
            "seconds": round(tk, 2),
            "gcell_updates_per_s_one_core": round(rate1 / 1e9, 4), "layers_timed_one_core": K1,
            "seconds_one_core": round(tk1, 2),
            "extrapolated_full_run_s_all_cores": round(dense / rate, 1),
            "note": f"the paper's literal layers on the whole {m.H}x{m.W} grid, timed for the layers shown and "
                    f"extrapolated to S_J = {effective_layers} layers (dense, no early exit)",
        },
    }


def kernel_source_hash(files=KERNEL_SOURCES) -> str:
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2004_00540_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, options: dict):
    """HBM bytes per sweep launch from the committed hardware-counter summary
    (FETCH_SIZE + WRITE_SIZE, calibrated against a plain copy), or None when
    the counters were taken on other kernel sources or another configuration."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash() or t.get("workload") != workload \
            or t.get("options") != options:
        return None
    return t.get("bytes_per_launch")


def _csv_rows(directory: str, suffix: str):
    import csv
    import glob
    rows = []
    for path in sorted(glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True)):
        with open(path, newline="") as f:
            rows += list(csv.DictReader(f))
    return rows


def _counter_per_dispatch(directory: str, counter: str, kernel_part: str):
    """Mean value of a rocprofv3 --pmc counter over the dispatches of the
    kernels whose name contains kernel_part (counter_collection.csv)."""
    vals = {}
    for r in _csv_rows(directory, "counter_collection.csv"):
        name = r.get("Kernel_Name", "")
        if kernel_part not in name or r.get("Counter_Name") != counter:
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    if not vals:
        raise SystemExit(f"no {counter} rows for {kernel_part} under {directory}")
    return sum(vals.values()) / len(vals), len(vals)


def summarize_counters(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, out_path, commands):
    """profiles/k_sweep_c3_traffic.json from four rocprofv3 --pmc runs: the
    sweep's FETCH_SIZE and WRITE_SIZE (KiB per dispatch), each scaled by what
    the counter reads for a plain pass of known size (bench.py --workload
    copy: 1 GiB read + 1 GiB written per launch)."""
    import paper_2004_00540_amd as omap
    kern = "omap::k_sweep_split<"
    f_kib, n = _counter_per_dispatch(fetch_dir, "FETCH_SIZE", kern)
    w_kib, _ = _counter_per_dispatch(write_dir, "WRITE_SIZE", kern)
    cf_kib, _ = _counter_per_dispatch(copy_fetch_dir, "FETCH_SIZE", "neg_kernel")
    cw_kib, _ = _counter_per_dispatch(copy_write_dir, "WRITE_SIZE", "neg_kernel")
    gib_kib = float(1 << 20)
    f_scale, w_scale = gib_kib / cf_kib, gib_kib / cw_kib
    fetch = f_kib * 1024 * f_scale
    write = w_kib * 1024 * w_scale
    out = {
        "kernel": "omap::k_sweep_split<16> (two waves per tile visit, per-round launch)",
        "workload": "config3_23170x23170_rect_overlay",
        "options": omap.resolve_options(),
        "kernel_source_sha256": kernel_source_hash(),
        "kernel_sources": list(KERNEL_SOURCES),
        "dispatches_counted": n,
        "calibration": {"kernel": "torch neg over 1 GiB int32 (1 GiB read + 1 GiB written per launch)",
                        "fetch_size_kib_raw": round(cf_kib, 1), "write_size_kib_raw": round(cw_kib, 1),
                        "fetch_scale": round(f_scale, 4), "write_scale": round(w_scale, 4)},
        "fetch_kib_raw_per_launch": round(f_kib, 1), "write_kib_raw_per_launch": round(w_kib, 1),
        "fetch_bytes_per_launch": round(fetch), "write_bytes_per_launch": round(write),
        "bytes_per_launch": round(fetch + write),
        "commands": commands,
    }
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def _kernel_avg_us(trace_dir: str, kernel_part: str) -> float:
    """Average duration of the kernels whose name contains kernel_part in a
    rocprofv3 --kernel-trace --stats run (kernel_stats.csv)."""
    calls, total_ns = 0, 0.0
    for r in _csv_rows(trace_dir, "kernel_stats.csv"):
        if kernel_part in r["Name"]:
            calls += int(r["Calls"])
            total_ns += float(r["TotalDurationNs"])
    if calls == 0:
        raise SystemExit(f"no {kernel_part} in the kernel trace under {trace_dir}")
    return total_ns / calls / 1e3


def summarize_lds(pmc_dir: str, trace_dir: str, out_path: str, commands):
    """profiles/lds_c3_23170.json from one rocprofv3 --pmc run with the LDS
    counters (SQ_INSTS_LDS, SQ_LDS_IDX_ACTIVE, SQ_LDS_BANK_CONFLICT, SQ_WAVES)
    and the kernel trace of the same command.  LDS bytes are counted as 256 per
    LDS instruction (64 lanes x 4 B: the ring rows, windows and counters are
    32-bit accesses; the two-wave visit's input sums, 64-bit, are one
    instruction per visit), an estimate of the data the instructions move."""
    import paper_2004_00540_amd as omap
    kernels = {}
    for part, label in LDS_KERNELS:
        vals = {}
        for c in LDS_COUNTERS:
            vals[c], n = _counter_per_dispatch(pmc_dir, c, part)
        us = _kernel_avg_us(trace_dir, part)
        lds_bytes = vals["SQ_INSTS_LDS"] * 256
        active, conflict = vals["SQ_LDS_IDX_ACTIVE"], vals["SQ_LDS_BANK_CONFLICT"]
        kernels[label] = {
            "dispatches_counted": n, "avg_us": round(us, 2),
            "lds_instructions_per_launch": round(vals["SQ_INSTS_LDS"]),
            "waves_per_launch": round(vals["SQ_WAVES"]),
            "lds_bytes_per_launch_est": round(lds_bytes),
            "lds_gbs": round(lds_bytes / (us * 1e-6) / 1e9, 1),
            "lds_peak_gbs": round(LDS_PEAK_GBS, 1),
            "lds_frac": round(lds_bytes / (us * 1e-6) / 1e9 / LDS_PEAK_GBS, 5),
            "lds_active_cycles_per_launch": round(active),
            "bank_conflict_cycles_per_launch": round(conflict),
            "bank_conflicts_per_access": round(conflict / (active - conflict), 4) if active > conflict else None,
        }
    out = {"workload": "config3_23170x23170_rect_overlay", "options": omap.resolve_options(),
           "kernel_source_sha256": kernel_source_hash(LDS_SOURCES), "kernel_sources": list(LDS_SOURCES),
           "kernels": kernels, "commands": commands}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    lines = ["| kernel | avg us | LDS instr. per launch | waves | est. LDS GB/s | of peak | LDS active cycles | "
             "bank-conflict cycles | conflicts per access |", "|---|---|---|---|---|---|---|---|---|"]
    for label, k in kernels.items():
        lines.append(f"| `{label}` | {k['avg_us']} | {k['lds_instructions_per_launch']} | {k['waves_per_launch']} | "
                     f"{k['lds_gbs']} | {k['lds_frac'] * 100:.2f} % | {k['lds_active_cycles_per_launch']} | "
                     f"{k['bank_conflict_cycles_per_launch']} | {k['bank_conflicts_per_access']} |")
    print("\n".join(lines))


def measured_lds(workload: str, options: dict):
    """The committed LDS counter summary of the sweep and walk kernels, or None
    when it was taken on other kernel sources or another configuration."""
    try:
        with open(LDS_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256") != kernel_source_hash(LDS_SOURCES) or t.get("workload") != workload \
            or t.get("options") != options:
        return None
    return t.get("kernels")


def stream_copy_gbs(dev, reps: int = 5) -> dict:
    """Device-to-device copy of 1 GiB (1 GiB read + 1 GiB written per copy),
    timed with events: the HBM rate a plain streaming kernel reaches."""
    import torch
    n = 1 << 28
    src = torch.ones(n, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        dst.copy_(src)
    ev[1].record()
    torch.cuda.synchronize()
    s = ev[0].elapsed_time(ev[1]) / 1e3 / reps
    del src, dst
    torch.cuda.empty_cache()
    gbs = 2 * 4 * n / s / 1e9
    return {"gbs": round(gbs, 1), "frac_of_peak": round(gbs / HBM_PEAK_GBS, 4),
            "kernel": "torch copy_ of 1 GiB int32, device to device (1 GiB read + 1 GiB written), "
                      f"mean of {reps}"}


def summarize_trace(directory: str, top: int = 14):
    """Markdown table of a rocprofv3 --kernel-trace --stats run (kernel_stats.csv)."""
    rows = _csv_rows(directory, "kernel_stats.csv")
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["| kernel | calls | total ms | avg us | min us | max us | % |", "|---|---|---|---|---|---|---|"]
    for r in rows[:top]:
        name = r["Name"] if len(r["Name"]) <= 70 else r["Name"][:67] + "..."
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                     f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    print("\n".join(lines))


def copy_probe(args):
    """A plain elementwise pass over 1 GiB (torch's negation kernel: 1 GiB read,
    1 GiB written per launch), run under the same hardware counters as the
    sweep to calibrate the HBM byte counters."""
    import torch
    n = 1 << 28
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(max(1, args.steps)):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    return {"metric": "copy_bytes", "value": 2 * 4 * n, "unit": "B", "read_bytes": 4 * n,
            "write_bytes": 4 * n, "launches": max(1, args.steps)}


def bench_plain(args):
    import torch
    import paper_2004_00540_amd as omap
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    t0 = time.perf_counter()
    if args.workload == "c3":
        m = workloads.config3()
    elif args.workload == "c2":
        m = workloads.config2()
    else:
        m = workloads.config1()
    log(f"generated {m.name} in {time.perf_counter() - t0:.1f} s")
    occ = torch.from_numpy(m.occ).to(dev)
    N = m.H * m.W
    opts = dict(temporal_depth=args.depth, tile_rows=args.tile_rows, schedule=args.schedule,
                lane_columns=args.lane_columns, round_launch=args.launch)
    stream = torch.cuda.current_stream()
    plan = omap.Plan(occ, m.sources, m.targets, **opts)
    nt = len(m.targets)
    lengths = torch.empty(nt, dtype=torch.int32, device=dev)
    offsets = torch.empty(nt + 1, dtype=torch.int64, device=dev)
    info = plan.propagate(omap.AUTO)
    _, _, cells0 = plan.paths()
    cells = torch.empty(max(cells0.numel(), 1), dtype=torch.int32, device=dev)
    L_star = info["layers"]
    S_J = L_star + 1
    log(f"info {info}")

    def step():
        plan.load(occ, m.sources, m.targets)
        plan.propagate(omap.AUTO, sync=False)
        plan.extract_into(lengths, offsets, cells)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev[0].record(stream)
    for _ in range(args.steps):
        step()
    ev[1].record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    ms = ev[0].elapsed_time(ev[1]) / args.steps

    # phase split of one step (events on the plan's stream)
    ph = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ph[0].record(stream)
    plan.load(occ, m.sources, m.targets)
    ph[1].record(stream)
    plan.propagate(omap.AUTO, sync=False)
    ph[2].record(stream)
    plan.extract_into(lengths, offsets, cells)
    ph[3].record(stream)
    torch.cuda.synchronize()
    t_load, t_prop, t_ext = (ph[i].elapsed_time(ph[i + 1]) for i in range(3))

    # sweep-kernel timing with HIP events around every launch
    plan.profile(True)
    plan.propagate(omap.AUTO, sync=False)
    prof = plan.profile_read()
    plan.profile(False)
    plan.close()

    step_s = wall
    path_steps = int(lengths.clamp(min=0).sum().item())
    resolved = omap.resolve_options(**opts)
    executed = prof["cell_updates"]            # per propagation = per step
    gcups = executed / step_s / 1e9
    alg_bytes = prof["cell_updates"] * BYTES_PER_CELL_UPDATE
    kern_s = prof["ms"] / 1e3
    launches = max(prof["launches"], 1)
    achieved = alg_bytes / kern_s / 1e9 if kern_s > 0 else 0.0
    ops_per_cell = 4.5
    alu_tops = prof["cell_updates"] * ops_per_cell / kern_s / 1e12 if kern_s > 0 else 0.0
    traffic = measured_traffic(m.name, resolved)
    out = {
        "metric": "Gcell-updates/s", "value": round(gcups, 3), "unit": "Gcell-updates/s",
        "value_definition": "cell-updates executed by the sweep kernels per step / step time",
        "dense_equivalent_gcell_updates_per_s": round(N * S_J / step_s / 1e9, 1),
        "dense_equivalent_definition": "cells x S_J / step time, S_J = L* + 1: the paper's layer-by-layer "
                                       "network reaches the same map with this many cell-updates",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(step_s * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": m.name, "cells": N, "sources": len(m.sources), "targets": nt,
                   "layers_run_time": L_star, "effective_layers": S_J,
                   "options": resolved},
        "paths_per_s": round(nt / step_s, 1),
        "paths_per_s_extract_only": round(nt / (t_ext / 1e3), 1) if t_ext > 0 else None,
        "path_steps_per_s_extract_only": round(path_steps / (t_ext / 1e3), 1) if t_ext > 0 else None,
        "path_cells": int(cells0.numel()),
        "phase_ms": {"ingest": round(t_load, 3), "propagate": round(t_prop, 3), "extract": round(t_ext, 3)},
        "event_ms_per_step": round(ms, 3),
        "sweep_kernel": {"launches": prof["launches"], "ms_total": round(prof["ms"], 3),
                         "avg_us": round(prof["ms"] * 1e3 / max(prof["launches"], 1), 2),
                         "cell_updates": prof["cell_updates"],
                         "dense_cell_updates": N * S_J},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "algorithmic_bytes_per_launch": round(alg_bytes / launches),
                     "avg_launch_us": round(prof["ms"] * 1e3 / launches, 2),
                     "measured_hbm_gbs": round(traffic / (kern_s / launches) / 1e9, 1) if traffic and kern_s > 0
                     else None},
        "roofline_alu": {"bound": "alu", "achieved": round(alu_tops, 2), "peak": round(VALU_PEAK_TOPS, 1),
                         "unit": "Tops/s", "frac": round(alu_tops / VALU_PEAK_TOPS, 4),
                         "ops_per_cell_update": ops_per_cell},
    }
    out["stream_copy"] = stream_copy_gbs(dev)
    out["lds"] = measured_lds(m.name, resolved)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(m, step_s, executed, S_J, args.cpu_budget)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=["c1", "c2", "c3", "batch", "serve", "copy", "paper"])
    ap.add_argument("--depth", type=int, default=0)
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--schedule", type=int, default=0)
    ap.add_argument("--lane-columns", type=int, default=0)
    ap.add_argument("--launch", type=int, default=0, help="0 one launch per round, 1 rounds replayed from HIP graphs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=25.0)
    ap.add_argument("--no-forms", action="store_true", help="leave the batched and serving forms out")
    ap.add_argument("--no-tune", action="store_true", help="batched and serving forms without the autotuner")
    ap.add_argument("--no-plain-loop", action="store_true", help="batched form without its plain-loop baseline")
    ap.add_argument("--serve-warmup", type=int, default=20)
    ap.add_argument("--serve-requests", type=int, default=500)
    ap.add_argument("--serve-plain", type=int, default=100, help="queries timed in the plain per-maze loop")
    ap.add_argument("--serve-budget-gb", type=float, default=64.0)
    ap.add_argument("--serve-slots", type=int, default=64)
    ap.add_argument("--serve-rounds", type=int, default=4)
    ap.add_argument("--summarize-counters", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR",
                                                              "COPY_WRITE_DIR"),
                    help="write profiles/k_sweep_c3_traffic.json from four rocprofv3 --pmc runs (no GPU)")
    ap.add_argument("--summarize-trace", metavar="DIR", help="markdown table of a rocprofv3 --stats run (no GPU)")
    ap.add_argument("--summarize-lds", nargs=2, metavar=("PMC_DIR", "TRACE_DIR"),
                    help="write profiles/lds_c3_23170.json from a rocprofv3 --pmc run of the LDS counters and "
                         "the kernel trace of the same command (no GPU)")
    ap.add_argument("--commands", nargs="*", default=[], help="commands recorded with --summarize-counters")
    args = ap.parse_args()
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, TRAFFIC_FILE, args.commands)
        return
    if args.summarize_lds:
        summarize_lds(*args.summarize_lds, LDS_FILE, args.commands)
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the path runs on a single MI355X "
              "(multi-GPU sharding is a design note, not part of this build)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "copy":
        out = copy_probe(args)
    elif args.workload in ("c1", "c2", "c3"):
        out = bench_plain(args)
        if args.workload == "c3" and not args.no_forms:
            import torch
            from bench_forms import bench_batch, bench_serve
            torch.cuda.empty_cache()
            b = bench_batch(args)
            out["batch"] = {k: b[k] for k in ("value", "unit", "ms_per_step", "plain_loop_mazes_per_s",
                                              "speedup_vs_plain_loop", "paths_per_s", "config", "options",
                                              "options_source", "default_options_mazes_per_s")}
            torch.cuda.empty_cache()
            sv = bench_serve(args)
            out["serve"] = {k: sv[k] for k in ("capacity_mazes_per_s", "open_loop_mazes_per_s", "latency_ms",
                                               "plain_loop_mazes_per_s", "capacity_vs_plain_loop", "config",
                                               "options", "options_source")}
    elif args.workload == "batch":
        from bench_forms import bench_batch
        out = bench_batch(args)
    elif args.workload == "paper":
        from bench_forms import bench_paper
        out = bench_paper(args)
    else:
        from bench_forms import bench_serve
        out = bench_serve(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
