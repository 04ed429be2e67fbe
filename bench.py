"""Benchmark: GP operations per second (tree nodes x fitness cases / s) on one MI355X.

Default workload: 4000 uniformly random trees with node counts log-uniform in
[10, 1e5] (about 4.3e7 nodes), 48 fitness cases in [-1, 1].  One step is one
generation of the method's hot path on that population: size-2 tournament
selection and Philox-drawn crossover points, subtree crossover, the structure
scan and split of the children, their evaluation on every case and their
fitness.  Every step starts from the same resident parents, so the work per
step is stationary.  value = sum over steps of child nodes x cases / timed
wall time.

Also reported: evaluation alone on the resident parents (device time and
p50/p99 latency per call), the dominant kernel (level-0 interpreter) against
the FP32 VALU roofline, and the C oracle timed on the host cores.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batched|tiny|giant]
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

PEAK_GPOPS = 256 * 64 * 2 * 2.4e9  # one FP32 op per lane, two per packed issue, 2.4 GHz
PEAK_UNPACKED = 256 * 64 * 2.4e9


def pct(a, q):
    return float(np.percentile(np.asarray(a, np.float64), q)) if len(a) else None


def cpu_baseline(buf, off, x, y, fit, n_cases, budget_s=12.0):
    """The oracle as it stands, on the host cores: generations of the same
    population (sequential selection + crossover, threaded evaluation)."""
    import oracle

    threads = min(os.cpu_count() or 1, 64)
    done_nodes, t0, gens = 0, time.perf_counter(), 0
    while True:
        cbuf, coff, _ = oracle.generation(buf, off, fit, 2, 1234, 10_000 + gens, 15_000_000)
        oracle.eval_population(cbuf, coff, x, y, threads=threads)
        done_nodes += int(coff[-1])
        gens += 1
        el = time.perf_counter() - t0
        if el >= budget_s or gens >= 50:
            break
    return {"value": done_nodes * n_cases / el, "unit": "GPops/s", "cores": threads, "kind": "oracle",
            "sample": f"{gens} oracle generations of the {off.size - 1}-tree population "
                      f"(selection+crossover single-threaded, evaluation on {threads} threads), {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched")
    ap.add_argument("--eval-reps", type=int, default=50)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--lds", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the evaluation path of this build is single-GPU "
              "(multi-GPU sharding is described in DESIGN.md, not built)", file=sys.stderr)
        sys.exit(2)

    import paper_1902_09215_amd as ev
    import workloads

    buf, off, n_cases = workloads.workload(args.workload)
    x, y = workloads.cases(n_cases)
    M = off.size - 1
    c = ev.Context(x, y, device=0)
    if args.chunk or args.lds:
        ev.ev_set_tuning(c.ctx, args.chunk, args.lds)
    t_load = time.perf_counter()
    parents = c.load(buf, off)
    t_load = time.perf_counter() - t_load
    plan = ev.ev_get_plan_info(c.ctx, parents)
    fit, _ = c.eval(parents)

    # ---- evaluation alone on the resident parents
    dev_ms, int_ms, lat = [], [], []
    for r in range(args.warmup + args.eval_reps):
        t0 = time.perf_counter()
        ev.ev_eval_fitness(c.ctx, parents)
        t1 = time.perf_counter()
        a, b = ev.ev_last_timing(c.ctx)
        if r >= args.warmup:
            lat.append((t1 - t0) * 1e3)
            dev_ms.append(a)
            int_ms.append(b)
    nodes = int(off[-1])
    eval_gpops = nodes * n_cases / (np.median(dev_ms) * 1e-3)
    interp_ms = float(np.mean(int_ms))
    interp_gpops = nodes * n_cases / (interp_ms * 1e-3)

    # ---- generation steps (the whole hot path)
    seed = 0x5EED
    for w in range(args.warmup):
        kids, _ = ev.ev_generation(c.ctx, parents, seed, 1_000_000 + w, 2, 15_000_000)
        ev.ev_eval_fitness(c.ctx, kids)
        ev.ev_free_pop(c.ctx, kids)
    step_ms, child_nodes = [], 0
    t_all = time.perf_counter()
    for s in range(args.steps):
        t0 = time.perf_counter()
        kids, _ = ev.ev_generation(c.ctx, parents, seed, s, 2, 15_000_000)
        ev.ev_eval_fitness(c.ctx, kids)
        t1 = time.perf_counter()
        child_nodes += ev.ev_pop_info(c.ctx, kids)[1]
        ev.ev_free_pop(c.ctx, kids)
        step_ms.append((t1 - t0) * 1e3)
    total_s = time.perf_counter() - t_all
    value = child_nodes * n_cases / sum(step_ms) * 1e3

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(buf, off, x, y, fit, n_cases)

    line = {
        "metric": "GPops/s (tree nodes x fitness cases /s) on 1 MI355X; p99 eval latency",
        "value": value,
        "unit": "GPops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": float(np.mean(step_ms)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": {"batched": "batched uneven population: 4000 random trees, log-uniform 10..1e5 nodes",
                         "tiny": "100 ramped half-and-half trees, depth 2-6",
                         "giant": "48 random trees, log-uniform 1e6..4e8 nodes",
                         "giant_max": "48 random trees of 4e8 nodes"}.get(args.workload, args.workload),
            "trees": M, "nodes": nodes, "fitness_cases": n_cases,
            "step": "generation: tournament(2) + Philox points + subtree crossover + scan/split + eval + fitness",
            "chunk": plan and ev.ev_get_plan_info(c.ctx, parents)["levels"] and None,
        },
        "p50_step_ms": pct(step_ms, 50),
        "p99_step_ms": pct(step_ms, 99),
        "eval": {
            "gpops_per_s": eval_gpops,
            "device_ms_median": float(np.median(dev_ms)),
            "p50_latency_ms": pct(lat, 50),
            "p99_latency_ms": pct(lat, 99),
            "plan": plan,
            "load_and_plan_s": t_load,
        },
        "roofline": {
            "kernel": "k_eval (level-0 interpreter launch)",
            "bound": "alu",
            "achieved": interp_gpops / 1e12,
            "peak": PEAK_GPOPS / 1e12,
            "unit": "TGPops/s",
            "frac": interp_gpops / PEAK_GPOPS,
            "frac_unpacked": interp_gpops / PEAK_UNPACKED,
            "avg_launch_ms": interp_ms,
            "traffic": None,
        },
        "cpu_baseline": cpu,
    }
    del line["config"]["chunk"]
    print(json.dumps(line), flush=True)
    c.close()


if __name__ == "__main__":
    main()
