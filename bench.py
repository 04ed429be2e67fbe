"""Benchmark: GP operations per second (tree nodes x fitness cases / s) on one MI355X.

Default workload: the giant population, 48 uniformly random trees of 4e8
nodes each (1.92e10 nodes, 19.2 GB of one-byte opcodes), 48 fitness cases in
[-1, 1].  One step is one generation of the method's hot path on that
population: size-2 tournament selection and Philox-drawn crossover points,
subtree crossover, the structure scan and split of the children, their
evaluation on every case and their fitness.  Every step starts from the same
resident parents, so the work per step is stationary.  value = sum over steps
of child nodes x cases / timed wall time.

Also reported: evaluation alone on the resident parents (device time and
p50/p99 latency per call), the plain form (one tree per launch, timed the
same way), the dominant kernel (the level-0 interpreter launch) against the
FP32 vector ALU peak, and the C oracle timed on the host cores.

  python bench.py [--gpus 1] [--steps K] [--warmup W]
                  [--workload giant_max|giant|batched|tiny|loop|serving]

The loop workload is the generational loop (population 48 from ramped
half-and-half trees of depth 2-6, size-2 tournaments, 15e6-node cap): a step
is one generation of the evolving population, run by ev_evolve from captured
graphs, and the same generations on the host-driven path beside it.
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

# FP32 vector peak of the MI355X: 256 CUs x 64 lanes x 2.4 GHz, an FMA
# counted as two operations and packed FP32 as two lanes per issue
PEAK_FP32 = 157.3e12
# one plain (non-FMA, unpacked) FP32 operation per lane per cycle
PEAK_UNPACKED = 256 * 64 * 2.4e9
WORKLOAD_NAMES = {"batched": "batched uneven population: 4000 random trees, log-uniform 10..1e5 nodes",
                  "tiny": "100 ramped half-and-half trees, depth 2-6",
                  "giant": "48 random trees, log-uniform 1e6..4e8 nodes",
                  "giant_max": "giant population: 48 random trees of 4e8 nodes (19.2 GB of opcodes)"}


def pct(a, q):
    return float(np.percentile(np.asarray(a, np.float64), q)) if len(a) else None


def cpu_baseline(buf, off, x, y, fit, n_cases, budget_s=12.0):
    """The oracle as it stands, on the host cores: generations of the same
    population (sequential selection + crossover, threaded evaluation); for
    populations too large for that, the evaluation of the smallest trees."""
    import oracle

    threads = min(len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count() or 1, 64)
    if int(off[-1]) > 2e8:
        sizes = np.diff(off)
        order = np.argsort(sizes)
        take = [int(t) for t in order[:threads]]
        parts = [buf[off[t]:off[t + 1]] for t in take]
        soff = np.zeros(len(parts) + 1, np.uint64)
        np.cumsum([p.size for p in parts], out=soff[1:])
        t0 = time.perf_counter()
        oracle.eval_population(np.concatenate(parts), soff, x, y, threads=threads)
        el = time.perf_counter() - t0
        return {"value": int(soff[-1]) * n_cases / el, "unit": "GPops/s", "cores": threads, "kind": "oracle",
                "cpu_model": cpu_model(),
                "sample": f"oracle evaluation (no selection or crossover) of the {len(take)} smallest trees "
                          f"({int(soff[-1])} nodes), one tree per thread, {el:.1f} s"}
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
            "cpu_model": cpu_model(),
            "sample": f"{gens} oracle generations of the {off.size - 1}-tree population "
                      f"(selection+crossover single-threaded, evaluation on {threads} threads), {el:.1f} s"}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def serve_bench(args, ev, workloads):
    """Serving: a Poisson stream of evaluation (80%) and crossover (20%)
    requests, one tree per evaluation request with sizes log-uniform in
    [10, 1e8], 48 or 1024 cases, with populations resident in HBM and a 200 GB
    memory budget.  The same stream, at the same arrival times, is run twice
    on the GPU: served (ev_submit: continuous batching, workers on their own
    streams) and plain (one request at a time through the synchronous calls,
    one tree per launch, first come first served)."""
    rng = np.random.default_rng(0x5EED0005)
    x48, y48 = workloads.cases(48)
    x1k, y1k = workloads.cases(1024)
    # a pool of distinct trees that the requests draw from
    pool_sizes = workloads.loguniform_sizes(0x5EED0005, 256, 10, 1e8)
    pbuf, poff = workloads.random_population(0x5EED0005, pool_sizes)
    c = ev.Context(x48, y48, device=0, mem_budget=200 << 30)
    t1k = c.add_cases(x1k, y1k)
    par_sizes = workloads.loguniform_sizes(0x5EED0006, 64, 10, 1e6)
    par_buf, par_off = workloads.random_population(0x5EED0006, par_sizes)
    parents = c.load(par_buf, par_off)
    c.eval(parents)
    reqs = []
    for i in range(args.requests):
        table = 0 if rng.random() < 0.5 else t1k
        if rng.random() < 0.8:
            t = int(rng.integers(0, pool_sizes.size))
            reqs.append(("eval", table, t, int(pool_sizes[t])))
        else:
            k = 4
            mum = rng.integers(0, 64, k).astype(np.int32)
            dad = rng.integers(0, 64, k).astype(np.int32)
            p = np.array([rng.integers(0, par_sizes[m]) for m in mum], np.uint64)
            q = np.array([rng.integers(0, par_sizes[d]) for d in dad], np.uint64)
            nodes = int(sum(par_sizes[m] for m in mum))
            reqs.append(("xo", table, (mum, dad, p, q), nodes))

    def tree(t):
        b = pbuf[poff[t]:poff[t + 1]]
        return b, np.array([0, b.size], np.uint64)

    def submit(r):
        kind, table, arg, _ = r
        if kind == "eval":
            b, o = tree(arg)
            return ev.ev_submit_eval(c.ctx, b, o, table)
        mum, dad, p, q = arg
        return ev.ev_submit_crossover(c.ctx, parents, mum, dad, p, q, table)

    def plain(r):
        """The plain form: one request, synchronously, alone on the device."""
        kind, table, arg, _ = r
        if kind == "eval":
            b, o = tree(arg)
            pop = ev.ev_load_trees(c.ctx, b, o)
        else:
            mum, dad, p, q = arg
            pop, _ = ev.ev_crossover(c.ctx, parents, parents, mum, dad, p, q)
        f, _ = ev.ev_eval_fitness(c.ctx, pop, table)
        ev.ev_free_pop(c.ctx, pop)
        return f

    def n_cases(table):
        return 48 if table == 0 else 1024

    work = sum(r[3] * n_cases(r[1]) for r in reqs)
    # plain service times of a prefix of the stream set the offered load
    for r in reqs[:20]:
        plain(r)
    service = []
    for r in reqs[: min(len(reqs), 200)]:
        t0 = time.perf_counter()
        plain(r)
        service.append(time.perf_counter() - t0)
    mean_service = float(np.mean(service))
    lam = args.load / mean_service
    arrivals = np.cumsum(rng.exponential(1.0 / lam, len(reqs)))
    print(f"# serving: {len(reqs)} requests, plain mean service {mean_service * 1e3:.2f} ms, "
          f"offered {lam:.1f}/s", file=sys.stderr, flush=True)

    # plain FIFO, run on the GPU at the stream's arrival times
    lat_plain = []
    t_start = time.perf_counter()
    for i, r in enumerate(reqs):
        now = time.perf_counter() - t_start
        if arrivals[i] > now:
            time.sleep(arrivals[i] - now)
        plain(r)
        lat_plain.append((time.perf_counter() - t_start - arrivals[i]) * 1e3)
    makespan_plain = time.perf_counter() - t_start
    print(f"# plain FIFO done in {makespan_plain:.1f} s", file=sys.stderr, flush=True)

    # served: open loop, continuous batching inside libev.  A request's
    # latency runs from its arrival: the wait before its submit call, the
    # call, then the library's submit-to-done time.
    tickets = []
    t_start = time.perf_counter()
    for i, r in enumerate(reqs):
        now = time.perf_counter() - t_start
        if arrivals[i] > now:
            time.sleep(arrivals[i] - now)
        tk = submit(r)
        tickets.append((tk, r, time.perf_counter() - t_start - arrivals[i]))
    lat, lat_lib = [], []
    for tk, r, to_submit in tickets:
        ev.ev_wait(c.ctx, tk)
        s_ns, _, d_ns = ev.ev_job_timing(c.ctx, tk)
        lat.append(to_submit * 1e3 + (d_ns - s_ns) / 1e6)
        lat_lib.append((d_ns - s_ns) / 1e6)
        ev.ev_result(c.ctx, tk, 8, n_cases(r[1]))
    makespan = time.perf_counter() - t_start
    line = {
        "metric": "GPops/s (tree nodes x fitness cases /s) on 1 MI355X; p99 eval latency",
        "value": work / makespan,
        "unit": "GPops/s",
        "n_gpus": 1,
        "steps": len(reqs),
        "warmup": 0,
        "ms_per_step": makespan / len(reqs) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "serving: Poisson stream, 80% eval / 20% crossover, trees log-uniform 10..1e8 "
                               "nodes, 48 or 1024 cases, 200 GB memory budget",
                   "requests": len(reqs), "offered_load": args.load,
                   "offered_rate_per_s": lam},
        "p50_latency_ms": pct(lat, 50),
        "p99_latency_ms": pct(lat, 99),
        "latency_from": "arrival",
        "submit_to_done_ms": {"p50": pct(lat_lib, 50), "p99": pct(lat_lib, 99)},
        "plain_fifo": {"p50_latency_ms": pct(lat_plain, 50), "p99_latency_ms": pct(lat_plain, 99),
                       "mean_service_ms": mean_service * 1e3,
                       "gpops_per_s": work / makespan_plain,
                       "how": "run on the GPU: each request alone through ev_load_trees/ev_crossover + "
                              "ev_eval_fitness, in arrival order, at the same arrival times"},
    }
    print(json.dumps(line), flush=True)
    c.close()


def calibrate_copy():
    """A plain copy of known size: its FETCH_SIZE / WRITE_SIZE readings give
    the factor that turns those counters into HBM bytes."""
    import torch

    n = 1 << 30
    src = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    src.fill_(1)
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "launches": 5}), flush=True)


def kernel_hash():
    """Hash of what the level-0 k_run launch runs: the interpreter text it
    expands (generated) and the kernel's own source text."""
    import hashlib
    import importlib.util

    spec = importlib.util.spec_from_file_location(
        "gen_interp", os.path.join(ROOT, "paper_1902_09215_amd/csrc/gen_interp.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    h = hashlib.sha256()
    h.update(gen.generate().encode())
    src = open(os.path.join(ROOT, "paper_1902_09215_amd/csrc/ev_kernels.hip")).read()
    i = src.index("void k_run(RunArgs a)")
    h.update(src[i:src.index("\n}\n", i)].encode())
    return h.hexdigest()[:16]


def measured_traffic(workload, chunk):
    """HBM bytes per level-0 k_run launch from the committed counter summary
    of this workload, or None when the kernel sources or the level-0
    work-item size (which sets the launch's items) differ from the ones the
    counters were taken with."""
    import re

    path = os.path.join(ROOT, "profiles", f"k_run_{workload}_traffic.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    vals = dict(re.findall(r"^- (\w+): ([0-9a-f.e+]+)$", text, re.M))
    if vals.get("kernel_hash") != kernel_hash() or vals.get("chunk") != str(chunk):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def evolve_pair(ev, c, parents, seed, gen0, gens, cap, tournament=2):
    """The same generations from the same parents, replayed from graphs and
    on the host-driven path: (graph report, plain report, bit-exact)."""
    kg, fg, cg, rg = ev.ev_evolve(c.ctx, parents, seed, gen0, gens, tournament, cap)
    kp, fp, cp, rp = ev.ev_evolve(c.ctx, parents, seed, gen0, gens, tournament, cap, flags=ev.EV_EVOLVE_NO_GRAPH)
    same = bool((fg.view(np.uint32) == fp.view(np.uint32)).all() or
                ((fg.view(np.uint32) == fp.view(np.uint32)) | (np.isnan(fg) & np.isnan(fp))).all())
    same &= bool(np.array_equal(cg, cp)) and rg["nodes"] == rp["nodes"]
    ev.ev_free_pop(c.ctx, kg)
    ev.ev_free_pop(c.ctx, kp)
    return rg, rp, same


def graph_summary(rg, rp, same, n_cases):
    g_ms, p_ms = rg["ms"] / max(1, rg["generations"]), rp["ms"] / max(1, rp["generations"])
    return {"generations": rg["generations"], "ms_per_generation": g_ms,
            "gpops_per_s": rg["nodes"] * n_cases / (rg["ms"] * 1e-3),
            "replayed": rg["replayed"], "fallbacks": rg["fallbacks"], "captures": rg["captures"],
            "ms_capture": rg["ms_capture"],
            "plain_host_driven": {"ms_per_generation": p_ms, "gpops_per_s": rp["nodes"] * n_cases / (rp["ms"] * 1e-3)},
            "speedup_vs_host_driven": p_ms / g_ms, "bitexact_vs_host_driven": same,
            "timing": "wall time of one ev_evolve call over the generations (host waits included)"}


def loop_bench(args, ev, workloads):
    """The generational loop: population 48, ramped half-and-half depth 2-6,
    tournaments of 2, 15e6-node cap.  The first `warmup` generations evolve
    the population (and capture the graphs); the next `steps` generations are
    timed, replayed from graphs, and again on the host-driven path."""
    x, y = workloads.cases(48)
    buf, off = workloads.rhh_population(workloads.SEED_BASE + 4, 48, 2, 6)
    seed, cap = 0x5EED0004, 15_000_000
    c = ev.Context(x, y, device=0)
    pop = c.load(buf, off)
    c.eval(pop)
    warm = args.warmup
    start, _, _, _ = ev.ev_evolve(c.ctx, pop, seed, 0, warm, 2, cap, history=False)
    rg, rp, same = evolve_pair(ev, c, start, seed, warm, args.steps, cap)
    # the memory-lean heap over the same generations
    kl, fl, cl, rl = ev.ev_evolve(c.ctx, start, seed, warm, args.steps, 2, cap, flags=ev.EV_EVOLVE_LEAN)
    kg, fg, _, _ = ev.ev_evolve(c.ctx, start, seed, warm, args.steps, 2, cap)
    lean = {"ms_per_generation": rl["ms"] / max(1, rl["generations"]),
            "peak_tree_bytes": rl["lean_peak_bytes"], "two_buffer_tree_bytes": rl["lean_two_buffer_bytes"],
            "peak_fraction": rl["lean_peak_bytes"] / max(1, rl["lean_two_buffer_bytes"]),
            "arena_bytes": rl["lean_arena_bytes"], "repacks": rl["lean_repacks"],
            "bitexact_vs_graph": bool(((fl.view(np.uint32) == fg.view(np.uint32)) |
                                       (np.isnan(fl) & np.isnan(fg))).all())}
    for k in (kl, kg):
        ev.ev_free_pop(c.ctx, k)
    cpu = None
    if not args.no_cpu:
        sb, so = ev.ev_get_trees(c.ctx, start)
        sf, _ = c.eval(start)
        cpu = cpu_baseline(sb, so, x, y, sf, 48)
    summ = graph_summary(rg, rp, same, 48)
    print(f"# loop: {summ}", file=sys.stderr, flush=True)
    line = {
        "metric": "GPops/s (tree nodes x fitness cases /s) on 1 MI355X; p99 eval latency",
        "value": summ["gpops_per_s"],
        "unit": "GPops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": summ["ms_per_generation"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "generational loop: population 48, ramped half-and-half depth 2-6 start, "
                        f"tournament 2, 15e6-node cap, generations {warm}..{warm + args.steps - 1}",
            "trees": 48, "fitness_cases": 48,
            "step": "one generation replayed from a captured HIP graph: tournament(2) + Philox points + "
                    "subtree crossover + device-made split plan + eval + fitness",
        },
        "graph_loop": summ,
        "lean_heap": lean,
        "roofline": None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    c.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="giant_max")
    ap.add_argument("--eval-reps", type=int, default=20)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--lds", type=int, default=0)
    ap.add_argument("--chunk-hi", type=int, default=0, help="work-item size of the skeleton levels")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default work-item sizes and grid instead of the autotuner's choice")
    ap.add_argument("--tune-cache", default="",
                    help="autotuner cache file read at start (a choice found there skips the search)")
    ap.add_argument("--plain-trees", type=int, default=-1,
                    help="trees evaluated one per launch (default: all 48 of a giant population, else 300)")
    ap.add_argument("--cap", type=int, default=-1,
                    help="child size cap of the generation step (default: 15e6 nodes, none for the giant "
                         "populations)")
    ap.add_argument("--graph-gens", type=int, default=20,
                    help="generations of the graph-replayed loop reported beside the step (not the giant "
                         "populations)")
    ap.add_argument("--requests", type=int, default=2000, help="serving: number of requests")
    ap.add_argument("--load", type=float, default=0.8, help="serving: offered load as a fraction of capacity")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 5 times (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: libev evaluates on a single device; sharding a "
              "population over several GPUs is not implemented", file=sys.stderr)
        sys.exit(2)

    if args.calibrate_copy:
        return calibrate_copy()

    import paper_1902_09215_amd as ev
    import workloads

    if args.workload == "serving":
        return serve_bench(args, ev, workloads)
    if args.workload == "loop":
        return loop_bench(args, ev, workloads)
    giant = args.workload.startswith("giant")
    cap = args.cap if args.cap >= 0 else (2**62 if giant else 15_000_000)
    buf, off, n_cases = workloads.workload(args.workload)
    x, y = workloads.cases(n_cases)
    M = off.size - 1
    print(f"# {args.workload}: {M} trees, {int(off[-1])} nodes", file=sys.stderr, flush=True)
    c = ev.Context(x, y, device=0)
    if args.chunk or args.lds or args.chunk_hi:
        ev.ev_set_tuning(c.ctx, args.chunk, args.lds, 0, args.chunk_hi)
    t_load = time.perf_counter()
    parents = c.load(buf, off)
    t_load = time.perf_counter() - t_load
    tuning = None
    if not args.no_autotune and not (args.chunk or args.lds or args.chunk_hi):
        if args.tune_cache and os.path.exists(args.tune_cache):
            ev.ev_tune_cache_load(args.tune_cache)
        t0 = time.perf_counter()
        tuning = ev.ev_autotune_ex(c.ctx, parents, 0, 2 if giant else 7)  # more timed runs where each is short
        tuning["search_s"] = time.perf_counter() - t0
        print(f"# tuning: {tuning}", file=sys.stderr, flush=True)
    # the level-0 work-item size in use
    chunk0 = args.chunk or (tuning["chunk"] if tuning else 6144)
    plan = ev.ev_get_plan_info(c.ctx, parents)
    levels = [ev.ev_get_level_info(c.ctx, parents, i) for i in range(plan["levels"])]
    funcs = ev.level_functions(c.ctx, parents)
    fit, _ = c.eval(parents)

    # ---- evaluation alone on the resident parents
    dev_ms, int_ms, lat, lvl_ms = [], [], [], []
    for r in range(args.warmup + args.eval_reps):
        t0 = time.perf_counter()
        ev.ev_eval_fitness(c.ctx, parents)
        t1 = time.perf_counter()
        a, b = ev.ev_last_timing(c.ctx)
        if r >= args.warmup:
            lat.append((t1 - t0) * 1e3)
            dev_ms.append(a)
            int_ms.append(b)
            lvl_ms.append(ev.ev_last_level_times(c.ctx))
    print(f"# evaluation: {np.median(dev_ms):.3f} ms device", file=sys.stderr, flush=True)
    nodes = int(off[-1])
    eval_gpops = nodes * n_cases / (np.median(dev_ms) * 1e-3)
    interp_ms = float(np.mean(int_ms))
    # the dominant kernel: the launch that runs level 0.  Its algorithmic
    # work is one FP32 operation per function node it evaluates, per case
    # (leaves are loads, not arithmetic).  A level-0 launch of its own leaves
    # the functions that span a work-item boundary to later launches; a
    # small level 0 runs in one chained launch with the levels after it,
    # which then evaluates all of their functions.
    in_launch0 = [i for i, lv in enumerate(levels) if lv["launch"] == levels[0]["launch"]]
    chained0 = len(in_launch0) > 1
    funcs0 = int(sum(funcs[i] for i in in_launch0))
    flops0 = funcs0 * n_cases
    achieved = flops0 / (interp_ms * 1e-3)

    # ---- generation steps (the whole hot path)
    seed = 0x5EED
    for w in range(args.warmup):
        kids, _ = ev.ev_generation(c.ctx, parents, seed, 1_000_000 + w, 2, cap)
        ev.ev_eval_fitness(c.ctx, kids)
        ev.ev_free_pop(c.ctx, kids)
    step_ms, child_nodes = [], 0
    for s in range(args.steps):
        t0 = time.perf_counter()
        kids, _ = ev.ev_generation(c.ctx, parents, seed, s, 2, cap)
        ev.ev_eval_fitness(c.ctx, kids)
        t1 = time.perf_counter()
        child_nodes += ev.ev_pop_info(c.ctx, kids)[1]
        ev.ev_free_pop(c.ctx, kids)
        step_ms.append((t1 - t0) * 1e3)
    value = child_nodes * n_cases / sum(step_ms) * 1e3
    print(f"# generation step: {np.mean(step_ms):.3f} ms", file=sys.stderr, flush=True)

    # ---- the same step as a loop of generations replayed from captured
    # graphs (the population evolves), and on the host-driven path
    graph_loop = None
    if not giant and args.graph_gens > 0:
        ev.ev_free_pop(c.ctx, ev.ev_evolve(c.ctx, parents, seed, 0, 1, 2, cap, history=False)[0])  # capture
        graph_loop = graph_summary(*evolve_pair(ev, c, parents, seed, 0, args.graph_gens, cap), n_cases)
        print(f"# graph loop: {graph_loop['ms_per_generation']:.3f} ms per generation", file=sys.stderr, flush=True)

    # ---- the plain form: one tree per launch (its own population and call),
    # timed like the batched evaluation, by HIP events around the call's kernels
    plain = None
    n_plain = args.plain_trees if args.plain_trees >= 0 else (M if giant else 300)
    if n_plain > 0 and args.workload in ("batched", "tiny", "giant", "giant_max"):
        rng = np.random.default_rng(7)
        pick = np.sort(rng.choice(M, size=min(M, n_plain), replace=False))
        t_plain, nodes_plain, same = 0.0, 0, True
        for t in pick:
            tb = np.ascontiguousarray(buf[off[t]:off[t + 1]])
            p1 = c.load(tb, np.array([0, tb.size], np.uint64))
            f1, _ = c.eval(p1)  # first call builds device caches
            f1, _ = c.eval(p1)
            t_plain += ev.ev_last_timing(c.ctx)[0] * 1e-3
            nodes_plain += tb.size
            same &= f1.view(np.uint32)[0] == fit.view(np.uint32)[t] or (np.isnan(f1[0]) and np.isnan(fit[t]))
            ev.ev_free_pop(c.ctx, p1)
        plain_gpops = nodes_plain * n_cases / t_plain
        plain = {"gpops_per_s": plain_gpops, "trees": int(pick.size),
                 "ms_per_tree": t_plain / pick.size * 1e3, "bitexact_vs_batched": bool(same),
                 "timing": "device time (HIP events) of each single-tree ev_eval_fitness, as for the batched figure",
                 "batched_speedup": eval_gpops / plain_gpops}
        print(f"# plain form: {plain_gpops:.3e} GPops/s", file=sys.stderr, flush=True)

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
            "workload": WORKLOAD_NAMES.get(args.workload, args.workload),
            "trees": M, "nodes": nodes, "fitness_cases": n_cases,
            "step": "generation: tournament(2) + Philox points + subtree crossover + scan/split + eval + fitness",
            "child_size_cap": cap if cap < 2**62 else None,
            "tuning": tuning,
        },
        "p50_step_ms": pct(step_ms, 50),
        "p99_step_ms": pct(step_ms, 99),
        "eval": {
            "gpops_per_s": eval_gpops,
            "device_ms_median": float(np.median(dev_ms)),
            "level_ms_median": [float(v) for v in np.median(np.asarray(lvl_ms), axis=0)] if lvl_ms else None,
            "p50_latency_ms": pct(lat, 50),
            "p99_latency_ms": pct(lat, 99),
            "plan": plan,
            "levels": levels,
            "load_and_plan_s": t_load,
        },
        "roofline": {
            "kernel": (f"k_run_chain (levels 0-{in_launch0[-1]} of the plan in one chained launch)" if chained0
                       else "k_run (level-0 register-stack interpreter launch)"),
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_FP32 / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32,
            "frac_of_unpacked_fp32": achieved / PEAK_UNPACKED,
            "avg_launch_ms": interp_ms,
            "work_per_launch": f"{funcs0} function nodes evaluated by the launch x {n_cases} cases "
                               f"(one FP32 operation each)",
            "gpops_per_s_level0": levels[0]["tokens"] * n_cases / (interp_ms * 1e-3),
            "traffic": measured_traffic(args.workload, chunk0),
        },
        "plain_one_tree_per_launch": plain,
        "graph_loop": graph_loop,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    c.close()


if __name__ == "__main__":
    main()
