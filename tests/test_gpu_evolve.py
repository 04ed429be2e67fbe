"""The generational loop replayed from captured HIP graphs (ev_evolve)
against the oracle's loop, generation by generation, bit for bit: every
generation's children's fitness, their number over the size cap, and the
last generation's trees."""
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

THREADS = min(os.cpu_count() or 1, 16)


def same_bits(a, b):
    a = np.asarray(a, np.float32)
    b = np.asarray(b, np.float32)
    return (a.view(np.uint32) == b.view(np.uint32)) | (np.isnan(a) & np.isnan(b))


def assert_same(got, want, what=""):
    ok = same_bits(got, want)
    if not ok.all():
        idx = np.argwhere(~ok)[:5]
        raise AssertionError(f"{what}: {int((~ok).sum())} mismatches, first {idx.tolist()}")


@pytest.fixture(scope="module")
def ev():
    import paper_1902_09215_amd as ev

    ev.load_library()
    return ev


def oracle_loop(buf, off, x, y, seed, gen0, gens, k, cap):
    """The oracle's generations gen0 .. gen0 + gens - 1: each generation's
    fitness and capped count, and the last generation's trees."""
    fit = oracle.eval_population(buf, off, x, y, threads=THREADS)
    fits, capped = [], []
    for g in range(gen0, gen0 + gens):
        buf, off, cp = oracle.generation(buf, off, fit, k, seed, g, cap)
        fit = oracle.eval_population(buf, off, x, y, threads=THREADS)
        fits.append(fit)
        capped.append(cp)
    return np.array(fits).reshape(gens, -1), np.array(capped), buf, off


def check_run(ev, c, kids, fh, ch, want, what):
    wfits, wcapped, wbuf, woff = want
    for g in range(wfits.shape[0]):
        assert_same(fh[g], wfits[g], f"{what}: generation {g} fitness")
    assert np.array_equal(ch, wcapped), f"{what}: capped counts"
    gbuf, goff = ev.ev_get_trees(c.ctx, kids)
    assert np.array_equal(goff, woff), f"{what}: last generation's offsets"
    assert np.array_equal(gbuf, wbuf), f"{what}: last generation's trees"
    fit, _ = c.eval(kids)
    assert_same(fit, wfits[-1], f"{what}: last generation evaluated again")


def test_evolve_1000_generations_replayed_from_graphs(ev):
    # the full generational loop: population 48, ramped half-and-half start,
    # size-2 tournaments, 15e6-node cap, 1000 generations, each one graph
    x, y = workloads.cases(48)
    buf, off = workloads.rhh_population(workloads.SEED_BASE + 4, 48, 2, 6)
    seed, gens, cap = 0x5EED0004, 1000, 15_000_000
    want = oracle_loop(buf, off, x, y, seed, 0, gens, 2, cap)
    print(f"oracle done: last mean size {np.diff(want[3]).mean():.0f}", flush=True)
    with ev.Context(x, y) as c:
        pop = c.load(buf, off)
        c.eval(pop)
        kids, fh, ch, rep = ev.ev_evolve(c.ctx, pop, seed, 0, gens, 2, cap)
        print(f"report: {rep}", flush=True)
        check_run(ev, c, kids, fh, ch, want, "graph loop")
        assert rep["generations"] == gens
        assert rep["replayed"] + rep["fallbacks"] == gens
        assert rep["replayed"] >= gens * 9 // 10, rep
        assert rep["captures"] >= 2


def test_evolve_plain_form_and_continued_calls(ev):
    # the host-driven loop, and the graph loop in two calls (the second
    # starting from the first's output, on the graphs the first captured)
    x, y = workloads.cases(48)
    buf, off = workloads.rhh_population(workloads.SEED_BASE + 5, 60, 2, 6)
    seed, cap = 77, 15_000_000
    want = oracle_loop(buf, off, x, y, seed, 0, 40, 2, cap)
    with ev.Context(x, y) as c:
        pop = c.load(buf, off)
        c.eval(pop)
        kids, fh, ch, rep = ev.ev_evolve(c.ctx, pop, seed, 0, 40, 2, cap, flags=ev.EV_EVOLVE_NO_GRAPH)
        assert rep["replayed"] == 0 and rep["generations"] == 40
        check_run(ev, c, kids, fh, ch, want, "plain loop")
        k1, fh1, ch1, r1 = ev.ev_evolve(c.ctx, pop, seed, 0, 20, 2, cap)
        k2, fh2, ch2, r2 = ev.ev_evolve(c.ctx, k1, seed, 20, 20, 2, cap)
        print(f"reports: {r1} {r2}", flush=True)
        check_run(ev, c, k2, np.concatenate([fh1, fh2]), np.concatenate([ch1, ch2]), want, "two calls")
        assert r1["replayed"] > 0 and r2["replayed"] > 0


def test_evolve_tight_capacities_fall_back(ev):
    # capacities of exactly the last sizes seen: most generations overflow
    # one and are done again on the host-driven path; results are unchanged
    x, y = workloads.cases(48)
    buf, off = workloads.rhh_population(workloads.SEED_BASE + 6, 48, 2, 6)
    seed, cap = 2024, 15_000_000
    want = oracle_loop(buf, off, x, y, seed, 0, 30, 7, cap)
    with ev.Context(x, y) as c:
        ev.ev_set_tuning(c.ctx, 64)  # many work items and levels, so every count can overflow
        pop = c.load(buf, off)
        c.eval(pop)
        kids, fh, ch, rep = ev.ev_evolve(c.ctx, pop, seed, 0, 30, 7, cap, flags=ev.EV_EVOLVE_TEST_TIGHT)
        print(f"report: {rep}", flush=True)
        check_run(ev, c, kids, fh, ch, want, "tight capacities")
        assert rep["fallbacks"] > 0


def test_evolve_batched_uneven_population(ev):
    # 4000 trees of 10 .. 1e5 nodes: several plan levels per generation,
    # with small work items so that the plan made on the device has many
    x, y = workloads.cases(48)
    sizes = workloads.loguniform_sizes(91, 4000, 10, 1e5)
    buf, off = workloads.random_population(91, sizes)
    seed, cap, gens = 4000, 15_000_000, 4
    want = oracle_loop(buf, off, x, y, seed, 0, gens, 2, cap)
    for chunk in (0, 1024):
        with ev.Context(x, y) as c:
            if chunk:
                ev.ev_set_tuning(c.ctx, chunk)
            pop = c.load(buf, off)
            c.eval(pop)
            kids, fh, ch, rep = ev.ev_evolve(c.ctx, pop, seed, 0, gens, 2, cap)
            print(f"chunk {chunk}: report {rep}", flush=True)
            check_run(ev, c, kids, fh, ch, want, f"batched chunk {chunk}")
            assert rep["replayed"] > 0


def test_evolve_capped_children_and_device_fitness(ev):
    # a tight size cap (children over it are copies of their mums) and the
    # parents' fitness handed over as a device tensor
    import torch

    x, y = workloads.cases(48)
    buf, off = workloads.rhh_population(workloads.SEED_BASE + 8, 100, 3, 8)
    seed, cap = 99, 200
    want = oracle_loop(buf, off, x, y, seed, 5, 25, 2, cap)
    assert want[1].sum() > 0
    with ev.Context(x, y) as c:
        pop = c.load(buf, off)
        fit, _ = c.eval(pop)
        dfit = torch.from_numpy(fit).cuda()
        kids, fh, ch, rep = ev.ev_evolve(c.ctx, pop, seed, 5, 25, 2, cap, fitness=dfit)
        check_run(ev, c, kids, fh, ch, want, "capped")
        kids0, fh0, ch0, rep0 = ev.ev_evolve(c.ctx, pop, seed, 5, 0, 2, cap)
        assert fh0.shape == (0, 100) and rep0["generations"] == 0
        b0, o0 = ev.ev_get_trees(c.ctx, kids0)
        assert np.array_equal(o0, off) and np.array_equal(b0, buf)


@pytest.mark.parametrize("m,k", [(200, 2), (500, 7)])
def test_evolve_lean_heap(ev, m, k):
    # the memory-lean loop: the population as a heap of trees, children made
    # in batches by lower parent index and parents' bytes reused once their
    # last child is made; every generation equals the oracle's, with fewer
    # bytes alive than separate parent and child buffers would hold
    x, y = workloads.cases(48)
    buf, off = workloads.rhh_population(workloads.SEED_BASE + 9 + k, m, 2, 6)
    seed, cap, gens = 31 + k, 15_000_000, 40
    want = oracle_loop(buf, off, x, y, seed, 0, gens, k, cap)
    with ev.Context(x, y) as c:
        pop = c.load(buf, off)
        c.eval(pop)
        kids, fh, ch, rep = ev.ev_evolve(c.ctx, pop, seed, 0, gens, k, cap, flags=ev.EV_EVOLVE_LEAN)
        print(f"report: {rep}", flush=True)
        check_run(ev, c, kids, fh, ch, want, f"lean heap m={m} k={k}")
        assert rep["generations"] == gens and rep["replayed"] == 0
        assert 0 < rep["lean_peak_bytes"] < 0.85 * rep["lean_two_buffer_bytes"], rep
        # the caller's population is untouched
        b0, o0 = ev.ev_get_trees(c.ctx, pop)
        assert np.array_equal(o0, off) and np.array_equal(b0, buf)
