"""GPU parity: libev (HIP, through the C ABI) against the oracle, bit for bit.

Floating-point results must match at 0 ULP (or both be NaN: NaN payloads
differ between x86 and AMD), because both sides apply the same binary32
operations to the same operands in the same order and reduce the fitness
in ascending case order.
"""
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

ADD, SUB, MUL, DIV, X = 0, 1, 2, 3, 4


def same_bits(a, b):
    a = np.asarray(a, np.float32)
    b = np.asarray(b, np.float32)
    return (a.view(np.uint32) == b.view(np.uint32)) | (np.isnan(a) & np.isnan(b))


def assert_same(got, want, what=""):
    ok = same_bits(got, want)
    if not ok.all():
        idx = np.argwhere(~ok)[:5]
        raise AssertionError(f"{what}: {int((~ok).sum())} mismatches, first {idx.tolist()}: "
                             f"got {np.asarray(got)[tuple(idx.T)]} want {np.asarray(want)[tuple(idx.T)]}")


@pytest.fixture(scope="module")
def ev():
    import paper_1902_09215_amd as ev

    ev.load_library()
    return ev


def run(ev, buf, off, x, y, chunk=0, lds=0, per_case=True, flags=0, chunk_hi=0):
    with ev.Context(x, y) as c:
        if chunk or lds or flags or chunk_hi:
            ev.ev_set_tuning(c.ctx, chunk, lds, flags, chunk_hi)
        pop = c.load(buf, off)
        info = ev.ev_get_plan_info(c.ctx, pop)
        fit, pc, hits = c.eval(pop, per_case=per_case, hits=True)
    return fit, pc, info, hits


def check(ev, buf, off, x, y, chunk=0, lds=0, threads=8, what="", both=True, chunk_hi=0):
    """Both interpreters (register-stack and general), and both ways of
    emitting the codes (placing the counting pass's recording, or a second
    pass), against the oracle: per-case values, fitness and hits."""
    want_fit, want_pc = oracle.eval_population(buf, off, x, y, threads=threads, per_case=True)
    want_hits = oracle.hits(want_pc, y)
    info = None
    for flags in ((0, ev.EV_TUNE_NO_REGSTACK, ev.EV_TUNE_NO_RECORD) if both else (0,)):
        fit, pc, inf, hits = run(ev, buf, off, x, y, chunk, lds, flags=flags, chunk_hi=chunk_hi)
        assert_same(pc, want_pc, f"per-case {what} flags={flags}")
        assert_same(fit, want_fit, f"fitness {what} flags={flags}")
        assert np.array_equal(hits, want_hits), f"hits {what} flags={flags}"
        info = info or inf
    return info


def test_tiny_rhh_population(ev):
    x, y = workloads.cases(48)
    buf, off = workloads.rhh_population(workloads.SEED_BASE + 1, 100, 2, 6)
    print("tiny rhh: 100 trees", flush=True)
    check(ev, buf, off, x, y, what="tiny")


@pytest.mark.parametrize("chunk", [64, 256, 4096, 1 << 20])
@pytest.mark.parametrize("lds", [64, 128])
def test_split_invariance(ev, chunk, lds):
    x, y = workloads.cases(48)
    sizes = workloads.loguniform_sizes(77, 150, 1, 40000)
    buf, off = workloads.random_population(77, sizes)
    print(f"split chunk={chunk} lds={lds} nodes={int(off[-1])}", flush=True)
    info = check(ev, buf, off, x, y, chunk=chunk, lds=lds, what=f"chunk {chunk} lds {lds}")
    if chunk <= 4096:
        assert info["levels"] >= 2


@pytest.mark.parametrize("chunk_hi", [64, 256, 4096])
def test_skeleton_split_invariance(ev, chunk_hi):
    # the skeleton levels split at their own work-item size
    x, y = workloads.cases(48)
    sizes = workloads.loguniform_sizes(78, 60, 1000, 200000)
    buf, off = workloads.random_population(78, sizes)
    print(f"skeleton split chunk_hi={chunk_hi} nodes={int(off[-1])}", flush=True)
    info = check(ev, buf, off, x, y, chunk=1024, chunk_hi=chunk_hi, what=f"chunk_hi {chunk_hi}")
    assert info["levels"] >= 2


@pytest.mark.parametrize("n_cases", [48, 130])
def test_skeleton_levels_chained_and_separate(ev, n_cases):
    # many skeleton levels (64-token work items), evaluated in one chained
    # launch (a tree's items at a level start once its items of the level
    # before are done) and in one launch per level, against the oracle;
    # deep trees spill at the skeleton levels too
    x, y = workloads.cases(n_cases)
    sizes = workloads.loguniform_sizes(79, 90, 10, 300000)
    buf, off = workloads.random_population(79, sizes)
    deep = np.array([ADD, MUL, SUB, DIV] * 2500 + [X] * 10001, np.uint8)
    buf = np.concatenate([buf, deep])
    off = np.append(off, off[-1] + deep.size).astype(np.uint64)
    want_fit, want_pc = oracle.eval_population(buf, off, x, y, threads=8, per_case=True)
    for flags in (0, ev.EV_TUNE_NO_CHAIN):
        fit, pc, info, hits = run(ev, buf, off, x, y, chunk=64, flags=flags)
        print(f"flags {flags}: levels {info['levels']}", flush=True)
        assert info["levels"] >= 4
        assert_same(pc, want_pc, f"per-case flags={flags}")
        assert_same(fit, want_fit, f"fitness flags={flags}")


def test_deep_stacks_spill_to_memory(ev):
    # (((x+x)*x)-x)... leans left: the right-to-left stack holds every leaf
    x, y = workloads.cases(48)
    trees = []
    for k, op_cycle in ((3000, [ADD, MUL, SUB, DIV]), (700, [DIV, SUB]), (129, [MUL])):
        ops = [op_cycle[i % len(op_cycle)] for i in range(k)]
        trees.append(np.array(ops + [X] * (k + 1), np.uint8))
        trees.append(np.array(sum(([o, X] for o in ops), []) + [X], np.uint8))  # leans right
    sizes = [t.size for t in trees]
    off = workloads.offsets_from_sizes(sizes)
    buf = np.concatenate(trees)
    print("deep stacks", flush=True)
    for chunk, lds in ((1 << 20, 64), (512, 64), (1 << 20, 128), (256, 128)):
        info = check(ev, buf, off, x, y, chunk=chunk, lds=lds, what=f"deep chunk {chunk} lds {lds}")
        assert info["max_stack"] >= 128


@pytest.mark.parametrize("n_cases", [1, 2, 47, 64, 65, 130, 1024])
def test_case_counts(ev, n_cases):
    x, y = workloads.cases(n_cases)
    sizes = workloads.loguniform_sizes(5, 60, 1, 9000)
    buf, off = workloads.random_population(5, sizes)
    print(f"cases N={n_cases}", flush=True)
    check(ev, buf, off, x, y, chunk=1024, what=f"N={n_cases}")


def test_special_inputs(ev):
    # zero, signed zero, subnormals, huge and infinite inputs drive every
    # path of protected division and NaN propagation
    x = np.array([0.0, -0.0, 1e-45, -1e-40, 3.4e38, -3.4e38, np.inf, -np.inf, np.nan, 1.0, -1.0, 0.5,
                  1e-20, 1e20, 2.0, -3.0], np.float32)
    y = np.linspace(-1, 1, x.size).astype(np.float32)
    sizes = workloads.loguniform_sizes(8, 200, 1, 3000)
    buf, off = workloads.random_population(8, sizes)
    print("special inputs", flush=True)
    check(ev, buf, off, x, y, chunk=512, what="special")


def test_single_leaf_and_tiny_trees(ev):
    x, y = workloads.cases(48)
    trees = [np.array([X], np.uint8), np.array([DIV, X, X], np.uint8), np.array([SUB, X, X], np.uint8),
             np.array([DIV, X, SUB, X, X], np.uint8)]
    off = workloads.offsets_from_sizes([t.size for t in trees])
    buf = np.concatenate(trees)
    check(ev, buf, off, x, y, what="tiny trees")


def test_batched_workload_full_size(ev):
    # 4000 trees, 10..1e5 nodes (~4.3e7 nodes), in the launch configuration
    # the benchmark uses
    buf, off, n = workloads.workload("batched")
    x, y = workloads.cases(n)
    print(f"batched: {int(off[-1])} nodes", flush=True)
    want_fit, want_pc = oracle.eval_population(buf, off, x, y, threads=16, per_case=True)
    fit, _, info, hits = run(ev, buf, off, x, y, per_case=False)
    assert_same(fit, want_fit, "batched fitness")
    assert np.array_equal(hits, oracle.hits(want_pc, y)), "batched hits"


def test_repeatable(ev):
    x, y = workloads.cases(48)
    sizes = workloads.loguniform_sizes(9, 300, 1, 20000)
    buf, off = workloads.random_population(9, sizes)
    with ev.Context(x, y) as c:
        pop = c.load(buf, off)
        a, pa = c.eval(pop, per_case=True)
        b, pb = c.eval(pop, per_case=True)
    assert_same(a, b, "repeat fitness")
    assert_same(pa, pb, "repeat per-case")


def test_malformed_trees_are_rejected(ev):
    x, y = workloads.cases(48)
    good = workloads.random_tree(1, 1, 21)
    cases = {
        "truncated": good[:-1],
        "trailing": np.append(good, X),
        "bad opcode": np.concatenate([good[:5], [7], good[6:]]).astype(np.uint8),
        "reserved token": np.concatenate([[ADD], [5], [X]]).astype(np.uint8),
    }
    with ev.Context(x, y) as c:
        for name, bad in cases.items():
            trees = [good, bad, good]
            off = workloads.offsets_from_sizes([t.size for t in trees])
            with pytest.raises(ev.EvError) as ei:
                c.load(np.concatenate(trees).astype(np.uint8), off)
            assert ei.value.code == ev.EV_EMALFORMED, name
            assert ei.value.bad_tree == 1, name
        # an empty tree
        with pytest.raises(ev.EvError):
            c.load(good, np.array([0, 0, good.size], np.uint64))


def test_malformed_multi_chunk_trees_are_rejected(ev):
    # Validity of trees split over many work items: the per-chunk counters are
    # combined across chunk boundaries on the device (Sec. 2.2's slot count).
    x, y = workloads.cases(48)
    good = workloads.random_tree(2, 2, 4001)
    mid = good.size // 2
    cases = {
        "truncated": good[:-1],
        "two trees in one": np.concatenate([good, good]),
        "leaf dropped mid-way": np.delete(good, mid + np.flatnonzero(good[mid:] == X)[0]),
        "function dropped mid-way": np.delete(good, mid + np.flatnonzero(good[mid:] < X)[0]),
        "bad opcode mid-way": np.concatenate([good[:mid], [9], good[mid + 1:]]).astype(np.uint8),
    }
    for chunk in (64, 1000):
        with ev.Context(x, y) as c:
            ev.ev_set_tuning(c.ctx, chunk, 0, 0, chunk)
            for name, bad in cases.items():
                trees = [good, bad.astype(np.uint8), good]
                off = workloads.offsets_from_sizes([t.size for t in trees])
                with pytest.raises(ev.EvError) as ei:
                    c.load(np.concatenate(trees).astype(np.uint8), off)
                assert ei.value.code == ev.EV_EMALFORMED, (name, chunk)
                assert ei.value.bad_tree == 1, (name, chunk)
            # the valid trees alone still load and match the oracle
            trees = [good, good]
            off = workloads.offsets_from_sizes([t.size for t in trees])
            fit, _ = c.eval(c.load(np.concatenate(trees).astype(np.uint8), off))
            ref = oracle.eval_population(np.concatenate(trees).astype(np.uint8), off, x, y)
            assert_same(fit, ref, f"valid trees, chunk {chunk}")


def test_crossover_matches_oracle(ev):
    x, y = workloads.cases(48)
    rng = np.random.default_rng(31)
    sizes = workloads.loguniform_sizes(31, 64, 1, 20000)
    buf, off = workloads.random_population(31, sizes)
    n = 100
    mum = rng.integers(0, 64, n).astype(np.int32)
    dad = rng.integers(0, 64, n).astype(np.int32)
    p = np.array([rng.integers(0, sizes[m]) for m in mum], np.uint64)
    q = np.array([rng.integers(0, sizes[d]) for d in dad], np.uint64)
    cap = int(np.median(sizes)) * 2
    with ev.Context(x, y) as c:
        pop = c.load(buf, off)
        kids, capped = ev.ev_crossover(c.ctx, pop, pop, mum, dad, p, q, cap)
        cbuf, coff = ev.ev_get_trees(c.ctx, kids)
        fit, pc = c.eval(kids, per_case=True)
    want = []
    n_cap = 0
    for j in range(n):
        mt = buf[off[mum[j]]:off[mum[j] + 1]]
        dt = buf[off[dad[j]]:off[dad[j] + 1]]
        child = oracle.crossover(mt, dt, int(p[j]), int(q[j]))
        if child.size > cap:
            child, n_cap = mt, n_cap + 1
        want.append(child)
    assert capped == n_cap
    woff = workloads.offsets_from_sizes([t.size for t in want])
    assert np.array_equal(coff, woff)
    assert np.array_equal(cbuf, np.concatenate(want))
    wfit, wpc = oracle.eval_population(cbuf, coff, x, y, threads=8, per_case=True)
    assert_same(fit, wfit, "children fitness")
    assert_same(pc, wpc, "children per-case")


def test_generations_match_oracle(ev):
    # population 48, size-2 tournament, Philox-drawn points, 15e6-node cap
    x, y = workloads.cases(48)
    buf, off = workloads.rhh_population(workloads.SEED_BASE + 4, 48, 2, 6)
    seed, gens, cap = 20240601, 60, 15_000_000
    with ev.Context(x, y) as c:
        pop = c.load(buf, off)
        fit, _ = c.eval(pop)
        wfit = oracle.eval_population(buf, off, x, y)
        assert_same(fit, wfit, "gen 0")
        for g in range(gens):
            kids, capped = ev.ev_generation(c.ctx, pop, seed, g, 2, cap)
            wbuf, woff, wcap = oracle.generation(buf, off, wfit, 2, seed, g, cap)
            gbuf, goff = ev.ev_get_trees(c.ctx, kids)
            assert capped == wcap
            assert np.array_equal(goff, woff), f"gen {g} offsets"
            assert np.array_equal(gbuf, wbuf), f"gen {g} trees"
            fit, _ = c.eval(kids)
            wfit = oracle.eval_population(wbuf, woff, x, y, threads=8)
            assert_same(fit, wfit, f"gen {g + 1} fitness")
            ev.ev_free_pop(c.ctx, pop)
            pop, buf, off = kids, wbuf, woff


def crossover_cases(buf, off, C, rng):
    """Crossover points around a mum's level-0 chunk boundaries (chunks of C
    tokens from the tree's root): p on a boundary and just before one, p
    whose subtree ends just before or on a boundary, the root (nothing
    kept), leaves, q = 0 (the whole dad inserted), random points."""
    sizes = np.diff(off).astype(np.int64)
    big = [t for t in range(sizes.size) if sizes[t] > 4 * C]
    mum, dad, p, q = [], [], [], []
    for m in big[:12]:
        tree = buf[off[m]:off[m + 1]]
        ends = np.array([oracle.subtree_end(tree, k) for k in range(tree.size)])
        pts = {0, C, C - 1, 2 * C, 2 * C + 1, int(tree.size) - 1}
        for want in (C - 1, 0, 1):  # subtree ending just before / on / after a boundary
            hit = np.nonzero(((ends + 1) % C == (want + 1) % C) & (np.arange(tree.size) > 0))[0]
            if hit.size:
                pts.add(int(rng.choice(hit)))
        leaves = np.nonzero(tree == X)[0]
        pts.add(int(rng.choice(leaves)))
        pts.update(int(v) for v in rng.integers(0, tree.size, 3))
        for pp in sorted(v for v in pts if 0 <= v < tree.size):
            d = int(rng.integers(0, sizes.size))
            qq = 0 if rng.random() < 0.2 else int(rng.integers(0, sizes[d]))
            mum.append(m), dad.append(d), p.append(pp), q.append(qq)
    return (np.array(mum, np.int32), np.array(dad, np.int32), np.array(p, np.uint64), np.array(q, np.uint64))


@pytest.mark.parametrize("chunk", [64, 300])
def test_children_reuse_their_mums_chunks(ev, chunk):
    # A child keeps its mum's level-0 work items that crossover leaves intact
    # (their codes and skeleton fragments are copied) and plans only the
    # tokens between them.  Around every kind of chunk boundary, and for
    # children over the size cap (copies of their mum), the children's bytes,
    # per-case values and fitness equal the oracle's and a plan from scratch.
    x, y = workloads.cases(48)
    rng = np.random.default_rng(chunk)
    sizes = workloads.loguniform_sizes(61, 40, 3, 6000)
    buf, off = workloads.random_population(61, sizes)
    mum, dad, p, q = crossover_cases(buf, off, chunk, rng)
    print(f"chunk {chunk}: {mum.size} children", flush=True)
    kids = [oracle.crossover(buf[off[m]:off[m + 1]], buf[off[d]:off[d + 1]], int(pp), int(qq))
            for m, d, pp, qq in zip(mum, dad, p, q)]
    koff = workloads.offsets_from_sizes([k.size for k in kids])
    kbuf = np.concatenate(kids)
    want_fit, want_pc = oracle.eval_population(kbuf, koff, x, y, threads=8, per_case=True)
    results = {}
    for flags in (0, ev.EV_TUNE_NO_REUSE, ev.EV_TUNE_NO_RECORD):
        with ev.Context(x, y) as c:
            ev.ev_set_tuning(c.ctx, chunk, 0, flags)
            pop = c.load(buf, off)
            k, capped = ev.ev_crossover(c.ctx, pop, pop, mum, dad, p, q)
            assert capped == 0
            gb, go = ev.ev_get_trees(c.ctx, k)
            assert np.array_equal(go, koff) and np.array_equal(gb, kbuf)
            fit, pc = c.eval(k, per_case=True)
            assert_same(pc, want_pc, f"children per-case flags={flags}")
            assert_same(fit, want_fit, f"children fitness flags={flags}")
            # children over the cap are copies of their mums: all kept
            cap = int(np.diff(koff).min()) - 1
            k2, capped2 = ev.ev_crossover(c.ctx, pop, pop, mum, dad, p, q, size_cap=max(cap, 1))
            gb2, go2 = ev.ev_get_trees(c.ctx, k2)
            f2, pc2 = c.eval(k2, per_case=True)
            results[flags] = (gb2, go2, f2, pc2, capped2)
            # and the children of children (non-uniform chunks in the mum)
            j = np.arange(mum.size, dtype=np.int32)
            ksz = np.diff(koff).astype(np.int64)
            p3 = np.array([int(rng.integers(0, s)) if s > 1 else 0 for s in ksz], np.uint64)
            q3 = np.array([int(rng.integers(0, ksz[(i + 1) % ksz.size])) for i in range(ksz.size)], np.uint64)
            d3 = ((j + 1) % mum.size).astype(np.int32)
            g3, _ = ev.ev_crossover(c.ctx, k, k, j, d3, p3, q3)
            gb3, go3 = ev.ev_get_trees(c.ctx, g3)
            f3, pc3 = c.eval(g3, per_case=True)
            want3 = [oracle.crossover(kids[a], kids[b], int(pp), int(qq)) for a, b, pp, qq in zip(j, d3, p3, q3)]
            w3off = workloads.offsets_from_sizes([w.size for w in want3])
            w3buf = np.concatenate(want3)
            assert np.array_equal(go3, w3off) and np.array_equal(gb3, w3buf)
            wf3, wpc3 = oracle.eval_population(w3buf, w3off, x, y, threads=8, per_case=True)
            assert_same(pc3, wpc3, f"grandchildren per-case flags={flags}")
            assert_same(f3, wf3, f"grandchildren fitness flags={flags}")
    # a child over the cap is a copy of its mum (a one-node child is not over it)
    cap = max(int(np.diff(koff).min()) - 1, 1)
    over = np.diff(koff) > cap
    capk = [buf[off[m]:off[m + 1]] if o else kk for m, o, kk in zip(mum, over, kids)]
    moff = workloads.offsets_from_sizes([t.size for t in capk])
    mbuf = np.concatenate(capk)
    for r in results.values():
        assert r[4] == int(over.sum()) > 0
        assert np.array_equal(r[0], mbuf) and np.array_equal(r[1], moff)
    wf, wpc = oracle.eval_population(mbuf, moff, x, y, threads=8, per_case=True)
    for flags, r in results.items():
        assert_same(r[2], wf, f"capped children fitness flags={flags}")
        assert_same(r[3], wpc, f"capped children per-case flags={flags}")


def test_generations_reusing_chunks_match_oracle(ev):
    # Generations of trees spanning many 64-token work items: every child
    # plan takes over its mum's intact chunks, and the mum's own chunks came
    # from its mum's, so chunk layouts grow uneven over the generations.
    x, y = workloads.cases(48)
    sizes = workloads.loguniform_sizes(62, 48, 200, 3000)
    buf, off = workloads.random_population(62, sizes)
    seed, gens, cap = 777, 25, 15_000_000
    with ev.Context(x, y) as c:
        ev.ev_set_tuning(c.ctx, 64)
        pop = c.load(buf, off)
        fit, _ = c.eval(pop)
        wfit = oracle.eval_population(buf, off, x, y, threads=8)
        assert_same(fit, wfit, "gen 0")
        for g in range(gens):
            kids, capped = ev.ev_generation(c.ctx, pop, seed, g, 2, cap)
            wbuf, woff, wcap = oracle.generation(buf, off, wfit, 2, seed, g, cap)
            gbuf, goff = ev.ev_get_trees(c.ctx, kids)
            assert capped == wcap
            assert np.array_equal(goff, woff) and np.array_equal(gbuf, wbuf), f"gen {g} trees"
            fit, pc = c.eval(kids, per_case=True)
            wfit, wpc = oracle.eval_population(wbuf, woff, x, y, threads=8, per_case=True)
            assert_same(pc, wpc, f"gen {g + 1} per-case")
            assert_same(fit, wfit, f"gen {g + 1} fitness")
            ev.ev_free_pop(c.ctx, pop)
            pop, buf, off = kids, wbuf, woff


def test_generations_tournament_7_population_500(ev):
    # Table 1's tournament size (7) on a population of 500: trees, fitness and
    # hits bit-identical to the oracle's generations.
    x, y = workloads.cases(48)
    buf, off = workloads.rhh_population(workloads.SEED_BASE + 7, 500, 2, 6)
    seed, gens, cap = 4242, 12, 15_000_000
    with ev.Context(x, y) as c:
        pop = c.load(buf, off)
        fit, _ = c.eval(pop)
        wfit = oracle.eval_population(buf, off, x, y, threads=8)
        assert_same(fit, wfit, "gen 0")
        for g in range(gens):
            kids, capped = ev.ev_generation(c.ctx, pop, seed, g, 7, cap)
            wbuf, woff, wcap = oracle.generation(buf, off, wfit, 7, seed, g, cap)
            gbuf, goff = ev.ev_get_trees(c.ctx, kids)
            assert capped == wcap
            assert np.array_equal(goff, woff) and np.array_equal(gbuf, wbuf), f"gen {g} trees"
            fit, _, hits = c.eval(kids, hits=True)
            wfit, wpc = oracle.eval_population(wbuf, woff, x, y, threads=8, per_case=True)
            assert_same(fit, wfit, f"gen {g + 1} fitness")
            assert np.array_equal(hits, oracle.hits(wpc, y)), f"gen {g + 1} hits"
            ev.ev_free_pop(c.ctx, pop)
            pop, buf, off = kids, wbuf, woff


@pytest.mark.parametrize("chunk", [64, 512, 1 << 20])
def test_constants_match_oracle(ev, chunk):
    # Ephemeral random constants (Sec. 2.1, Table 1): 250 constants from
    # -1.000 .. +1.000 as terminals beside x; constant-rich trees (half the
    # leaves constants), split at several work-item sizes so that constants
    # also reach the skeleton levels; per-case values, fitness and hits equal
    # the oracle's, and single-constant trees give their constant.
    x, y = workloads.cases(48)
    consts = workloads.erc_table(81, 250)
    sizes = workloads.loguniform_sizes(82, 300, 1, 20000)
    buf, off = workloads.random_population(82, sizes)
    buf = workloads.with_constants(buf, 83, 250, 0.5)
    singles = np.arange(6, 256, dtype=np.uint8)
    buf = np.concatenate([buf, singles])
    off = np.concatenate([off, off[-1] + np.arange(1, singles.size + 1, dtype=np.uint64)])
    want_fit, want_pc = oracle.eval_population(buf, off, x, y, threads=8, per_case=True, consts=consts)
    assert (want_pc[-250:] == consts[:, None]).all()
    with ev.Context(x, y) as c:
        ev.ev_set_constants(c.ctx, consts)
        ev.ev_set_tuning(c.ctx, chunk)
        pop = c.load(buf, off)
        fit, pc, hits = c.eval(pop, per_case=True, hits=True)
    assert_same(pc, want_pc, f"constants per-case chunk={chunk}")
    assert_same(fit, want_fit, f"constants fitness chunk={chunk}")
    assert np.array_equal(hits, oracle.hits(want_pc, y))


def test_constants_in_generations_and_serving(ev):
    # children of constant-rich parents (planned from scratch in a context
    # with constants), their evaluation, and served requests, against the
    # oracle; tokens outside the table are refused
    x, y = workloads.cases(48)
    consts = workloads.erc_table(84, 100)
    pbuf, poff = workloads.rhh_population(workloads.SEED_BASE + 8, 64, 2, 6)
    pbuf = workloads.with_constants(pbuf, 85, 100, 0.4)
    seed, cap = 91, 15_000_000
    with ev.Context(x, y) as c:
        ev.ev_set_constants(c.ctx, consts)
        pop = c.load(pbuf, poff)
        fit, _ = c.eval(pop)
        wfit = oracle.eval_population(pbuf, poff, x, y, threads=8, consts=consts)
        assert_same(fit, wfit, "parents")
        buf, off = pbuf, poff
        for g in range(8):
            kids, capped = ev.ev_generation(c.ctx, pop, seed, g, 7, cap)
            wbuf, woff, wcap = oracle.generation(buf, off, wfit, 7, seed, g, cap)
            gbuf, goff = ev.ev_get_trees(c.ctx, kids)
            assert capped == wcap and np.array_equal(goff, woff) and np.array_equal(gbuf, wbuf), f"gen {g}"
            fit, _ = c.eval(kids)
            wfit = oracle.eval_population(wbuf, woff, x, y, threads=8, consts=consts)
            assert_same(fit, wfit, f"gen {g + 1}")
            ev.ev_free_pop(c.ctx, pop)
            pop, buf, off = kids, wbuf, woff
        tickets = [ev.ev_submit_eval(c.ctx, buf[off[t]:off[t + 1]], np.array([0, off[t + 1] - off[t]], np.uint64))
                   for t in range(0, 64, 3)]
        for k, tk in zip(range(0, 64, 3), tickets):
            assert ev.ev_wait(c.ctx, tk) == 0
            f, _ = ev.ev_result(c.ctx, tk, 1, 48)
            assert_same(f, wfit[k:k + 1], f"served tree {k}")
        bad = np.array([ADD, X, 6 + 100], np.uint8)
        with pytest.raises(ev.EvError) as e:
            c.load(bad, np.array([0, 3], np.uint64))
        assert e.value.code == ev.EV_EMALFORMED
        with pytest.raises(ev.EvError) as e:
            c.load(np.array([ADD, X, 5], np.uint8), np.array([0, 3], np.uint64))
        assert e.value.code == ev.EV_EMALFORMED
        with pytest.raises(ev.EvError):
            ev.ev_set_constants(c.ctx, consts)  # populations are held


def assert_stats(got, want, what):
    for k in ("best_tree", "best_hits", "converged", "best_size", "best_depth", "min_size", "max_size",
              "min_depth", "max_depth"):
        assert got[k] == want[k], f"{what}: {k} {got[k]} != {want[k]}"
    assert same_bits(np.float32(got["best_fitness"]), np.float32(want["best_fitness"])), what
    for k in ("mean_size", "mean_depth"):
        assert got[k] == pytest.approx(want[k], rel=1e-12), f"{what}: {k}"
    # a mean of float32 values summed in double in another order
    assert got["mean_fitness"] == pytest.approx(want["mean_fitness"], rel=1e-9, nan_ok=True), f"{what}: mean_fitness"


def test_population_4000_generations_with_statistics(ev):
    # Table 1's population of 4000 trees with tournaments of 7: every
    # generation's trees, fitness and hits equal the oracle's, and so do the
    # per-generation statistics the paper reports (Sec. 4: best error, its
    # hits, convergence on the best fitness, sizes and depths).
    x, y = workloads.cases(48)
    buf, off = workloads.rhh_population(workloads.SEED_BASE + 7, 4000, 2, 6)
    seed, gens, cap = 4000, 12, 15_000_000
    with ev.Context(x, y) as c:
        pop = c.load(buf, off)
        fit, _, hits = c.eval(pop, hits=True)
        wfit, wpc = oracle.eval_population(buf, off, x, y, threads=8, per_case=True)
        assert_same(fit, wfit, "gen 0")
        for g in range(gens + 1):
            st = ev.ev_population_stats(c.ctx, pop, depths=True)
            want = oracle.population_stats(buf, off, wfit, oracle.hits(wpc, y))
            assert_stats(st, want, f"gen {g}")
            assert np.array_equal(st["depths"], want["depths"]), f"gen {g} depths"
            print(f"gen {g}: best {st['best_fitness']:.6g} hits {st['best_hits']} conv {st['converged']} "
                  f"size {st['mean_size']:.1f} depth {st['mean_depth']:.2f}", flush=True)
            if g == gens:
                break
            kids, capped = ev.ev_generation(c.ctx, pop, seed, g, 7, cap)
            wbuf, woff, wcap = oracle.generation(buf, off, wfit, 7, seed, g, cap)
            gbuf, goff = ev.ev_get_trees(c.ctx, kids)
            assert capped == wcap
            assert np.array_equal(goff, woff) and np.array_equal(gbuf, wbuf), f"gen {g} trees"
            fit, _, hits = c.eval(kids, hits=True)
            wfit, wpc = oracle.eval_population(wbuf, woff, x, y, threads=8, per_case=True)
            assert_same(fit, wfit, f"gen {g + 1} fitness")
            assert np.array_equal(hits, oracle.hits(wpc, y)), f"gen {g + 1} hits"
            ev.ev_free_pop(c.ctx, pop)
            pop, buf, off = kids, wbuf, woff
        # statistics without hits, and of a population with NaN fitness
        c.eval(pop)
        assert ev.ev_population_stats(c.ctx, pop)["best_hits"] == -1


def test_population_statistics_of_special_trees(ev):
    # depths of combs, a full tree and a single leaf; with x = inf some
    # trees' errors are inf and others NaN (inf - inf), which rank worst
    xs = np.array([np.inf, 0.5], np.float32)
    ys = np.zeros(2, np.float32)
    trees = [np.array([X], np.uint8), np.array([ADD] * 30 + [X] * 31, np.uint8),
             np.array([MUL, X] * 25 + [X], np.uint8), np.array([SUB, X, X], np.uint8)]
    full = workloads.rhh_population(workloads.SEED_BASE + 1, 10, 6, 6)
    trees.append(full[0][full[1][0]:full[1][1]])
    off = workloads.offsets_from_sizes([t.size for t in trees])
    buf = np.concatenate(trees)
    with ev.Context(xs, ys) as c:
        pop = c.load(buf, off)
        fit, pc, hits = c.eval(pop, per_case=True, hits=True)
        st = ev.ev_population_stats(c.ctx, pop, depths=True)
    want = oracle.population_stats(buf, off, fit, hits)
    assert list(st["depths"]) == [0, 30, 25, 1, 6] == list(want["depths"])
    assert_stats(st, want, "special trees")


def test_generation_with_caller_fitness(ev):
    # ev_generation's tournaments over a caller-given device fitness vector:
    # the same children as the oracle's generation over that vector.
    import torch

    x, y = workloads.cases(48)
    buf, off = workloads.rhh_population(workloads.SEED_BASE + 6, 48, 2, 6)
    seed, cap = 77, 15_000_000
    with ev.Context(x, y) as c:
        pop = c.load(buf, off)
        fit, _ = c.eval(pop)
        # the stored fitness and the same values passed in give one result
        a, _ = ev.ev_generation(c.ctx, pop, seed, 0, 2, cap)
        fit_dev = torch.from_numpy(fit).cuda()
        torch.cuda.synchronize()
        b, _ = ev.ev_generation(c.ctx, pop, seed, 0, 2, cap, fitness=fit_dev)
        ab, ao = ev.ev_get_trees(c.ctx, a)
        bb, bo = ev.ev_get_trees(c.ctx, b)
        assert np.array_equal(ao, bo) and np.array_equal(ab, bb)
        # another fitness vector (ranks reversed) selects other parents
        other = (-fit).astype(np.float32)
        other_dev = torch.from_numpy(other).cuda()
        torch.cuda.synchronize()
        k, capped = ev.ev_generation(c.ctx, pop, seed, 0, 2, cap, fitness=other_dev)
        kb, ko = ev.ev_get_trees(c.ctx, k)
    wbuf, woff, wcap = oracle.generation(buf, off, other, 2, seed, 0, cap)
    assert capped == wcap
    assert np.array_equal(ko, woff) and np.array_equal(kb, wbuf)
    assert not (np.array_equal(ko, ao) and np.array_equal(kb, ab))


def test_device_pointer_load_and_device_outputs(ev):
    # ev_load_trees with EV_DEVICE_PTR (bytes and offsets in device memory,
    # here torch tensors) and ev_eval_fitness with EV_OUT_DEVICE (fitness,
    # per-case values and hits written to device tensors): the same results
    # as the oracle, and the same as the host-pointer forms.
    import torch

    x, y = workloads.cases(48)
    sizes = workloads.loguniform_sizes(45, 300, 1, 30000)
    buf, off = workloads.random_population(45, sizes)
    want_fit, want_pc = oracle.eval_population(buf, off, x, y, threads=8, per_case=True)
    M = off.size - 1
    with ev.Context(x, y) as c:
        dbuf = torch.from_numpy(buf).cuda()
        doff = torch.from_numpy(off.view(np.int64)).cuda()
        torch.cuda.synchronize()
        pop = ev.ev_load_trees(c.ctx, dbuf, doff)
        del dbuf, doff
        gbuf, goff = ev.ev_get_trees(c.ctx, pop)
        assert np.array_equal(gbuf, buf) and np.array_equal(goff, off)
        fit = torch.full((M,), -1.0, dtype=torch.float32, device="cuda")
        pc = torch.full((M, 48), -1.0, dtype=torch.float32, device="cuda")
        hits = torch.full((M,), -1, dtype=torch.int32, device="cuda")
        for _ in range(2):  # the second call reuses the cached result slots
            ev.ev_eval_fitness(c.ctx, pop, 0, out=fit, out_per_case=pc, out_hits=hits)
            torch.cuda.synchronize()
            assert_same(fit.cpu().numpy(), want_fit, "device fitness")
            assert_same(pc.cpu().numpy(), want_pc, "device per-case")
            assert np.array_equal(hits.cpu().numpy(), oracle.hits(want_pc, y))
        hf, hpc = c.eval(pop, per_case=True)
        assert_same(hf, want_fit, "host fitness")
        assert_same(hpc, want_pc, "host per-case")
        # a malformed tree in device memory is refused like a host one
        bad = buf.copy()
        bad[int(off[7])] = 9
        dbad, doff = torch.from_numpy(bad).cuda(), torch.from_numpy(off.view(np.int64)).cuda()
        torch.cuda.synchronize()
        with pytest.raises(ev.EvError) as e:
            ev.ev_load_trees(c.ctx, dbad, doff)
        assert e.value.code == ev.EV_EMALFORMED and e.value.bad_tree == 7


def test_deferred_validation_verdict(ev):
    # The children of ev_generation leave their last plan level's validation
    # verdict to the device and to their first evaluation.  A verdict forced
    # to fail from the host (test hook) makes that evaluation fail with
    # EV_EDEVICE, every time, while a plan built by ev_load_trees is refused
    # at once; with the hook off, the same children evaluate as the oracle.
    x, y = workloads.cases(48)
    sizes = workloads.loguniform_sizes(43, 60, 10, 20000)
    buf, off = workloads.random_population(43, sizes)
    seed, cap = 99, 15_000_000
    with ev.Context(x, y) as c:
        pop = c.load(buf, off)
        fit, _ = c.eval(pop)
        good, _ = ev.ev_generation(c.ctx, pop, seed, 0, 2, cap)
        gfit, _ = c.eval(good)
        gbuf, goff = ev.ev_get_trees(c.ctx, good)
        assert same_bits(gfit, oracle.eval_population(gbuf, goff, x, y, threads=8)).all()
        assert same_bits(c.eval(good)[0], gfit).all()

        ev.ev_set_tuning(c.ctx, flags=ev.EV_TUNE_TEST_FAIL_CHECK)
        bad, _ = ev.ev_generation(c.ctx, pop, seed, 0, 2, cap)
        bbuf, boff = ev.ev_get_trees(c.ctx, bad)
        assert np.array_equal(bbuf, gbuf) and np.array_equal(boff, goff)
        for _ in range(2):
            with pytest.raises(ev.EvError) as e:
                c.eval(bad)
            assert e.value.code == ev.EV_EDEVICE and "malformed code stream" in str(e.value)
        with pytest.raises(ev.EvError) as e:
            c.load(buf, off)
        assert e.value.code == ev.EV_EDEVICE
        # parents and earlier children are untouched
        assert same_bits(c.eval(pop)[0], fit).all()
        assert same_bits(c.eval(good)[0], gfit).all()

        ev.ev_set_tuning(c.ctx, flags=0)
        again, _ = ev.ev_generation(c.ctx, pop, seed, 0, 2, cap)
        assert same_bits(c.eval(again)[0], gfit).all()
        for q in (bad, good, again):
            ev.ev_free_pop(c.ctx, q)


def test_caller_allocator(ev):
    # Every device block of a context can come from the caller's allocator
    # (here torch's caching allocator); results are the same, and every block
    # goes back by the time the context is destroyed.
    import torch

    x, y = workloads.cases(48)
    sizes = workloads.loguniform_sizes(41, 200, 10, 50000)
    buf, off = workloads.random_population(41, sizes)
    calls = {"alloc": 0, "free": 0, "live": set()}

    def alloc(nbytes, _user):
        p = torch.cuda.caching_allocator_alloc(int(nbytes), 0)
        calls["alloc"] += 1
        calls["live"].add(p)
        return p

    def free(ptr, _user):
        calls["free"] += 1
        calls["live"].discard(ptr)
        torch.cuda.caching_allocator_delete(ptr)

    a = ev.ev_allocator(ev._ALLOC_FN(alloc), ev._FREE_FN(free), None)
    with ev.Context(x, y) as c0:
        pop = c0.load(buf, off)
        want, wpc = c0.eval(pop, per_case=True)
        k0, _ = ev.ev_generation(c0.ctx, pop, 5, 1, 2, 10**7)
        wk, _ = c0.eval(k0)
    with ev.Context(x, y, allocator=a) as c:
        pop = c.load(buf, off)
        got, gpc = c.eval(pop, per_case=True)
        k, _ = ev.ev_generation(c.ctx, pop, 5, 1, 2, 10**7)
        gk, _ = c.eval(k)
    assert calls["alloc"] > 0
    assert calls["free"] == calls["alloc"] and not calls["live"]
    assert_same(got, want, "fitness")
    assert_same(gpc, wpc, "per-case")
    assert_same(gk, wk, "children's fitness")


def test_generation_loop_1000_generations(ev):
    # The full generational loop on the device: population 48, ramped
    # half-and-half start, size-2 tournaments, Philox points, 15e6-node cap,
    # 1000 generations.  Every generation's trees and fitness are compared
    # with the oracle's, bit for bit.
    x, y = workloads.cases(48)
    buf, off = workloads.rhh_population(workloads.SEED_BASE + 4, 48, 2, 6)
    seed, gens, cap = 0x5EED0004, 1000, 15_000_000
    threads = min(os.cpu_count() or 1, 16)
    with ev.Context(x, y) as c:
        pop = c.load(buf, off)
        fit, _ = c.eval(pop)
        wfit = oracle.eval_population(buf, off, x, y, threads=threads)
        assert_same(fit, wfit, "gen 0")
        for g in range(gens):
            kids, capped = ev.ev_generation(c.ctx, pop, seed, g, 2, cap)
            wbuf, woff, wcap = oracle.generation(buf, off, wfit, 2, seed, g, cap)
            gbuf, goff = ev.ev_get_trees(c.ctx, kids)
            assert capped == wcap, f"gen {g} capped"
            assert np.array_equal(goff, woff), f"gen {g} offsets"
            assert np.array_equal(gbuf, wbuf), f"gen {g} trees"
            fit, _ = c.eval(kids)
            wfit = oracle.eval_population(wbuf, woff, x, y, threads=threads)
            assert_same(fit, wfit, f"gen {g + 1} fitness")
            ev.ev_free_pop(c.ctx, pop)
            pop, buf, off = kids, wbuf, woff
            if g % 100 == 99:
                print(f"generation {g + 1}: mean size {np.diff(off).mean():.0f}, best {np.nanmin(wfit):.6g}",
                      flush=True)


def test_autotune_keeps_results(ev):
    x, y = workloads.cases(48)
    sizes = workloads.loguniform_sizes(53, 500, 10, 1e5)
    buf, off = workloads.random_population(53, sizes)
    with ev.Context(x, y) as c:
        pop = c.load(buf, off)
        fit0, pc0 = c.eval(pop, per_case=True)
        chunk, ms = ev.ev_autotune(c.ctx, pop, 0, 3)
        assert chunk in (1024, 2048, 4096, 6144, 8192, 12288, 16384, 32768) and ms > 0
        fit1, pc1 = c.eval(pop, per_case=True)
        pop2 = c.load(buf, off)  # planned with the tuned size
        fit2, _ = c.eval(pop2)
        # the full search (sizes at both levels, waves per CU), then the cache
        t = ev.ev_autotune_ex(c.ctx, pop, 0, 2, ev.EV_AUTOTUNE_NO_CACHE)
        assert t["from_cache"] == 0 and t["ms"] > 0 and t["chunk"] >= 1024
        assert t["chunk_hi"] in (0, t["chunk"], 4 * t["chunk"])
        fit3, pc3 = c.eval(pop, per_case=True)
        again = ev.ev_autotune_ex(c.ctx, pop2, 0, 2)
        assert again["from_cache"] == 1
        assert (again["chunk"], again["chunk_hi"], again["waves_per_cu"]) == (t["chunk"], t["chunk_hi"],
                                                                             t["waves_per_cu"])
        fit4, pc4 = c.eval(pop2, per_case=True)
        # children planned and evaluated with the tuned grid
        ev.ev_set_tuning(c.ctx, 4096)
        k, _ = ev.ev_generation(c.ctx, pop, 7, 0, 2, 10**7)
        fk, _ = c.eval(k)
        kb, ko = ev.ev_get_trees(c.ctx, k)
    assert_same(fit0, fit1, "fitness after autotune")
    assert_same(pc0, pc1, "per-case after autotune")
    assert_same(fit0, fit2, "fitness of a population planned with the tuned size")
    assert_same(pc0, pc3, "per-case after the full search")
    assert_same(pc0, pc4, "per-case with the cached choice")
    assert_same(fk, oracle.eval_population(kb, ko, x, y, threads=8), "children after tuning")


def test_serving_results_same_alone_and_mixed(ev):
    x, y = workloads.cases(48)
    x2, y2 = workloads.cases(1024)
    rng = np.random.default_rng(41)
    jobs = []
    for k in range(24):
        sizes = workloads.loguniform_sizes(100 + k, int(rng.integers(1, 20)), 1, 50000)
        b, o = workloads.random_population(100 + k, sizes)
        jobs.append((b, o, int(k % 3 == 0)))
    with ev.Context(x, y) as c:
        t1 = c.add_cases(x2, y2)
        assert t1 == 1
        alone = []
        for b, o, tab in jobs:
            t = ev.ev_submit_eval(c.ctx, b, o, tab)
            assert ev.ev_wait(c.ctx, t) == 0
            alone.append(ev.ev_result(c.ctx, t, o.size - 1, c.n_cases(tab), per_case=True))
        tickets = [ev.ev_submit_eval(c.ctx, b, o, tab) for b, o, tab in jobs]
        mixed = []
        for t, (b, o, tab) in zip(tickets, jobs):
            assert ev.ev_wait(c.ctx, t) == 0
            mixed.append(ev.ev_result(c.ctx, t, o.size - 1, c.n_cases(tab), per_case=True))
    for k, ((fa, pa), (fm, pm), (b, o, tab)) in enumerate(zip(alone, mixed, jobs)):
        assert_same(fa, fm, f"job {k} fitness alone vs mixed")
        assert_same(pa, pm, f"job {k} per-case alone vs mixed")
        xs, ys = (x2, y2) if tab else (x, y)
        wf = oracle.eval_population(b, o, xs, ys, threads=8)
        assert_same(fa, wf, f"job {k} vs oracle")


def test_serving_malformed_request_fails_alone(ev):
    # trees are checked on the device when their batch is planned: requests
    # holding a tree that is not a valid prefix tree end with EV_EMALFORMED,
    # and the requests queued (and possibly batched) with them still get
    # the oracle's results
    x, y = workloads.cases(48)
    sizes = workloads.loguniform_sizes(61, 40, 1, 20000)
    b, o = workloads.random_population(61, sizes)
    want = oracle.eval_population(b, o, x, y, threads=8)
    bads = [np.array([ADD, X, X, X], np.uint8), np.array([MUL, X], np.uint8), np.array([X, 200], np.uint8)]
    with ev.Context(x, y) as c:
        good, bad = [], []
        for t in range(40):
            good.append(ev.ev_submit_eval(c.ctx, b[o[t]:o[t + 1]], np.array([0, o[t + 1] - o[t]], np.uint64)))
            if t % 13 == 5:
                bb = bads[len(bad)]
                bad.append(ev.ev_submit_eval(c.ctx, bb, np.array([0, bb.size], np.uint64)))
        for t, tk in enumerate(good):
            assert ev.ev_wait(c.ctx, tk) == 0, f"request {t}"
            f, _ = ev.ev_result(c.ctx, tk, 1, 48)
            assert_same(f, want[t:t + 1], f"request {t}")
        for tk in bad:
            assert ev.ev_wait(c.ctx, tk) == ev.EV_EMALFORMED
            with pytest.raises(ev.EvError) as e:
                ev.ev_result(c.ctx, tk, 1, 48)
            assert e.value.code == ev.EV_EMALFORMED


def test_serving_under_load(ev):
    # 600 requests queued at once on two case tables: single trees of up to
    # 4e6 nodes drawn from a pool (so batches of a few hundred trees, with
    # repeats) and crossover requests; every served result must equal the
    # direct evaluation of the same tree, bit for bit.
    x, y = workloads.cases(48)
    x2, y2 = workloads.cases(1024)
    rng = np.random.default_rng(47)
    psizes = workloads.loguniform_sizes(47, 48, 10, 4e6)
    pbuf, poff = workloads.random_population(47, psizes)
    qsizes = workloads.loguniform_sizes(48, 32, 1, 5000)
    qbuf, qoff = workloads.random_population(48, qsizes)
    with ev.Context(x, y) as c:
        t1 = c.add_cases(x2, y2)
        pool = c.load(pbuf, poff)
        direct = [c.eval(pool, 0)[0], c.eval(pool, t1)[0]]
        parents = c.load(qbuf, qoff)
        reqs, tickets = [], []
        for _ in range(600):
            tab = int(rng.integers(0, 2))
            if rng.random() < 0.8:
                t = int(rng.integers(0, psizes.size))
                reqs.append(("eval", tab, t))
                tickets.append(ev.ev_submit_eval(c.ctx, pbuf[poff[t]:poff[t + 1]],
                                                 np.array([0, psizes[t]], np.uint64), tab))
            else:
                mum = rng.integers(0, 32, 4).astype(np.int32)
                dad = rng.integers(0, 32, 4).astype(np.int32)
                p = np.array([rng.integers(0, qsizes[m]) for m in mum], np.uint64)
                q = np.array([rng.integers(0, qsizes[d]) for d in dad], np.uint64)
                reqs.append(("xo", tab, (mum, dad, p, q)))
                tickets.append(ev.ev_submit_crossover(c.ctx, parents, mum, dad, p, q, tab))
        got = []
        for t, r in zip(tickets, reqs):
            assert ev.ev_wait(c.ctx, t) == 0, f"request {r[:2]} failed"
            got.append(ev.ev_result(c.ctx, t, 4, c.n_cases(r[1]))[0])
    cases = [(x, y), (x2, y2)]
    for k, (r, f) in enumerate(zip(reqs, got)):
        if r[0] == "eval":
            assert_same(f, direct[r[1]][r[2]:r[2] + 1], f"request {k} (tree {r[2]}, table {r[1]})")
        else:
            mum, dad, p, q = r[2]
            kids = [oracle.crossover(qbuf[qoff[m]:qoff[m + 1]], qbuf[qoff[d]:qoff[d + 1]], int(pp), int(qq))
                    for m, d, pp, qq in zip(mum, dad, p, q)]
            koff = workloads.offsets_from_sizes([kk.size for kk in kids])
            want = oracle.eval_population(np.concatenate(kids), koff, *cases[r[1]])
            assert_same(f, want, f"request {k} (crossover, table {r[1]})")


def test_serving_crossover_jobs(ev):
    x, y = workloads.cases(48)
    rng = np.random.default_rng(43)
    sizes = workloads.loguniform_sizes(43, 32, 1, 5000)
    buf, off = workloads.random_population(43, sizes)
    with ev.Context(x, y) as c:
        pop = c.load(buf, off)
        n = 20
        mum = rng.integers(0, 32, n).astype(np.int32)
        dad = rng.integers(0, 32, n).astype(np.int32)
        p = np.array([rng.integers(0, sizes[m]) for m in mum], np.uint64)
        q = np.array([rng.integers(0, sizes[d]) for d in dad], np.uint64)
        t = ev.ev_submit_crossover(c.ctx, pop, mum, dad, p, q)
        assert ev.ev_wait(c.ctx, t) == 0
        fit, _ = ev.ev_result(c.ctx, t, n, 48)
    kids = [oracle.crossover(buf[off[m]:off[m + 1]], buf[off[d]:off[d + 1]], int(pp), int(qq))
            for m, d, pp, qq in zip(mum, dad, p, q)]
    koff = workloads.offsets_from_sizes([k.size for k in kids])
    wf = oracle.eval_population(np.concatenate(kids), koff, x, y)
    assert_same(fit, wf, "served crossover")


def test_serving_parents_freed_while_jobs_run(ev):
    # Crossover jobs read a resident population on the workers' streams; the
    # caller frees it right after submitting.  Jobs that had started finish
    # with the oracle's results (the population lives until the last one is
    # done); jobs that had not are refused with EV_ENOTFOUND.  Evaluation
    # jobs submitted beside them are unaffected.
    x, y = workloads.cases(48)
    rng = np.random.default_rng(53)
    sizes = workloads.loguniform_sizes(53, 64, 1, 200000)
    buf, off = workloads.random_population(53, sizes)
    esizes = workloads.loguniform_sizes(54, 40, 10, 300000)
    ebuf, eoff = workloads.random_population(54, esizes)
    want_e = oracle.eval_population(ebuf, eoff, x, y, threads=8)
    with ev.Context(x, y) as c:
        for rep in range(3):
            pop = c.load(buf, off)
            jobs, evals = [], []
            for k in range(24):
                mum = rng.integers(0, 64, 4).astype(np.int32)
                dad = rng.integers(0, 64, 4).astype(np.int32)
                p = np.array([rng.integers(0, sizes[m]) for m in mum], np.uint64)
                q = np.array([rng.integers(0, sizes[d]) for d in dad], np.uint64)
                jobs.append(((mum, dad, p, q), ev.ev_submit_crossover(c.ctx, pop, mum, dad, p, q)))
                t = int(rng.integers(0, 40))
                evals.append((t, ev.ev_submit_eval(c.ctx, ebuf[eoff[t]:eoff[t + 1]],
                                                   np.array([0, esizes[t]], np.uint64))))
            ev.ev_free_pop(c.ctx, pop)
            done = 0
            for (mum, dad, p, q), tk in jobs:
                st = ev.ev_wait(c.ctx, tk)
                if st == ev.EV_ENOTFOUND:
                    with pytest.raises(ev.EvError):
                        ev.ev_result(c.ctx, tk, 4, 48)
                    continue
                assert st == 0, st
                f, _ = ev.ev_result(c.ctx, tk, 4, 48)
                kids = [oracle.crossover(buf[off[m]:off[m + 1]], buf[off[d]:off[d + 1]], int(pp), int(qq))
                        for m, d, pp, qq in zip(mum, dad, p, q)]
                koff = workloads.offsets_from_sizes([kk.size for kk in kids])
                assert_same(f, oracle.eval_population(np.concatenate(kids), koff, x, y), f"rep {rep} crossover")
                done += 1
            for t, tk in evals:
                assert ev.ev_wait(c.ctx, tk) == 0
                f, _ = ev.ev_result(c.ctx, tk, 1, 48)
                assert_same(f, want_e[t:t + 1], f"rep {rep} eval of tree {t}")
            print(f"rep {rep}: {done} of {len(jobs)} crossover jobs ran", flush=True)


def oracle_in_background(buf, off, x, y, threads=None):
    """Start the oracle's evaluation of a population on every host core in a
    thread (the C call releases the interpreter lock), so that it overlaps the
    device work; returns a function that waits for (fitness, per_case)."""
    import threading

    threads = threads or max(1, len(os.sched_getaffinity(0)))
    out = {}

    def work():
        try:
            out["r"] = oracle.eval_population(buf, off, x, y, threads=threads, per_case=True)
        except BaseException as e:  # noqa: BLE001 - re-raised in the waiting thread
            out["e"] = e

    th = threading.Thread(target=work, daemon=True)
    th.start()

    def wait():
        th.join()
        if "e" in out:
            raise out["e"]
        return out["r"]

    return wait


@pytest.mark.timeout(600)
def test_giant_population_all_trees(ev):
    # 48 random trees with log-uniform sizes in [1e6, 4e8] (about 4.4e9
    # nodes), evaluated in the benchmark's launch configuration; every tree's
    # per-case values and fitness against the oracle, bit for bit.
    buf, off, n = workloads.workload("giant")
    x, y = workloads.cases(n)
    sizes = np.diff(off)
    print(f"giant: {int(off[-1])} nodes, largest {int(sizes.max())}", flush=True)
    want = oracle_in_background(buf, off, x, y)
    with ev.Context(x, y) as c:
        pop = c.load(buf, off)
        info = ev.ev_get_plan_info(c.ctx, pop)
        fit, pc, hits = c.eval(pop, per_case=True, hits=True)
    print(f"giant plan {info}", flush=True)
    want_fit, want_pc = want()
    assert_same(pc, want_pc, "giant per-case")
    assert_same(fit, want_fit, "giant fitness")
    assert np.array_equal(hits, oracle.hits(want_pc, y))


@pytest.fixture(scope="module")
def giant_max():
    buf, off, n = workloads.workload("giant_max")
    x, y = workloads.cases(n)
    return buf, off, x, y


@pytest.mark.timeout(900)
def test_giant_max_population_all_trees(ev, giant_max):
    # 48 random trees of 4e8 nodes (19.2e9 nodes, the 20 GB population),
    # evaluated whole in the benchmark's launch configuration; all 48 trees
    # against the oracle, bit for bit.
    buf, off, x, y = giant_max
    print(f"giant_max: {int(off[-1])} nodes", flush=True)
    want = oracle_in_background(buf, off, x, y)
    with ev.Context(x, y) as c:
        pop = c.load(buf, off)
        info = ev.ev_get_plan_info(c.ctx, pop)
        fit, pc = c.eval(pop, per_case=True)
    print(f"giant_max plan {info}", flush=True)
    want_fit, want_pc = want()
    assert_same(pc, want_pc, "giant_max per-case")
    assert_same(fit, want_fit, "giant_max fitness")


@pytest.mark.timeout(600)
def test_giant_max_crossover_matches_oracle(ev, giant_max):
    # Children of 4e8-node parents (64-bit child offsets, multi-GB children,
    # subtree ends found by scans over long subtrees): the children's bytes
    # against the oracle's crossover, then their evaluation against the
    # oracle.  Points include the roots (p = 0: the child is the dad's
    # subtree; q = 0: the whole dad is inserted) and points with long
    # subtrees (the first few nodes, whose subtrees span most of the tree).
    buf, off, x, y = giant_max
    sizes = np.diff(off).astype(np.int64)
    rng = np.random.default_rng(2024)
    mum = np.array([0, 5, 47, 12, 30], np.int32)
    dad = np.array([47, 5, 1, 33, 30], np.int32)
    p = np.array([0, 1, int(rng.integers(0, sizes[47])), 2, int(rng.integers(0, sizes[30]))], np.uint64)
    q = np.array([3, 0, int(rng.integers(0, sizes[1])), 1, 2], np.uint64)
    want_kids = [oracle.crossover(buf[off[m]:off[m + 1]], buf[off[d]:off[d + 1]], int(pp), int(qq))
                 for m, d, pp, qq in zip(mum, dad, p, q)]
    print("giant_max crossover: child sizes", [k.size for k in want_kids], flush=True)
    koff = workloads.offsets_from_sizes([k.size for k in want_kids])
    kbuf = np.concatenate(want_kids)
    want = oracle_in_background(kbuf, koff, x, y)
    with ev.Context(x, y) as c:
        pop = c.load(buf, off)
        kids, capped = ev.ev_crossover(c.ctx, pop, pop, mum, dad, p, q)
        assert capped == 0
        got_buf, got_off = ev.ev_get_trees(c.ctx, kids)
        assert np.array_equal(got_off, koff)
        assert np.array_equal(got_buf, kbuf)
        del got_buf
        fit, pc = c.eval(kids, per_case=True)
    want_fit, want_pc = want()
    assert_same(pc, want_pc, "giant_max children per-case")
    assert_same(fit, want_fit, "giant_max children fitness")


def test_single_tree_populations(ev):
    # every tree alone as its own population: each plan stands on its own
    # (a lone tree whose stack only reaches the window's upper quarter still
    # needs its spill slab)
    buf, off, n = workloads.workload("batched")
    x, y = workloads.cases(n)
    sizes = np.diff(off)
    pick = [int(t) for t in np.argsort(sizes)[::37][:120]] + [55, 57, 150, 155]
    parts = [buf[off[t]:off[t + 1]] for t in pick]
    want = oracle.eval_population(np.concatenate(parts), workloads.offsets_from_sizes([p.size for p in parts]), x, y,
                                  threads=8)
    with ev.Context(x, y) as c:
        for i, p in enumerate(parts):
            pop = c.load(np.ascontiguousarray(p), np.array([0, p.size], np.uint64))
            f, _ = c.eval(pop)
            assert_same(f, want[i:i + 1], f"tree {pick[i]} alone")
            ev.ev_free_pop(c.ctx, pop)
