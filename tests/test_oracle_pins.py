"""Pins of the C oracle against facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: binary64
arithmetic rounded once (correctly rounded for + - * / on binary32 because
53 >= 2*24+2, Figueroa 1995), an independent recursive evaluator written
here, closed forms, summation-order adversaries, brute force on tiny trees,
and published Philox known answers.
"""
import itertools
import os

import numpy as np
import pytest

import oracle
import workloads

HERE = os.path.dirname(os.path.abspath(__file__))
ADD, SUB, MUL, DIV, X = 0, 1, 2, 3, 4
SYM = {"+": ADD, "-": SUB, "*": MUL, "/": DIV, "x": X}


def same_bits(a, b):
    """Equal bit patterns, or both NaN (NaN payloads differ across ISAs)."""
    a = np.asarray(a, np.float32)
    b = np.asarray(b, np.float32)
    return (a.view(np.uint32) == b.view(np.uint32)) | (np.isnan(a) & np.isnan(b))


# ------------------------------------------------ independent reference

def ref_op(op, a, b):
    """binary64 compute, one rounding to binary32 (= correctly rounded)."""
    a64 = np.asarray(a, np.float32).astype(np.float64)
    b64 = np.asarray(b, np.float32).astype(np.float64)
    with np.errstate(all="ignore"):
        if op == ADD:
            r = a64 + b64
        elif op == SUB:
            r = a64 - b64
        elif op == MUL:
            r = a64 * b64
        else:
            r = np.where(b64 != 0.0, a64 / np.where(b64 != 0.0, b64, 1.0), 1.0)
        return r.astype(np.float32)


def ref_eval(tree, x):
    """Recursive evaluation of a prefix tree (first argument evaluated first)."""
    x = np.asarray(x, np.float32)

    def ev(i):
        t = tree[i]
        if t == X:
            return x.copy(), i + 1
        a, j = ev(i + 1)
        b, k = ev(j)
        return ref_op(t, a, b), k

    v, end = ev(0)
    assert end == len(tree)
    return v


def parse(expr: str) -> np.ndarray:
    return np.array([SYM[s] for s in expr.split()], np.uint8)


def special_values():
    f = np.float32
    vals = [0.0, -0.0, 1.0, -1.0, 0.5, 2.0, 3.0, 1e-45, -1e-45, 1e-40, 1.17549435e-38, 3.4028235e38,
            -3.4028235e38, np.inf, -np.inf, np.nan, 1.0000001, 0.99999994, 1e-20, 1e20, 7.0, 0.1]
    return np.array(vals, np.float32)


def operand_pairs(rng, n):
    sp = special_values()
    a = np.concatenate([np.repeat(sp, sp.size), rng.standard_normal(n).astype(np.float32),
                        (rng.standard_normal(n) * 1e30).astype(np.float32),
                        rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32).view(np.float32)])
    b = np.concatenate([np.tile(sp, sp.size), rng.standard_normal(n).astype(np.float32),
                        (rng.standard_normal(n) * 1e-30).astype(np.float32),
                        rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32).view(np.float32)])
    return a, b


# ------------------------------------------------------------ per-op pins

@pytest.mark.parametrize("op", [ADD, SUB, MUL, DIV])
def test_op_is_correctly_rounded(op):
    rng = np.random.default_rng(100 + op)
    a, b = operand_pairs(rng, 3000)
    got = np.array([oracle.op(op, float(u), float(v)) for u, v in zip(a, b)], np.float32)
    want = ref_op(op, a, b)
    bad = ~same_bits(got, want)
    assert not bad.any(), list(zip(a[bad][:5], b[bad][:5], got[bad][:5], want[bad][:5]))


def test_protected_division_rule():
    # (y != 0) ? x/y : 1.0f (Table 1 footnote): -0 counts as zero, NaN does not
    assert oracle.op(DIV, 5.0, 0.0) == 1.0
    assert oracle.op(DIV, 5.0, -0.0) == 1.0
    assert oracle.op(DIV, float("nan"), 0.0) == 1.0
    assert np.isnan(oracle.op(DIV, 5.0, float("nan")))
    assert oracle.op(DIV, 5.0, float("inf")) == 0.0


# ------------------------------------------------------ tree evaluation

def all_trees(n_nodes):
    """Every prefix tree with exactly n_nodes nodes (n odd)."""
    if n_nodes == 1:
        yield [X]
        return
    for left in range(1, n_nodes - 1, 2):
        right = n_nodes - 1 - left
        for lt in all_trees(left):
            for rt in all_trees(right):
                for op in (ADD, SUB, MUL, DIV):
                    yield [op] + lt + rt


def test_exhaustive_trees_up_to_7_nodes():
    trees = [t for n in (1, 3, 5, 7) for t in all_trees(n)]
    assert len(trees) == 1 + 4 + 32 + 320
    x48, _ = workloads.cases(48)
    xs = np.concatenate([x48, special_values()])
    for t in trees:
        tree = np.array(t, np.uint8)
        got = oracle.eval_cases(tree, xs)
        want = ref_eval(t, xs)
        assert same_bits(got, want).all(), (t, got, want)


def test_random_trees_against_recursive_reference():
    rng = np.random.default_rng(7)
    x48, _ = workloads.cases(48)
    xs = np.concatenate([x48, (rng.standard_normal(16) * 10).astype(np.float32), special_values()])
    for k in range(400):
        n = int(rng.integers(0, 32)) * 2 + 1
        tree = workloads.random_tree(11, k, n)
        got = oracle.eval_cases(tree, xs)
        want = ref_eval(list(tree), xs)
        assert same_bits(got, want).all(), (k, n)


def test_deep_tree_within_fp64_error_bound():
    # A long random tree evaluated in binary32 stays within the forward error
    # bound of its binary64 evaluation wherever the binary64 value is modest.
    x = np.linspace(-0.9, 0.9, 48).astype(np.float32)
    tree = parse("* + x / x x - x * x x")  # x*(x+1)... exact small polynomial-ish tree
    got = oracle.eval_cases(tree, x).astype(np.float64)
    xd = x.astype(np.float64)
    exact = (xd + 1.0) * (xd - xd * xd)
    # 4 operations, each within 2^-24 relative: |err| <= ~4u * sum of magnitudes
    u = 2.0 ** -24
    bound = 6 * u * ((np.abs(xd) + 1) * (np.abs(xd) + xd * xd)) + 1e-30
    assert np.all(np.abs(got - exact) <= bound)


# ----------------------------------------------------------- closed forms

def test_t_minus_t_is_zero():
    rng = np.random.default_rng(3)
    x48, _ = workloads.cases(48)
    for k in range(50):
        sub = workloads.random_tree(5, k, int(rng.integers(1, 40)) * 2 + 1)
        tree = np.concatenate([[SUB], sub, sub]).astype(np.uint8)
        t_val = oracle.eval_cases(sub, x48)
        got = oracle.eval_cases(tree, x48)
        fin = np.isfinite(t_val)
        assert np.all(got[fin] == 0.0) and not np.signbit(got[fin]).any()
        assert np.all(np.isnan(got[~fin]))


def test_x_over_x_is_one_and_zero_divisor_gives_one():
    x48, _ = workloads.cases(48)
    assert np.all(x48 != 0)  # 48 evenly spaced points never hit 0
    assert np.all(oracle.eval_cases(parse("/ x x"), x48) == 1.0)
    rng = np.random.default_rng(4)
    for k in range(30):
        num = workloads.random_tree(6, k, int(rng.integers(0, 30)) * 2 + 1)
        tree = np.concatenate([[DIV], num, parse("- x x")]).astype(np.uint8)
        assert np.all(oracle.eval_cases(tree, x48) == 1.0)


def test_operand_order_of_sub_and_div():
    x = np.linspace(-1, 1, 48).astype(np.float32)
    got = oracle.eval_cases(parse("- x * x x"), x)
    assert same_bits(got, x - x * x).all()
    got = oracle.eval_cases(parse("/ x + x x"), x)
    assert np.all(got == 0.5)


def test_constant_tree_fitness_is_mean_abs_target():
    x, y = workloads.cases(48)
    out = oracle.eval_cases(parse("- x x"), x)
    assert np.all(out == 0.0)
    fit = float(oracle.fitness(out, y))
    exact = float(np.abs(y.astype(np.float64)).sum() / 48)
    assert abs(fit - exact) <= 48 * 2.0 ** -24 * exact


def load_sextic():
    trees = {}
    for line in open(os.path.join(HERE, "golden", "sextic_trees.txt")):
        if line.startswith("#") or not line.strip():
            continue
        name, expr = line.split(":", 1)
        trees[name.strip()] = parse(expr)
    return trees


def test_exact_sextic_trees():
    trees = load_sextic()
    x, y = workloads.cases(48)
    xd = x.astype(np.float64)
    y64 = xd ** 6 - 2 * xd ** 4 + xd ** 2
    one = np.float32(1)
    # the same tree evaluated by numpy binary32 in the tree's own order
    f_fact = ((x * x) * ((x - one) * (x - one))) * ((x + one) * (x + one))
    x2 = x * x
    f_exp = (x2 * (x2 * x2)) - (((x2 * x2) + (x2 * x2)) - x2)
    for name, same_order, bound in (("factored", f_fact, 2e-7), ("expanded", f_exp, 1e-6)):
        tree = trees[name]
        ok, _ = oracle.validate(tree)
        assert ok
        out = oracle.eval_cases(tree, x)
        assert same_bits(out, same_order).all(), name
        # table computed in binary32 in the same order -> MAE exactly 0
        assert oracle.fitness(out, same_order) == 0.0
        # against the binary64 target: tiny error
        assert float(oracle.fitness(out, y)) <= bound
        assert np.max(np.abs(out.astype(np.float64) - y64)) <= 4 * bound


def test_hits_closed_forms():
    # Sec. 3.2: a hit is a case within 0.01 of the target (reading S18:
    # |out - y| <= 0.01f on the fitness's own binary32 error term).
    x, y = workloads.cases(48)
    zero = oracle.eval_cases(parse("- x x"), x)
    want = int(np.count_nonzero(np.abs(y) <= np.float32(0.01)))
    assert oracle.hits(zero[None, :], y)[0] == want
    assert 0 < want < 48  # the constant 0 is close to the target only near x = 0 and x = +-1
    # both exact Sextic trees are solutions: 48 hits (Sec. 4: "48 out of 48")
    for name, tree in load_sextic().items():
        out = oracle.eval_cases(tree, x)
        assert oracle.hits(out[None, :], y)[0] == 48, name
    # the boundary is inclusive; NaN is never a hit
    t = np.zeros(3, np.float32)
    edge = np.array([[0.01, np.nextafter(np.float32(0.01), np.float32(1)), np.nan]], np.float32)
    assert oracle.hits(edge, t)[0] == 1
    assert oracle.hits(-edge, t)[0] == 1


def test_fitness_sums_in_ascending_order():
    # e = |0 - y| with y = [1e8, 1, 1, ...]: ascending binary32 sum stays 1e8
    # (each +1 rounds away), a reversed sum would reach 1e8 + 48.
    y = np.ones(48, np.float32)
    y[0] = 1e8
    out = np.zeros(48, np.float32)
    got = oracle.fitness(out, y)
    assert got == np.float32(1e8) / np.float32(48)
    assert got != np.float32(100000048.0) / np.float32(48)


# ------------------------------------------------------------- validation

def test_validation_and_stack_invariants():
    rng = np.random.default_rng(9)
    for k in range(200):
        n = int(rng.integers(0, 200)) * 2 + 1
        t = workloads.random_tree(9, k, n)
        ok, ms = oracle.validate(t)
        assert ok and t.size % 2 == 1
        assert np.sum(t == X) == np.sum(t != X) + 1
        # right-to-left height: +1 per leaf, -1 per function
        h = np.cumsum(np.where(t[::-1] == X, 1, -1))
        assert ms == h.max() and h[-1] == 1
        if n > 1:
            assert not oracle.validate(t[:-1])[0]  # truncated
        assert not oracle.validate(np.append(t, X))[0]  # trailing leaf
        bad = t.copy()
        bad[int(rng.integers(0, n))] = 5 + int(rng.integers(0, 250))
        assert not oracle.validate(bad)[0]
    assert not oracle.validate(np.array([], np.uint8))[0]
    for k in range(1, 20):
        left = np.array([ADD] * k + [X] * (k + 1), np.uint8)  # (((x+x)+x)...)
        right = np.array([ADD, X] * k + [X], np.uint8)       # x+(x+(x+...))
        assert oracle.validate(left) == (True, k + 1)
        assert oracle.validate(right) == (True, 2)


# -------------------------------------------------------------- crossover

def brute_subtree_end(t, p):
    def walk(i):
        return i + 1 if t[i] == X else walk(walk(i + 1))
    return walk(p) - 1


def test_crossover_invariants():
    rng = np.random.default_rng(12)
    for k in range(300):
        mum = workloads.random_tree(21, k, int(rng.integers(0, 60)) * 2 + 1)
        dad = workloads.random_tree(22, k, int(rng.integers(0, 60)) * 2 + 1)
        p = int(rng.integers(0, mum.size))
        q = int(rng.integers(0, dad.size))
        ep, eq = oracle.subtree_end(mum, p), oracle.subtree_end(dad, q)
        assert ep == brute_subtree_end(mum, p) and eq == brute_subtree_end(dad, q)
        child = oracle.crossover(mum, dad, p, q)
        assert child.size == mum.size - (ep - p + 1) + (eq - q + 1)
        assert np.array_equal(child[:p], mum[:p])
        assert np.array_equal(child[p:p + eq - q + 1], dad[q:eq + 1])
        assert np.array_equal(child[p + eq - q + 1:], mum[ep + 1:])
        assert oracle.validate(child)[0]
        if p == 0:
            assert np.array_equal(child, dad[q:eq + 1])


# ------------------------------------------------------- Philox, selection

def load_kat():
    rows = []
    for line in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(s, 16) for s in line.split()]
        rows.append((v[:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers():
    for ctr, key, want in load_kat():
        assert oracle.philox4x32_10(ctr, key).tolist() == want


def test_tournament_prefers_better_and_treats_nan_as_worst():
    sizes = np.full(4, 7, np.uint64)
    fit = np.array([np.nan, 0.5, np.nan, np.nan], np.float32)
    for child in range(50):
        m, d, p, q = oracle.choose(fit, 32, 99, 3, child, sizes)
        assert m == 1 and d == 1  # 32 draws over 4 trees: misses with prob 2^-64
        assert 0 <= p < 7 and 0 <= q < 7
    fit = np.array([np.inf, np.nan, 1.0, np.inf], np.float32)
    for child in range(50):
        m, _, _, _ = oracle.choose(fit, 32, 5, 0, child, sizes)
        assert m == 2


def test_selection_draws_are_uniform():
    m_count = np.zeros(10, np.int64)
    p_count = np.zeros(13, np.int64)
    fit = np.zeros(10, np.float32)
    sizes = np.full(10, 13, np.uint64)
    for child in range(4000):
        m, d, p, q = oracle.choose(fit, 1, 1234, 77, child, sizes)
        m_count[m] += 1
        p_count[p] += 1
    # chi-square at far-out thresholds (df 9 and 12)
    assert ((m_count - 400.0) ** 2 / 400.0).sum() < 40
    e = 4000 / 13
    assert ((p_count - e) ** 2 / e).sum() < 45


def test_generation_children_are_crossovers_of_chosen_parents():
    x, y = workloads.cases(48)
    buf, off = workloads.rhh_population(workloads.SEED_BASE + 9, 48, 2, 6)
    fit = oracle.eval_population(buf, off, x, y)
    cbuf, coff, capped = oracle.generation(buf, off, fit, 2, 42, 0, 10**9)
    assert capped == 0
    sizes = np.diff(off)
    for j in range(48):
        m, d, p, q = oracle.choose(fit, 2, 42, 0, j, sizes)
        mum = buf[off[m]:off[m + 1]]
        dad = buf[off[d]:off[d + 1]]
        child = cbuf[coff[j]:coff[j + 1]]
        assert np.array_equal(child, oracle.crossover(mum, dad, p, q))
    # a cap below every child size turns every child into a copy of its mum
    cbuf2, coff2, capped2 = oracle.generation(buf, off, fit, 2, 42, 0, 0)
    assert capped2 == 48
    for j in range(48):
        m, _, _, _ = oracle.choose(fit, 2, 42, 0, j, sizes)
        assert np.array_equal(cbuf2[coff2[j]:coff2[j + 1]], buf[off[m]:off[m + 1]])


def test_population_eval_threads_do_not_change_results():
    x, y = workloads.cases(48)
    sizes = workloads.loguniform_sizes(3, 64, 3, 3000)
    buf, off = workloads.random_population(3, sizes)
    f1, p1 = oracle.eval_population(buf, off, x, y, threads=1, per_case=True)
    f8, p8 = oracle.eval_population(buf, off, x, y, threads=8, per_case=True)
    assert same_bits(f1, f8).all() and same_bits(p1, p8).all()


def test_fitness_divides_once_by_n():
    # MAE = (sum) / (float)N with one correctly rounded division; a multiply
    # by a rounded 1/N differs for some sums, and those must not be taken.
    rng = np.random.default_rng(21)
    out = np.zeros(48, np.float32)
    differs = 0
    for v in rng.uniform(0.01, 100.0, 2000).astype(np.float32):
        y = np.zeros(48, np.float32)
        y[0] = v
        want = np.float32(v) / np.float32(48)
        differs += int(want != np.float32(v) * (np.float32(1) / np.float32(48)))
        assert oracle.fitness(out, y) == want
    assert differs > 0


def test_population_rows_match_per_tree_evaluation():
    # Each row t of the population result is tree t's own evaluation: its
    # per-case values against the recursive evaluator above, its fitness
    # against a plain ascending binary32 sum of |out - y| divided by N.
    x, y = workloads.cases(48)
    rng = np.random.default_rng(31)
    trees = [np.array([X], np.uint8)]  # a single leaf first
    for n in list(rng.integers(0, 40, 20) * 2 + 1) + [1, 3, 255]:
        sizes = np.array([n], np.uint64)
        b, _ = workloads.random_population(int(rng.integers(1 << 30)), sizes)
        trees.append(b)
    trees.append(np.array([X], np.uint8))  # and a single leaf last
    off = np.zeros(len(trees) + 1, np.uint64)
    off[1:] = np.cumsum([t.size for t in trees])
    buf = np.concatenate(trees)
    for threads in (1, 5):
        fit, pc = oracle.eval_population(buf, off, x, y, threads=threads, per_case=True)
        assert pc.shape == (len(trees), 48)
        for t, tree in enumerate(trees):
            want = ref_eval(tree, x)
            assert same_bits(pc[t], want).all(), t
            s = np.float32(0)
            for i in range(48):
                s = np.float32(s + np.float32(abs(np.float32(want[i] - y[i]))))
            assert same_bits(fit[t], np.float32(s / np.float32(48))), t


def tournament_by_hand(fit, M, k, seed, gen, child, role):
    # Candidate c of a tournament is word c % 4 of the Philox block with
    # counter (child, ((role + 1) << 8) | c // 4, gen lo, gen hi) under key
    # (seed lo, seed hi), mapped to [0, M) by a 32x32 multiply-high; the
    # first-drawn candidate among those of least fitness wins.
    key = [seed & 0xFFFFFFFF, seed >> 32]
    cands = []
    for c in range(k):
        w = oracle.philox4x32_10([child, ((role + 1) << 8) | (c // 4), gen & 0xFFFFFFFF, gen >> 32], key)
        cands.append((int(w[c % 4]) * M) >> 32)
    best = min(float(fit[c]) for c in cands)
    return next(c for c in cands if float(fit[c]) == best), cands


@pytest.mark.parametrize("k", [2, 7])
def test_tournament_ties_keep_the_earlier_draw(k):
    M = 16
    sizes = np.full(M, 9, np.uint64)
    rng = np.random.default_rng(k)
    all_equal = np.full(M, 0.25, np.float32)
    # two fitness levels only, so most tournaments hold several tied best
    partly = np.where(rng.random(M) < 0.5, 0.5, 0.75).astype(np.float32)
    seen_tie = 0
    for fit in (all_equal, partly):
        for child in range(200):
            m, d, _, _ = oracle.choose(fit, k, 0xABCDEF12345, 9, child, sizes)
            for role, got in ((0, m), (1, d)):
                want, cands = tournament_by_hand(fit, M, k, 0xABCDEF12345, 9, child, role)
                best = min(float(fit[c]) for c in cands)
                tied = {c for c in cands if float(fit[c]) == best}
                seen_tie += len(tied) > 1
                assert got == want, (k, child, role, cands)
    assert seen_tie > 100  # the rule was exercised, not a unique best


# ------------------------------------------------------------ depth, statistics

def ref_depth(tree):
    """Recursive depth (root 0) written here independently."""
    def d(i):
        if tree[i] == X:
            return 0, i + 1
        a, j = d(i + 1)
        b, k = d(j)
        return 1 + max(a, b), k

    v, end = d(0)
    assert end == len(tree)
    return v


def test_depth_exhaustive_small_trees_and_closed_forms():
    for n in range(1, 10, 2):
        for tree in all_trees(n):
            assert oracle.depth(tree) == ref_depth(tree)
    for k in range(1, 40):
        left = np.array([ADD] * k + [X] * (k + 1), np.uint8)        # op op ... x x ...
        right = np.array([MUL, X] * k + [X], np.uint8)              # op x op x ... x
        assert oracle.depth(left) == k and oracle.depth(right) == k
    # full trees of ramped half-and-half: depth d, 2^(d+1) - 1 nodes
    buf, off = workloads.rhh_population(workloads.SEED_BASE + 1, 100, 2, 6)
    for i in range(0, 100):
        if (i // 5) % 2 == 0:
            t = buf[off[i]:off[i + 1]]
            d = 2 + i % 5
            assert t.size == 2 ** (d + 1) - 1 and oracle.depth(t) == d
    with pytest.raises(ValueError):
        oracle.depth(np.array([ADD, X], np.uint8))


def test_depth_of_random_trees():
    rng = np.random.default_rng(5)
    for i in range(200):
        n = int(rng.integers(0, 2000)) * 2 + 1
        t = workloads.random_tree(77, i, n)
        assert oracle.depth(t) == workloads.depth(t)  # the generator's own left-to-right count
    # the random-tree law the paper quotes (depth near sqrt(2 pi size))
    n = 20001
    ds = [oracle.depth(workloads.random_tree(78, i, n)) for i in range(60)]
    assert 0.7 < np.mean(ds) / np.sqrt(2 * np.pi * n) < 1.3


def test_population_statistics_closed_forms():
    # fitness with NaN (worst), ties (first kept), and the convergence count
    trees = [np.array([X], np.uint8), np.array([SUB, X, X], np.uint8), np.array([ADD, ADD, X, X, X], np.uint8),
             np.array([MUL, X, X], np.uint8), np.array([X], np.uint8)]
    off = workloads.offsets_from_sizes([t.size for t in trees])
    buf = np.concatenate(trees)
    fit = np.array([np.nan, 0.25, 0.125, 0.125, np.inf], np.float32)
    hits = np.array([0, 3, 7, 9, 1], np.int32)
    s = oracle.population_stats(buf, off, fit, hits)
    assert s["best_tree"] == 2 and s["best_fitness"] == 0.125 and s["best_hits"] == 7
    assert s["best_size"] == 5 and s["best_depth"] == 2 and s["converged"] == 2
    assert s["min_size"] == 1 and s["max_size"] == 5 and s["mean_size"] == 13 / 5
    assert s["max_depth"] == 2 and s["min_depth"] == 0 and s["mean_depth"] == (0 + 1 + 2 + 1 + 0) / 5
    assert s["mean_fitness"] == (0.25 + 0.125 + 0.125) / 3
    allnan = oracle.population_stats(buf, off, np.full(5, np.nan, np.float32), hits)
    assert allnan["best_tree"] == 0 and allnan["converged"] == 5 and np.isnan(allnan["mean_fitness"])


# ------------------------------------------------- ephemeral random constants

def ref_eval_c(tree, x, consts):
    """Recursive evaluation with constant leaves (token 6 + i is consts[i])."""
    x = np.asarray(x, np.float32)

    def ev(i):
        t = int(tree[i])
        if t == X:
            return x.copy(), i + 1
        if t >= 6:
            return np.full(x.shape, consts[t - 6], np.float32), i + 1
        a, j = ev(i + 1)
        b, k = ev(j)
        return ref_op(t, a, b), k

    v, end = ev(0)
    assert end == len(tree)
    return v


def test_constant_table_draw():
    c = workloads.erc_table(11, 250)
    assert c.size == 250 and len(set(c.tolist())) == 250
    k = np.round(c.astype(np.float64) * 1000.0)
    assert np.all(np.abs(k) <= 1000)
    assert np.array_equal(c, (k / 1000.0).astype(np.float32))  # each the binary32 nearest k/1000


def test_constant_trees_evaluate_to_their_constant():
    x, y = workloads.cases(48)
    consts = workloads.erc_table(12, 250)
    for i in (0, 1, 77, 249):
        tree = np.array([6 + i], np.uint8)
        out = oracle.eval_cases(tree, x, consts)
        assert (out.view(np.uint32) == np.full(48, consts[i], np.float32).view(np.uint32)).all()
        s = np.float32(0)
        for v in y:
            s = np.float32(s + np.float32(abs(np.float32(consts[i] - v))))
        assert oracle.fitness(out, y) == np.float32(s / np.float32(48))
    # c - c is 0 and c % c is 1 for a nonzero constant
    i = int(np.argmax(np.abs(consts)))
    assert (oracle.eval_cases(np.array([SUB, 6 + i, 6 + i], np.uint8), x, consts) == 0).all()
    assert (oracle.eval_cases(np.array([DIV, 6 + i, 6 + i], np.uint8), x, consts) == 1).all()


def test_constant_rich_trees_against_recursive_reference():
    x, _ = workloads.cases(48)
    consts = workloads.erc_table(13, 250)
    rng = np.random.default_rng(14)
    for i in range(300):
        n = int(rng.integers(0, 60)) * 2 + 1
        t = workloads.with_constants(workloads.random_tree(15, i, n), 16 + i, 250, 0.5)
        assert same_bits(oracle.eval_cases(t, x, consts), ref_eval_c(t, x, consts)).all()


def test_constant_tokens_are_validated_against_the_table():
    assert oracle.validate(np.array([ADD, 6, 255], np.uint8), 250)[0]
    assert not oracle.validate(np.array([ADD, 6, 255], np.uint8), 249)[0]
    assert not oracle.validate(np.array([ADD, X, 5], np.uint8), 250)[0]  # 5 is never a tree token
    assert not oracle.validate(np.array([ADD, X, 6], np.uint8), 0)[0]
    with pytest.raises(ValueError):
        oracle.eval_cases(np.array([ADD, X, 7], np.uint8), np.zeros(4, np.float32), np.zeros(1, np.float32))
    # crossover and subtree ends treat constants as leaves
    t = np.array([MUL, 9, ADD, X, 200], np.uint8)
    assert oracle.subtree_end(t, 1) == 1 and oracle.subtree_end(t, 2) == 4 and oracle.depth(t) == 2
