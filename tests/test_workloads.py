"""Sanity of the seeded input generators (shapes, sizes, validity)."""
import math

import numpy as np

import oracle
import workloads


def test_case_table():
    x, y = workloads.cases(48)
    assert x.dtype == np.float32 and x.size == 48
    assert x[0] == -1.0 and x[-1] == 1.0 and np.all(np.diff(x) > 0) and np.all(x != 0)
    xd = x.astype(np.float64)
    assert np.array_equal(y, (xd ** 6 - 2 * xd ** 4 + xd ** 2).astype(np.float32))
    x2, _ = workloads.cases(1024)
    assert x2.size == 1024 and np.all(np.abs(x2) <= 1)


def test_ramped_half_and_half():
    buf, off = workloads.rhh_population(workloads.SEED_BASE + 1, 100, 2, 6)
    sizes = np.diff(off)
    for i in range(100):
        t = buf[off[i]:off[i + 1]]
        assert oracle.validate(t)[0]
        d = 2 + i % 5
        depth = workloads.depth(t)
        if (i // 5) % 2 == 0:  # full
            assert sizes[i] == 2 ** (d + 1) - 1 and depth == d
        else:
            assert 1 <= depth <= d
    assert sizes.max() <= 127


def test_random_trees_valid_and_sized():
    for n in (1, 3, 5, 101, 4097):
        t = workloads.random_tree(1, n, n)
        assert t.size == n and oracle.validate(t)[0]
        assert np.all(t <= 4)


def test_random_tree_depth_follows_random_tree_law():
    # depth of random binary trees tends to 2*sqrt(pi*ceil(n/2)) (Sec. 2.2)
    n = 20001
    d = np.mean([workloads.depth(workloads.random_tree(2, k, n)) for k in range(24)])
    want = 2 * math.sqrt(math.pi * math.ceil(n / 2))
    assert 0.75 * want < d < 1.25 * want


def test_op_labels_uniform():
    t = workloads.random_tree(3, 0, 200001)
    ops = t[t != 4]
    counts = np.bincount(ops, minlength=4)
    assert np.all(np.abs(counts / ops.size - 0.25) < 0.01)


def test_batched_workload_shape():
    buf, off, n_cases = workloads.workload("batched")
    sizes = np.diff(off)
    assert n_cases == 48 and sizes.size == 4000
    assert sizes.min() >= 9 and sizes.max() <= 100001 and np.all(sizes % 2 == 1)
    assert 3.0e7 < off[-1] < 6.0e7  # mean of log-uniform [10, 1e5] is ~10856
    for t in (0, 1, 1999, 3999):
        assert oracle.validate(buf[off[t]:off[t + 1]])[0]


def test_generators_are_seeded():
    a = workloads.random_tree(5, 9, 1001)
    b = workloads.random_tree(5, 9, 1001)
    c = workloads.random_tree(5, 10, 1001)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
