"""ctypes wrapper of the C oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the library path.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    src = os.path.join(_HERE, "oracle.c")
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                           "-o", tmp, src, "-lpthread", "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P, u64, i32, u32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int32, ctypes.c_uint32
    lib.or_op.argtypes = [ctypes.c_int, ctypes.c_float, ctypes.c_float]
    lib.or_op.restype = ctypes.c_float
    lib.or_validate.argtypes = [P, u64, P]
    lib.or_validate.restype = ctypes.c_int
    lib.or_validate_c.argtypes = [P, u64, i32, P]
    lib.or_validate_c.restype = ctypes.c_int
    lib.or_eval_cases_c.argtypes = [P, u64, P, i32, P, i32, P]
    lib.or_eval_cases_c.restype = ctypes.c_int
    lib.or_eval_population_c.argtypes = [P, P, i32, P, P, i32, P, i32, P, P, i32]
    lib.or_eval_population_c.restype = ctypes.c_int64
    lib.or_eval_cases.argtypes = [P, u64, P, i32, P]
    lib.or_eval_cases.restype = ctypes.c_int
    lib.or_fitness.argtypes = [P, P, i32]
    lib.or_fitness.restype = ctypes.c_float
    lib.or_hits.argtypes = [P, P, i32]
    lib.or_hits.restype = ctypes.c_int32
    lib.or_eval_population.argtypes = [P, P, i32, P, P, i32, P, P, i32]
    lib.or_eval_population.restype = ctypes.c_int64
    lib.or_depth.argtypes = [P, u64]
    lib.or_depth.restype = ctypes.c_int64
    lib.or_subtree_end.argtypes = [P, u64, u64]
    lib.or_subtree_end.restype = u64
    lib.or_crossover.argtypes = [P, u64, P, u64, u64, u64, P]
    lib.or_crossover.restype = u64
    lib.or_philox4x32_10.argtypes = [P, P, P]
    lib.or_choose.argtypes = [P, i32, i32, u64, u64, u32, P, P, P, P, P]
    lib.or_generation.argtypes = [P, P, i32, P, i32, u64, u64, u64, P, u64, P]
    lib.or_generation.restype = ctypes.c_int64
    _lib = lib
    return lib


def _p(a: np.ndarray) -> int:
    return a.ctypes.data


def _u8(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint8)


def op(o: int, a: float, b: float) -> np.float32:
    return np.float32(_load().or_op(o, a, b))


def _consts(consts):
    if consts is None:
        return None, 0
    c = np.ascontiguousarray(consts, dtype=np.float32)
    return c, int(c.size)


def validate(tree, n_consts: int = 0):
    t = _u8(tree)
    ms = np.zeros(1, np.uint64)
    ok = _load().or_validate_c(_p(t), t.size, n_consts, _p(ms))
    return bool(ok), int(ms[0])


def eval_cases(tree, x, consts=None) -> np.ndarray:
    """consts: the ephemeral random constants (token 6 + i is consts[i])."""
    t = _u8(tree)
    x = np.ascontiguousarray(x, dtype=np.float32)
    c, nc = _consts(consts)
    out = np.empty(x.size, np.float32)
    if _load().or_eval_cases_c(_p(t), t.size, _p(x), x.size, _p(c) if nc else None, nc, _p(out)) != 0:
        raise ValueError("invalid tree")
    return out


def fitness(out, y) -> np.float32:
    out = np.ascontiguousarray(out, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    return np.float32(_load().or_fitness(_p(out), _p(y), out.size))


def eval_population(buf, off, x, y, threads: int = 1, per_case: bool = False, consts=None):
    buf = _u8(buf)
    off = np.ascontiguousarray(off, dtype=np.uint64)
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    c, nc = _consts(consts)
    m = off.size - 1
    fit = np.empty(m, np.float32)
    pc = np.empty((m, x.size), np.float32) if per_case else None
    rc = _load().or_eval_population_c(_p(buf), _p(off), m, _p(x), _p(y), x.size, _p(c) if nc else None, nc,
                                      _p(fit), _p(pc) if pc is not None else None, threads)
    if rc != 0:
        raise ValueError(f"tree {-rc - 1} invalid")
    return (fit, pc) if per_case else fit


def hits(per_case, y) -> np.ndarray:
    """Hits of each tree from its per-case outputs (Sec. 3.2)."""
    pc = np.ascontiguousarray(per_case, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    lib = _load()
    return np.array([lib.or_hits(_p(pc[t]), _p(y), y.size) for t in range(pc.shape[0])], np.int32)


def depth(tree) -> int:
    t = _u8(tree)
    d = int(_load().or_depth(_p(t), t.size))
    if d < 0:
        raise ValueError("invalid tree")
    return d


def population_stats(buf, off, fitness, hits):
    """Per-generation statistics of an evaluated population, as the paper
    reports them (Sec. 4, the columns of its result tables and its size and
    depth plots): the best (least) fitness with NaN worst and the first of
    equals chosen, that tree's hits and size and depth, the number of trees
    whose fitness equals the best bit for bit, or is NaN with a NaN best
    (convergence: NaN payloads differ across machines), the mean
    fitness over trees whose fitness is finite, and the sizes' and depths'
    minimum, maximum and mean."""
    f = np.ascontiguousarray(fitness, np.float32)
    off = np.ascontiguousarray(off, np.uint64)
    M = f.size
    best = -1
    for t in range(M):
        if best < 0:
            best = t
        elif not np.isnan(f[t]) and (np.isnan(f[best]) or f[t] < f[best]):
            best = t
    sizes = np.diff(off).astype(np.int64)
    depths = np.array([depth(buf[off[t]:off[t + 1]]) for t in range(M)], np.int64)
    fin = np.isfinite(f)
    return {
        "best_fitness": float(f[best]),
        "best_tree": int(best),
        "best_hits": int(hits[best]),
        "best_size": int(sizes[best]),
        "best_depth": int(depths[best]),
        "converged": int(np.sum((f.view(np.uint32) == f[best:best + 1].view(np.uint32)[0])
                                | (np.isnan(f) & np.isnan(f[best])))),
        "mean_fitness": float(np.mean(f[fin].astype(np.float64))) if fin.any() else float("nan"),
        "min_size": int(sizes.min()), "max_size": int(sizes.max()), "mean_size": float(sizes.mean()),
        "min_depth": int(depths.min()), "max_depth": int(depths.max()), "mean_depth": float(depths.mean()),
        "depths": depths,
    }


def subtree_end(tree, p: int) -> int:
    t = _u8(tree)
    return int(_load().or_subtree_end(_p(t), t.size, p))


def crossover(mum, dad, p: int, q: int) -> np.ndarray:
    m, d = _u8(mum), _u8(dad)
    lib = _load()
    n = lib.or_crossover(_p(m), m.size, _p(d), d.size, p, q, None)
    child = np.empty(n, np.uint8)
    lib.or_crossover(_p(m), m.size, _p(d), d.size, p, q, _p(child))
    return child


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, np.uint32)
    _load().or_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def choose(fitness_arr, k: int, seed: int, gen: int, child: int, sizes):
    f = np.ascontiguousarray(fitness_arr, dtype=np.float32)
    s = np.ascontiguousarray(sizes, dtype=np.uint64)
    m = np.zeros(1, np.int32)
    d = np.zeros(1, np.int32)
    p = np.zeros(1, np.uint64)
    q = np.zeros(1, np.uint64)
    _load().or_choose(_p(f), f.size, k, seed, gen, child, _p(s), _p(m), _p(d), _p(p), _p(q))
    return int(m[0]), int(d[0]), int(p[0]), int(q[0])


def generation(buf, off, fitness_arr, k: int, seed: int, gen: int, size_cap: int):
    buf = _u8(buf)
    off = np.ascontiguousarray(off, dtype=np.uint64)
    f = np.ascontiguousarray(fitness_arr, dtype=np.float32)
    m = off.size - 1
    sizes = np.diff(off)
    cap_bytes = int(m * max(int(size_cap), int(sizes.max()) if m else 0)) + 1
    cbuf = np.empty(cap_bytes, np.uint8)
    coff = np.empty(m + 1, np.uint64)
    capped = _load().or_generation(_p(buf), _p(off), m, _p(f), k, seed, gen, size_cap,
                                   _p(cbuf), cap_bytes, _p(coff))
    if capped < 0:
        raise RuntimeError("child buffer too small")
    return cbuf[: int(coff[-1])].copy(), coff, int(capped)
