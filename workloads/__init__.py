"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

Only input data lives here (case tables and tree populations); none of the
evaluation, fitness, crossover or selection arithmetic does.  The C source
is ``gen.c``; ``build()`` compiles it into ``libworkloads.so`` next to it.

Population format: ``(buf, off)`` where ``buf`` is a uint8 array of prefix
opcodes (0 ADD, 1 SUB, 2 MUL, 3 DIV, 4 X; root first, Sec. 2.2 of the paper)
and ``off`` is a uint64 array of M+1 offsets, tree t = buf[off[t]:off[t+1]].

Workload recipes (the paper's own cases and evolved trees are not printed,
so these stand in for their shapes and sizes):

* ``tiny``     100 ramped half-and-half trees, depth 2-6, 48 cases.
* ``batched``  4000 uniformly random trees, sizes log-uniform in [10, 1e5].
* ``giant``    48 uniformly random trees, sizes log-uniform in [1e6, 4e8].
* ``giant_max``48 uniformly random trees of ~4e8 nodes each (~19.2 GB).
* ``serving``  sizes log-uniform in [10, 1e8], 48 or 1024 cases.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libworkloads.so")
_lib = None

SEED_BASE = 0x5EED0000
OP_ADD, OP_SUB, OP_MUL, OP_DIV, OP_X = 0, 1, 2, 3, 4


def build() -> str:
    """Compile gen.c into libworkloads.so (always recompiles)."""
    src = os.path.join(_HERE, "gen.c")
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-o", tmp, src, "-lpthread", "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    lib.wl_cases.argtypes = [ctypes.c_int32, P, P]
    lib.wl_rhh.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_uint64, P]
    lib.wl_rhh.restype = ctypes.c_int64
    lib.wl_random_tree.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64, P]
    lib.wl_loguniform_sizes.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_double, ctypes.c_double, P]
    lib.wl_random_pop.argtypes = [ctypes.c_uint64, ctypes.c_int32, P, P, ctypes.c_int32]
    lib.wl_depth.argtypes = [P, ctypes.c_uint64, P]
    lib.wl_depth.restype = ctypes.c_int64
    lib.wl_erc_table.argtypes = [ctypes.c_uint64, ctypes.c_int32, P]
    lib.wl_relabel_leaves.argtypes = [ctypes.c_uint64, P, ctypes.c_uint64, ctypes.c_int32, ctypes.c_double]
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def cases(n: int = 48):
    """Evenly spaced x in [-1, 1] and y = x^6 - 2x^4 + x^2 (binary64, rounded once)."""
    lib = _load()
    x = np.empty(n, np.float32)
    y = np.empty(n, np.float32)
    lib.wl_cases(n, _ptr(x), _ptr(y))
    return x, y


def rhh_population(seed: int, m: int, dmin: int = 2, dmax: int = 6):
    lib = _load()
    cap = m * ((1 << (dmax + 1)) - 1) + 16
    buf = np.empty(cap, np.uint8)
    off = np.empty(m + 1, np.uint64)
    total = lib.wl_rhh(seed, m, dmin, dmax, _ptr(buf), cap, _ptr(off))
    if total < 0:
        raise RuntimeError("rhh buffer too small")
    return buf[:total].copy(), off


def loguniform_sizes(seed: int, m: int, lo: float, hi: float) -> np.ndarray:
    lib = _load()
    s = np.empty(m, np.uint64)
    lib.wl_loguniform_sizes(seed, m, lo, hi, _ptr(s))
    return s


def offsets_from_sizes(sizes) -> np.ndarray:
    sizes = np.asarray(sizes, dtype=np.uint64)
    off = np.zeros(len(sizes) + 1, np.uint64)
    np.cumsum(sizes, out=off[1:])
    return off


def random_population(seed: int, sizes, out: np.ndarray | None = None, threads: int | None = None):
    """Uniformly random trees with the given odd sizes.  ``out`` may be a
    preallocated uint8 array (e.g. a view of pinned memory) of len >= sum."""
    lib = _load()
    sizes = np.asarray(sizes, dtype=np.uint64)
    if np.any(sizes % 2 == 0):
        raise ValueError("tree sizes must be odd")
    off = offsets_from_sizes(sizes)
    total = int(off[-1])
    buf = np.empty(total, np.uint8) if out is None else out
    if buf.size < total or buf.dtype != np.uint8 or not buf.flags.c_contiguous:
        raise ValueError("out buffer must be contiguous uint8 of at least the total size")
    if threads is None:
        threads = min(16, os.cpu_count() or 1)
    lib.wl_random_pop(seed, len(sizes), _ptr(off), _ptr(buf), threads)
    return buf[:total], off


def random_tree(seed: int, stream: int, n: int) -> np.ndarray:
    lib = _load()
    t = np.empty(n, np.uint8)
    lib.wl_random_tree(seed, stream, n, _ptr(t))
    return t


def depth(tree: np.ndarray) -> int:
    lib = _load()
    tree = np.ascontiguousarray(tree, dtype=np.uint8)
    scratch = np.empty(tree.size + 2, np.int64)
    return int(lib.wl_depth(_ptr(tree), tree.size, _ptr(scratch)))


def erc_table(seed: int, n: int = 250) -> np.ndarray:
    """n distinct ephemeral random constants from the 2001 values k/1000,
    k = -1000..1000 (binary32 nearest each)."""
    out = np.empty(n, np.float32)
    _load().wl_erc_table(seed, n, _ptr(out))
    return out


def with_constants(buf, seed: int, n_consts: int = 250, p_x: float = 0.5) -> np.ndarray:
    """A copy of the trees in buf with each x leaf turned into a random
    constant token (6 + j) with probability 1 - p_x."""
    b = np.array(buf, dtype=np.uint8, copy=True)
    _load().wl_relabel_leaves(seed, _ptr(b), b.size, n_consts, p_x)
    return b


# ------------------------------------------------------------ workloads

def workload(name: str, **kw):
    """Return (buf, off, n_cases) for a named workload."""
    if name == "tiny":
        buf, off = rhh_population(SEED_BASE + 1, kw.get("m", 100), 2, 6)
        return buf, off, 48
    if name == "batched":
        m = kw.get("m", 4000)
        sizes = loguniform_sizes(SEED_BASE + 2, m, 10.0, 1e5)
        buf, off = random_population(SEED_BASE + 2, sizes, out=kw.get("out"))
        return buf, off, 48
    if name == "giant":
        m = kw.get("m", 48)
        sizes = loguniform_sizes(SEED_BASE + 3, m, kw.get("lo", 1e6), kw.get("hi", 4e8))
        buf, off = random_population(SEED_BASE + 3, sizes, out=kw.get("out"))
        return buf, off, 48
    if name == "giant_max":
        m = kw.get("m", 48)
        n = int(kw.get("n", 400_000_001))
        sizes = np.full(m, n | 1, np.uint64)
        buf, off = random_population(SEED_BASE + 4, sizes, out=kw.get("out"))
        return buf, off, 48
    raise KeyError(name)
