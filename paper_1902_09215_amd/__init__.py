"""Python binding of libev (GP-tree evaluation on MI355X).

Argument marshalling only: every step of evaluation, crossover and selection
runs in the HIP kernels of ``libev.so`` (built from ``csrc/`` by
``build.build()``).  The functions carry the names of the C ABI in
``include/ev.h``; ``Context`` is a small convenience wrapper over them.

Inputs may be numpy arrays (host) or torch tensors on the GPU (device
pointers, passed with EV_DEVICE_PTR / EV_OUT_DEVICE).  There is no fallback:
if ``libev.so`` is missing or fails to load, importing the library raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libev.so")

EV_OK, EV_EINVAL, EV_EMALFORMED, EV_ENOMEM, EV_ECAP, EV_EBUSY, EV_ENOTFOUND, EV_EDEVICE = 0, -1, -2, -3, -4, -5, -6, -7
EV_ADD, EV_SUB, EV_MUL, EV_DIV, EV_X = 0, 1, 2, 3, 4
EV_C0, EV_MAX_CONSTS = 6, 250
EV_DEVICE_PTR, EV_OUT_DEVICE = 0x1, 0x2
EV_STATIC_SCRATCH_BYTES = 0x4000000
EV_JOB_EVAL, EV_JOB_CROSSOVER = 0, 1

EXPORTS = [
    "ev_create", "ev_add_cases", "ev_destroy", "ev_last_error", "ev_load_trees", "ev_pop_info",
    "ev_get_trees", "ev_free_pop", "ev_eval_fitness", "ev_crossover", "ev_generation", "ev_submit",
    "ev_poll", "ev_wait", "ev_result", "ev_job_timing", "ev_get_plan_info", "ev_get_level_info", "ev_set_tuning",
    "ev_autotune", "ev_last_level_times", "ev_last_timing", "ev_eval_fitness_static", "ev_population_stats",
    "ev_set_constants", "ev_autotune_ex", "ev_tune_cache_save", "ev_tune_cache_load", "ev_evolve",
]


class EvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libev error {code}: {msg}")
        self.code = code


class ev_plan_info(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("chunks", ctypes.c_uint64), ("slots", ctypes.c_uint64),
                ("max_stack", ctypes.c_uint64), ("plan_bytes", ctypes.c_uint64)]


class ev_level_info(ctypes.Structure):
    _fields_ = [("tokens", ctypes.c_uint64), ("trees", ctypes.c_uint32), ("items", ctypes.c_uint32),
                ("slots", ctypes.c_uint32), ("launch", ctypes.c_uint32), ("codes", ctypes.c_uint64)]


class ev_evolve_report(ctypes.Structure):
    _fields_ = [("generations", ctypes.c_int32), ("replayed", ctypes.c_int32), ("fallbacks", ctypes.c_int32),
                ("captures", ctypes.c_int32), ("capped", ctypes.c_uint64), ("nodes", ctypes.c_uint64),
                ("ms", ctypes.c_double),
                ("ms_capture", ctypes.c_double), ("lean_peak_bytes", ctypes.c_uint64),
                ("lean_two_buffer_bytes", ctypes.c_uint64), ("lean_arena_bytes", ctypes.c_uint64),
                ("lean_repacks", ctypes.c_int32), ("pad", ctypes.c_int32)]


class ev_pop_stats(ctypes.Structure):
    _fields_ = [("best_fitness", ctypes.c_float), ("best_tree", ctypes.c_int32), ("best_hits", ctypes.c_int32),
                ("converged", ctypes.c_int32), ("mean_fitness", ctypes.c_double), ("best_size", ctypes.c_uint64),
                ("min_size", ctypes.c_uint64), ("max_size", ctypes.c_uint64), ("mean_size", ctypes.c_double),
                ("best_depth", ctypes.c_uint32), ("min_depth", ctypes.c_uint32), ("max_depth", ctypes.c_uint32),
                ("pad", ctypes.c_uint32), ("mean_depth", ctypes.c_double)]


class ev_tune_choice(ctypes.Structure):
    _fields_ = [("chunk", ctypes.c_uint32), ("chunk_hi", ctypes.c_uint32), ("waves_per_cu", ctypes.c_uint32),
                ("from_cache", ctypes.c_uint32), ("ms", ctypes.c_float)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class ev_allocator(ctypes.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", ctypes.c_void_p)]


class ev_job(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("table", ctypes.c_int32),
                ("bytes", ctypes.c_void_p), ("off", ctypes.c_void_p), ("n_trees", ctypes.c_int32),
                ("parents", ctypes.c_int32),
                ("mum", ctypes.c_void_p), ("dad", ctypes.c_void_p), ("p", ctypes.c_void_p), ("q", ctypes.c_void_p),
                ("n_children", ctypes.c_int32), ("size_cap", ctypes.c_uint64)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libev.so and declare its C signatures (raises if absent)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libev.so not built ({path}); run __graft_entry__.build()")
    # One HIP runtime per process: torch ships its own, and a process that
    # loaded another one first cannot use torch's device memory (or torch at
    # all) afterwards.  Loading torch first makes libev use torch's runtime,
    # so device tensors and torch's caching allocator work with it.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P, i32, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
    sig = {
        "ev_create": [ctypes.POINTER(P), ctypes.c_int, P, P, i32, u64, ctypes.POINTER(ev_allocator), P],
        "ev_add_cases": [P, P, P, i32, ctypes.POINTER(i32)],
        "ev_destroy": [P],
        "ev_last_error": [],
        "ev_load_trees": [P, P, P, i32, u32, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "ev_pop_info": [P, i32, ctypes.POINTER(i32), ctypes.POINTER(u64)],
        "ev_get_trees": [P, i32, P, P, u64],
        "ev_free_pop": [P, i32],
        "ev_eval_fitness": [P, i32, i32, P, P, P, u32],
        "ev_crossover": [P, i32, i32, P, P, P, P, i32, u64, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "ev_generation": [P, i32, P, u64, u64, i32, u64, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "ev_submit": [P, ctypes.POINTER(ev_job), ctypes.POINTER(u64)],
        "ev_poll": [P, u64, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "ev_wait": [P, u64, ctypes.POINTER(i32)],
        "ev_result": [P, u64, P, P, i32, ctypes.POINTER(i32)],
        "ev_job_timing": [P, u64, ctypes.POINTER(u64), ctypes.POINTER(u64), ctypes.POINTER(u64)],
        "ev_get_plan_info": [P, i32, ctypes.POINTER(ev_plan_info)],
        "ev_get_level_info": [P, i32, i32, ctypes.POINTER(ev_level_info)],
        "ev_set_tuning": [P, u32, u32, u32, u32],
        "ev_autotune": [P, i32, i32, i32, ctypes.POINTER(u32), ctypes.POINTER(ctypes.c_float)],
        "ev_last_level_times": [P, ctypes.POINTER(ctypes.c_float), i32, ctypes.POINTER(i32)],
        "ev_last_timing": [P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)],
        "ev_eval_fitness_static": [P, i32, i32, P, P, P],
        "ev_population_stats": [P, i32, ctypes.POINTER(ev_pop_stats), P],
        "ev_set_constants": [P, P, i32],
        "ev_autotune_ex": [P, i32, i32, i32, u32, ctypes.POINTER(ev_tune_choice)],
        "ev_tune_cache_save": [ctypes.c_char_p],
        "ev_tune_cache_load": [ctypes.c_char_p],
        "ev_evolve": [P, i32, P, i32, u64, u64, i32, i32, u64, u32, ctypes.POINTER(i32), P, P,
                      ctypes.POINTER(ev_evolve_report)],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_char_p if name == "ev_last_error" else ctypes.c_int32
    _lib = lib
    return lib


def _check(rc: int):
    if rc != EV_OK:
        raise EvError(rc, (_lib.ev_last_error() or b"").decode(errors="replace"))


def _ptr(a) -> int:
    """Address of a numpy array or a torch tensor."""
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _is_device(a) -> bool:
    return (not isinstance(a, np.ndarray)) and getattr(a, "is_cuda", False)


# ---------------------------------------------------------------- C names

def ev_create(x, y, device: int = 0, mem_budget: int = 0, stream: int | None = None, allocator=None):
    """allocator: None (hipMalloc), or an ev_allocator (see torch_allocator);
    the caller keeps it alive for the context's lifetime."""
    lib = load_library()
    x = np.ascontiguousarray(x, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    ctx = ctypes.c_void_p()
    _check(lib.ev_create(ctypes.byref(ctx), device, _ptr(x), _ptr(y), x.size, mem_budget,
                         ctypes.byref(allocator) if allocator is not None else None, stream))
    return ctx


def torch_allocator(device: int = 0):
    """An ev_allocator drawing device blocks from torch's caching allocator
    (``torch.cuda.caching_allocator_alloc`` / ``_delete``).  Keep the returned
    object alive while a context uses it."""
    import torch

    def alloc(nbytes, _user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device)
        except RuntimeError:
            return None

    def free(ptr, _user):
        torch.cuda.caching_allocator_delete(ptr)

    a = ev_allocator(_ALLOC_FN(alloc), _FREE_FN(free), None)
    a._keep = (alloc, free)  # the Python functions behind the C callbacks
    return a


def ev_add_cases(ctx, x, y) -> int:
    x = np.ascontiguousarray(x, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    t = ctypes.c_int32()
    _check(_lib.ev_add_cases(ctx, _ptr(x), _ptr(y), x.size, ctypes.byref(t)))
    return t.value


def ev_set_constants(ctx, consts):
    """The context's ephemeral random constants: token 6 + i is consts[i]."""
    c = np.ascontiguousarray(consts, np.float32)
    _check(_lib.ev_set_constants(ctx, _ptr(c) if c.size else None, c.size))


def ev_destroy(ctx):
    _check(_lib.ev_destroy(ctx))


def ev_last_error() -> str:
    return (load_library().ev_last_error() or b"").decode(errors="replace")


def ev_load_trees(ctx, buf, off):
    """buf/off: numpy (host) or torch cuda tensors (device).  Returns a pop."""
    dev = _is_device(buf)
    if not dev:
        buf = np.ascontiguousarray(buf, np.uint8)
        off = np.ascontiguousarray(off, np.uint64)
        n = off.size - 1
    else:
        n = off.numel() - 1
    pop = ctypes.c_int32()
    bad = ctypes.c_int32(-1)
    rc = _lib.ev_load_trees(ctx, _ptr(buf), _ptr(off), n, EV_DEVICE_PTR if dev else 0, ctypes.byref(pop),
                            ctypes.byref(bad))
    if rc != EV_OK:
        err = EvError(rc, ev_last_error())
        err.bad_tree = bad.value
        raise err
    return pop.value


def ev_pop_info(ctx, pop):
    n = ctypes.c_int32()
    b = ctypes.c_uint64()
    _check(_lib.ev_pop_info(ctx, pop, ctypes.byref(n), ctypes.byref(b)))
    return n.value, b.value


def ev_get_trees(ctx, pop):
    n, total = ev_pop_info(ctx, pop)
    buf = np.empty(max(total, 1), np.uint8)
    off = np.empty(n + 1, np.uint64)
    _check(_lib.ev_get_trees(ctx, pop, _ptr(buf), _ptr(off), buf.size))
    return buf[:total], off


def ev_free_pop(ctx, pop):
    _check(_lib.ev_free_pop(ctx, pop))


def ev_eval_fitness(ctx, pop, table: int = 0, per_case: bool = False, out=None, out_per_case=None,
                    hits: bool = False, out_hits=None):
    """Host results (numpy) by default: (fitness, per_case or None), plus the
    hits (int32 per tree) when hits=True.  Pass torch cuda tensors as out /
    out_per_case / out_hits to receive device results without a host copy."""
    if out is not None:
        _check(_lib.ev_eval_fitness(ctx, pop, table, _ptr(out), _ptr(out_per_case), _ptr(out_hits), EV_OUT_DEVICE))
        return (out, out_per_case, out_hits) if out_hits is not None else (out, out_per_case)
    n, _ = ev_pop_info(ctx, pop)
    fit = np.empty(max(n, 1), np.float32)
    pc = None
    if per_case:
        N = _table_n(ctx, table)
        pc = np.empty((max(n, 1), N), np.float32)
    h = np.empty(max(n, 1), np.int32) if hits else None
    _check(_lib.ev_eval_fitness(ctx, pop, table, _ptr(fit), _ptr(pc), _ptr(h), 0))
    res = (fit[:n], pc[:n] if pc is not None else None)
    return res + (h[:n],) if hits else res


def ev_population_stats(ctx, pop, depths: bool = False):
    """Statistics of the population's last evaluation (see ev.h): a dict,
    with every tree's depth under "depths" when asked for."""
    st = ev_pop_stats()
    n, _ = ev_pop_info(ctx, pop)
    d = np.empty(max(n, 1), np.uint32) if depths else None
    _check(_lib.ev_population_stats(ctx, pop, ctypes.byref(st), _ptr(d)))
    out = {k: getattr(st, k) for k, _ in ev_pop_stats._fields_ if k != "pad"}
    if depths:
        out["depths"] = d[:n]
    return out


def ev_eval_fitness_static(ctx, pop, out, table: int = 0, out_per_case=None, out_hits=None):
    """ev_eval_fitness into device tensors with no allocation (see ev.h)."""
    _check(_lib.ev_eval_fitness_static(ctx, pop, table, _ptr(out), _ptr(out_per_case), _ptr(out_hits)))
    return out


_table_sizes: dict = {}


def _table_n(ctx, table: int) -> int:
    return _table_sizes[(ctx.value, table)]


def ev_crossover(ctx, mums, dads, mum, dad, p, q, size_cap: int = 2**63):
    mum = np.ascontiguousarray(mum, np.int32)
    dad = np.ascontiguousarray(dad, np.int32)
    p = np.ascontiguousarray(p, np.uint64)
    q = np.ascontiguousarray(q, np.uint64)
    out = ctypes.c_int32()
    capped = ctypes.c_int32()
    _check(_lib.ev_crossover(ctx, mums, dads, _ptr(mum), _ptr(dad), _ptr(p), _ptr(q), mum.size, size_cap,
                             ctypes.byref(out), ctypes.byref(capped)))
    return out.value, capped.value


def ev_generation(ctx, parents, seed: int, gen: int, tournament: int = 2, size_cap: int = 2**63, fitness=None):
    """fitness: a torch CUDA tensor of the parents' fitness, or None for the
    values of their last evaluation."""
    out = ctypes.c_int32()
    capped = ctypes.c_int32()
    _check(_lib.ev_generation(ctx, parents, _ptr(fitness), seed, gen, tournament, size_cap, ctypes.byref(out),
                              ctypes.byref(capped)))
    return out.value, capped.value


def ev_evolve(ctx, parents, seed: int, gen0: int, n_gen: int, tournament: int = 2, size_cap: int = 2**63,
              table: int = 0, flags: int = 0, fitness=None, history: bool = True):
    """n_gen generations from parents; returns (population, fitness history
    [n_gen, n_trees] or None, capped counts [n_gen] or None, report dict).
    fitness: a torch CUDA tensor of the parents' fitness, or None for the
    values of their last evaluation."""
    m = ctypes.c_int32()
    _check(_lib.ev_pop_info(ctx, parents, ctypes.byref(m), None))
    fh = np.zeros((n_gen, m.value), np.float32) if history else None
    ch = np.zeros(n_gen, np.int32) if history else None
    out = ctypes.c_int32()
    rep = ev_evolve_report()
    _check(_lib.ev_evolve(ctx, parents, _ptr(fitness), table, seed, gen0, n_gen, tournament, size_cap, flags,
                          ctypes.byref(out), _ptr(fh), _ptr(ch), ctypes.byref(rep)))
    return out.value, fh, ch, {k: getattr(rep, k) for k, _ in ev_evolve_report._fields_ if k != "pad"}


def ev_submit_eval(ctx, buf, off, table: int = 0) -> int:
    buf = np.ascontiguousarray(buf, np.uint8)
    off = np.ascontiguousarray(off, np.uint64)
    j = ev_job(kind=EV_JOB_EVAL, table=table, bytes=_ptr(buf), off=_ptr(off), n_trees=off.size - 1)
    return ev_submit(ctx, j)


def ev_submit_crossover(ctx, parents, mum, dad, p, q, table: int = 0, size_cap: int = 2**63) -> int:
    mum = np.ascontiguousarray(mum, np.int32)
    dad = np.ascontiguousarray(dad, np.int32)
    p = np.ascontiguousarray(p, np.uint64)
    q = np.ascontiguousarray(q, np.uint64)
    j = ev_job(kind=EV_JOB_CROSSOVER, table=table, parents=parents, mum=_ptr(mum), dad=_ptr(dad), p=_ptr(p),
               q=_ptr(q), n_children=mum.size, size_cap=size_cap)
    return ev_submit(ctx, j)


def ev_submit(ctx, job: ev_job) -> int:
    t = ctypes.c_uint64()
    _check(_lib.ev_submit(ctx, ctypes.byref(job), ctypes.byref(t)))
    return t.value


def ev_poll(ctx, ticket: int):
    done = ctypes.c_int32()
    st = ctypes.c_int32()
    _check(_lib.ev_poll(ctx, ticket, ctypes.byref(done), ctypes.byref(st)))
    return bool(done.value), st.value


def ev_wait(ctx, ticket: int) -> int:
    st = ctypes.c_int32()
    _check(_lib.ev_wait(ctx, ticket, ctypes.byref(st)))
    return st.value


def ev_result(ctx, ticket: int, n: int, N: int, per_case: bool = False):
    fit = np.empty(max(n, 1), np.float32)
    pc = np.empty((max(n, 1), N), np.float32) if per_case else None
    got = ctypes.c_int32()
    _check(_lib.ev_result(ctx, ticket, _ptr(fit), _ptr(pc), fit.size, ctypes.byref(got)))
    k = got.value
    return fit[:k], (pc[:k] if pc is not None else None)


def ev_job_timing(ctx, ticket: int):
    a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(_lib.ev_job_timing(ctx, ticket, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


def ev_get_plan_info(ctx, pop) -> dict:
    info = ev_plan_info()
    _check(_lib.ev_get_plan_info(ctx, pop, ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in ev_plan_info._fields_}


def ev_get_level_info(ctx, pop, level: int) -> dict:
    info = ev_level_info()
    _check(_lib.ev_get_level_info(ctx, pop, level, ctypes.byref(info)))
    return {k: getattr(info, k) for k, _ in ev_level_info._fields_ if k != "pad"}


def level_functions(ctx, pop) -> list:
    """Function nodes each plan level's launch evaluates (see ev.h)."""
    lv = [ev_get_level_info(ctx, pop, i) for i in range(ev_get_plan_info(ctx, pop)["levels"])]
    f = [(v["tokens"] - v["trees"]) // 2 for v in lv] + [0]
    return [f[i] - f[i + 1] for i in range(len(lv))]


EV_AUTOTUNE_NO_CACHE = 0x1
EV_EVOLVE_NO_GRAPH = 0x1
EV_EVOLVE_TEST_TIGHT = 0x2
EV_EVOLVE_LEAN = 0x4


def ev_autotune_ex(ctx, pop, table: int = 0, reps: int = 3, flags: int = 0) -> dict:
    """Search work-item sizes and the interpreter's waves per CU (see ev.h);
    the choice is applied to the context and cached per process."""
    t = ev_tune_choice()
    _check(_lib.ev_autotune_ex(ctx, pop, table, reps, flags, ctypes.byref(t)))
    return {k: getattr(t, k) for k, _ in ev_tune_choice._fields_}


def ev_tune_cache_save(path: str):
    _check(load_library().ev_tune_cache_save(path.encode()))


def ev_tune_cache_load(path: str):
    _check(load_library().ev_tune_cache_load(path.encode()))


EV_TUNE_NO_REGSTACK = 0x1
EV_TUNE_NO_RECORD = 0x2
EV_TUNE_NO_REUSE = 0x4
EV_TUNE_NO_CHAIN = 0x8
EV_TUNE_TEST_FAIL_CHECK = 0x100


def ev_set_tuning(ctx, chunk: int = 0, lds_depth: int = 0, flags: int = 0, chunk_hi: int = 0):
    _check(_lib.ev_set_tuning(ctx, chunk, chunk_hi, lds_depth, flags))


def ev_autotune(ctx, pop, table: int = 0, reps: int = 5):
    """Pick the fastest work-item size for pop (see ev.h); returns (chunk, ms)."""
    best = ctypes.c_uint32()
    ms = ctypes.c_float()
    _check(_lib.ev_autotune(ctx, pop, table, reps, ctypes.byref(best), ctypes.byref(ms)))
    return best.value, ms.value


def ev_last_level_times(ctx):
    """Device ms per plan level of the last ev_eval_fitness (a list)."""
    ms = (ctypes.c_float * 64)()
    n = ctypes.c_int32()
    _check(_lib.ev_last_level_times(ctx, ms, 64, ctypes.byref(n)))
    return [ms[i] for i in range(min(n.value, 64))]


def ev_last_timing(ctx):
    a = ctypes.c_float()
    b = ctypes.c_float()
    _check(_lib.ev_last_timing(ctx, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


# ------------------------------------------------------------ convenience

class Context:
    """Owns an ev_ctx; case table 0 is (x, y)."""

    def __init__(self, x, y, device: int = 0, mem_budget: int = 0, stream: int | None = None, allocator=None):
        self.allocator = allocator  # kept alive with the context
        self.ctx = ev_create(x, y, device, mem_budget, stream, allocator)
        _table_sizes[(self.ctx.value, 0)] = int(np.asarray(x).size)

    def add_cases(self, x, y) -> int:
        t = ev_add_cases(self.ctx, x, y)
        _table_sizes[(self.ctx.value, t)] = int(np.asarray(x).size)
        return t

    def n_cases(self, table: int = 0) -> int:
        return _table_sizes[(self.ctx.value, table)]

    def load(self, buf, off) -> int:
        return ev_load_trees(self.ctx, buf, off)

    def eval(self, pop, table: int = 0, per_case: bool = False, hits: bool = False):
        return ev_eval_fitness(self.ctx, pop, table, per_case, hits=hits)

    def close(self):
        if self.ctx is not None:
            ev_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
