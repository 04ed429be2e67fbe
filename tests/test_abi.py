"""The C-ABI library loads on any host and exports every declared entry point."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ev.h")
LIB = os.path.join(ROOT, "paper_1902_09215_amd", "libev.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ev_[a-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared()
    for need in ("ev_create", "ev_load_trees", "ev_eval_fitness", "ev_crossover", "ev_submit", "ev_poll"):
        assert need in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libev.so not built")
def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(ev_\w+)", out))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libev.so not built")
def test_library_loads_and_binding_matches_header():
    import paper_1902_09215_amd as ev

    lib = ev.load_library()
    for n in declared():
        assert hasattr(lib, n)
    assert sorted(ev.EXPORTS) == declared()


def header_constants():
    """Every EV_ constant the header defines, by #define or in an enum."""
    src = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    vals = {}
    for name, v in re.findall(r"#define\s+(EV_[A-Z0-9_]+)\s+(0x[0-9a-fA-F]+|\d+)u?\b", src):
        vals[name] = int(v, 0)
    for body in re.findall(r"enum\s*\{(.*?)\}", src, flags=re.S):
        for name, v in re.findall(r"(EV_[A-Z0-9_]+)\s*=\s*(-?\d+)", body):
            vals[name] = int(v)
    return vals


def test_binding_constants_match_header():
    # the binding restates the header's flags, status codes, opcodes and job
    # kinds for Python callers: they must agree (no library needed)
    import importlib.util

    spec = importlib.util.spec_from_file_location(
        "ev_binding_consts", os.path.join(ROOT, "paper_1902_09215_amd", "__init__.py"))
    src = open(spec.origin).read()
    vals = header_constants()
    assert len(vals) >= 20
    bound = {}
    for line in src.splitlines():
        m = re.match(r"^((?:EV_[A-Z0-9_]+\s*,\s*)*EV_[A-Z0-9_]+)\s*=\s*(.+)$", line)
        if not m:
            continue
        names = [n.strip() for n in m.group(1).split(",")]
        exprs = [e.strip() for e in m.group(2).split(",")]
        if len(names) == len(exprs):
            for n, e in zip(names, exprs):
                bound[n] = int(e, 0)
    missing = sorted(n for n in vals if n != "EV_H" and n not in bound)
    assert not missing, f"constants the binding does not define: {missing}"
    wrong = sorted(n for n in bound if n in vals and bound[n] != vals[n])
    assert not wrong, f"constants that disagree with the header: {wrong}"


@pytest.mark.skipif(not os.path.exists(LIB), reason="libev.so not built")
def test_tuning_cache_file_round_trip(tmp_path):
    # the autotuner's cache as text: loaded, saved and loaded again unchanged
    # (host code only), and a malformed line refused
    import paper_1902_09215_amd as ev

    ev.load_library()
    src = tmp_path / "tune.txt"
    src.write_text("# arch n_cases size_bin tree_bin chunk chunk_hi waves_per_cu ms\n"
                   "gfx950:sramecc+:xnack- 48 34 5 8192 16384 20 157.5\n"
                   "gfx950:sramecc+:xnack- 1024 20 3 2048 0 0 1.25\n")
    ev.ev_tune_cache_load(str(src))
    out = tmp_path / "out.txt"
    ev.ev_tune_cache_save(str(out))
    lines = [l for l in out.read_text().splitlines() if not l.startswith("#")]
    assert "gfx950:sramecc+:xnack- 48 34 5 8192 16384 20 157.5" in lines
    assert "gfx950:sramecc+:xnack- 1024 20 3 2048 0 0 1.25" in lines
    bad = tmp_path / "bad.txt"
    bad.write_text("gfx950 48 34 five 8192 16384 20 1.0\n")
    with pytest.raises(ev.EvError) as e:
        ev.ev_tune_cache_load(str(bad))
    assert e.value.code == ev.EV_EINVAL
    with pytest.raises(ev.EvError):
        ev.ev_tune_cache_load(str(tmp_path / "missing.txt"))
