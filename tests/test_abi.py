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
