"""The device-block cache against a host model of streams (CPU only).

The library keeps freed device blocks for reuse.  A block may be freed while
kernels queued on the freeing stream still use it; the cache must never hand
it to another stream before that stream has been waited for.  The model in
``native/cache_model.cpp`` drives the cache's own code (``ev_cache.h``) with a
scripted case (plan scratch freed while its placement kernel is queued, then
wanted by another worker's stream) and random walks over several streams.
"""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_cache_never_hands_a_block_in_use_to_another_stream(tmp_path):
    exe = tmp_path / "cache_model"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror",
                    "-I", os.path.join(ROOT, "paper_1902_09215_amd", "csrc"),
                    "-o", str(exe), os.path.join(ROOT, "tests", "native", "cache_model.cpp")], check=True)
    res = subprocess.run([str(exe)], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-2000:]
    assert int(res.stdout.strip()) > 1000  # hand-outs that were checked
