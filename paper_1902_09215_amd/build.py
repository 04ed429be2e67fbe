"""Build libev.so (HIP, gfx950) in-tree."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["ev_kernels.hip", "ev_runtime.cpp", "ev_serve.cpp", "ev_static.hip", "ev_graph.cpp", "ev_lean.cpp"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # binary32 arithmetic exactly as written: no contraction, no fast math
    "-ffp-contract=off", "-fno-fast-math",
    # never form packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build(verbose: bool = False) -> str:
    import importlib.util

    spec = importlib.util.spec_from_file_location("gen_interp", os.path.join(CSRC, "gen_interp.py"))
    gen = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(gen)
    gen.write(os.path.join(CSRC, "ev_interp.inc"))
    out = os.path.join(HERE, "libev.so")
    tmp = out + ".tmp"
    cmd = ["hipcc", *FLAGS, "-o", tmp, *[os.path.join(CSRC, s) for s in SOURCES], "-lpthread"]
    res = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("libev build failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
