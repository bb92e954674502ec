"""Build the HIP library ``libtfft.so`` in-tree with hipcc for gfx950.

    python paper_2405_02520_amd/build.py [--resource-usage]

The two translation units are compiled in parallel and linked into a shared
library next to this file.  Every HIP source is built with packed FP32
instructions disabled (the compiler still vectorises nothing by hand).
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtfft.so")
ARCH = os.environ.get("TFFT_OFFLOAD_ARCH", "gfx950")

COMMON = [
    "hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]
SOURCES = ["tfft_kernels.hip", "tfft_plan.cpp"]


def _compile(src: str, obj: str, extra: list[str]) -> str:
    cmd = COMMON + extra + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-8000:]}")
    return r.stderr


def build(resource_usage: bool = False, verbose: bool = False, defines=(), lib: str | None = None) -> str:
    """Compile and link.  ``defines`` are extra -D options (compile-time
    configuration); ``lib`` is the output path (default: next to this file)."""
    out = lib or LIB
    objdir = os.path.join(os.path.dirname(out), "_build")
    os.makedirs(objdir, exist_ok=True)
    extra = ["-Rpass-analysis=kernel-resource-usage"] if resource_usage else []
    extra += [f"-D{d}" for d in defines]
    objs = [os.path.join(objdir, s + ".o") for s in SOURCES]
    with ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        logs = list(ex.map(lambda so: _compile(so[0], so[1], extra), zip(SOURCES, objs)))
    if resource_usage:
        with open(os.path.join(objdir, "resource_usage.log"), "w") as f:
            f.write("\n".join(logs))
    tmp = out + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr[-8000:]}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    defs = [a[2:] for a in sys.argv[1:] if a.startswith("-D")]
    outs = [a.split("=", 1)[1] for a in sys.argv[1:] if a.startswith("--out=")]
    build(resource_usage="--resource-usage" in sys.argv, verbose=True, defines=defs, lib=outs[0] if outs else None)
