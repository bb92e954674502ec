"""Build the HIP library ``libtfft.so`` in-tree with hipcc for gfx950.

    python paper_2405_02520_amd/build.py [--resource-usage] [-DNAME=VALUE ...] [--out=PATH]

The kernels are instantiated per (element type, pass length): ``tfft_inst.hip``
is compiled once for each pair, in parallel with the dispatch unit and the
host code, and the objects are linked into a shared library next to this
file.  Every HIP source is built with packed FP32 instructions disabled (the
compiler still vectorises nothing by hand).
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
# (source, extra defines, object name)
LENGTHS = [2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048, 4096, 8192]
UNITS = [("tfft_kernels.hip", [], "tfft_kernels"), ("tfft_plan.cpp", [], "tfft_plan"),
         ("tfft_scratch.hip", [], "tfft_scratch")] + [
    ("tfft_inst.hip", [f"-DTFFT_INST_R={r}", f"-DTFFT_INST_M={m}"], f"tfft_inst_{r}_{m}")
    for r in ("float", "double") for m in LENGTHS] + [
    ("tfft_persist_inst.hip", [f"-DTFFT_INST_R={r}", f"-DTFFT_INST_FT={ft}"], f"tfft_persist_{r}_{ft}")
    for r in ("float", "double") for ft in ("FT_NONE", "FT_BLOCK")]


def _compile(src: str, defs: list[str], obj: str, extra: list[str]) -> str:
    cmd = COMMON + extra + defs + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src} {' '.join(defs)}:\n{r.stderr[-8000:]}")
    return r.stderr


def build(resource_usage: bool = False, verbose: bool = False, defines=(), lib: str | None = None) -> str:
    """Compile and link.  ``defines`` are extra -D options (compile-time
    configuration); ``lib`` is the output path (default: next to this file)."""
    out = lib or LIB
    objdir = os.path.join(os.path.dirname(out), "_build")
    os.makedirs(objdir, exist_ok=True)
    extra = ["-Rpass-analysis=kernel-resource-usage"] if resource_usage else []
    extra += [f"-D{d}" for d in defines]
    objs = [os.path.join(objdir, name + ".o") for _, _, name in UNITS]
    jobs = int(os.environ.get("MAX_JOBS", "0")) or os.cpu_count() or 4
    # the longest units first
    order = sorted(range(len(UNITS)), key=lambda i: -max([int(d.split("=")[1]) for d in UNITS[i][1]
                                                          if d.startswith("-DTFFT_INST_M")] or
                                                         [16384 if "persist" in UNITS[i][2] else 8192]))
    with ThreadPoolExecutor(max_workers=min(jobs, len(UNITS))) as ex:
        futs = {i: ex.submit(_compile, UNITS[i][0], UNITS[i][1], objs[i], extra) for i in order}
        logs = [futs[i].result() for i in range(len(UNITS))]
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
