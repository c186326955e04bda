"""Builds libgsopt.so (the gfx950 HIP library) next to this file with hipcc.

Each csrc/*.hip source is compiled to its own object in parallel (no device
code crosses a source file, so no relocatable device code is needed), then
the objects are linked into the shared library.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgsopt.so")
OBJ_DIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMPILE_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed-FP32 instructions in the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # a multiply and an add fuse only where one expression of the source
    # holds both, so an element's bits do not depend on the code around the
    # inlined update (the per-group and the packed passes agree bit for bit)
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-result",
    f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}",
]
LINK_FLAGS = [f"--offload-arch={ARCH}", "-shared", "-fPIC"]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _jobs() -> int:
    try:
        n = int(os.environ.get("MAX_JOBS", "0"))
    except ValueError:
        n = 0
    return max(1, min(n or (os.cpu_count() or 1), 16))


def compile_objects(srcs, flags, out_dir: str, verbose: bool):
    """hipcc -c of every source into out_dir, in parallel; returns the object paths."""
    os.makedirs(out_dir, exist_ok=True)

    def one(src):
        obj = os.path.join(out_dir, os.path.basename(src) + ".o")
        cmd = [HIPCC, *flags, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        # hipcc's host pass names the packed-FP32 feature it does not know: harmless
        noise = "'-packed-fp32-ops' is not a recognized feature"
        msg = "\n".join(line for line in (r.stdout + r.stderr).splitlines() if noise not in line)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{msg}")
        if msg.strip() and verbose:
            print(msg, flush=True)
        return obj

    with ThreadPoolExecutor(max_workers=_jobs()) as pool:
        return list(pool.map(one, srcs))


def link(out: str, objs, verbose: bool, extra=()) -> None:
    tmp = out + ".tmp"
    cmd = [HIPCC, *LINK_FLAGS, *extra, "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """Compile every csrc/.hip source and link libgsopt.so (always rebuilds)."""
    objs = compile_objects(sources(), COMPILE_FLAGS, OBJ_DIR, verbose)
    link(LIB, objs, verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
