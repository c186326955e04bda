"""The benchmark's streaming-ceiling kernels (stream_probe.hip), built into
libgsprobe.so next to this file.  Measurement support for bench.py only:
the AdamW-GS library (paper_2601_16736_amd) neither builds nor links it."""
from __future__ import annotations

import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "stream_probe.hip")
LIB = os.path.join(HERE, "libgsprobe.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # no packed-FP32 instructions in the generated code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall"]


def build(verbose: bool = False) -> str:
    """Compile stream_probe.hip into libgsprobe.so (always rebuilds)."""
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def load():
    """The library with its argument types set (OSError if it is not built)."""
    lib = ctypes.CDLL(LIB)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    lib.gsprobe_rmw_4r3w.argtypes = [vp, vp, vp, vp, i64, vp]
    lib.gsprobe_copy.argtypes = [vp, vp, i64, vp]
    lib.gsprobe_read.argtypes = [vp, i64, vp, vp]
    lib.gsprobe_rmw_4r3w_cfg.argtypes = [vp, vp, vp, vp, i64, i32, i32, i32, i32, i32, vp]
    lib.gsprobe_copy_cfg.argtypes = [vp, vp, i64, i32, i32, i32, i32, i32, vp]
    lib.gsprobe_read_cfg.argtypes = [vp, i64, vp, i32, i32, i32, i32, vp]
    pp = ctypes.POINTER(ctypes.c_void_p)
    lib.gsprobe_rows_4r3w.argtypes = [vp, vp, pp, pp, pp, pp, ctypes.POINTER(ctypes.c_int32), i32, i64, vp]
    lib.gsprobe_rows_4r3w_cfg.argtypes = [vp, vp, pp, pp, pp, pp, ctypes.POINTER(ctypes.c_int32), i32, i64, i32, i32,
                                          i32, vp]
    return lib
