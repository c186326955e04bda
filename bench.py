"""Benchmark of the AdamW-GS hot path on one MI355X.

Workload: the 3M-primitive scene -- 3,000,000 Gaussians with 59 FP32
attributes each (mean 3, log-scale 3, quaternion 4, opacity logit 1, SH 48),
means uniform in [-10, 10]^3, every other attribute N(0, 1); 200 cameras on
a radius-15 Fibonacci sphere looking at the origin (60 deg FOV, 1000 x 1000,
z_near 0.2, z_far 17.5), one camera per step from a seeded shuffle; photometric
gradients N(0, 1e-3) (four pre-drawn sets, rotated per step); DAR with
lambda_o = 1e-3, lambda_s = 1e-5, C = 10, N_I' = 1e5; RSR every 100 iterations
with p = 0.05, alpha = (0.2, 0.04).

Layout: before timing, the scene is put in spatial (Morton) order with the
library's gs_spatial_order + gs_gather_rows, so that a view's visible rows
form contiguous index runs (--order index keeps the generated order).

One step = visibility of the view, Re-State rescale (on RSR iterations) and
the fused Sparse-Adam + DAR pass, all in the HIP library.  By default the
three run in one launch (adamw_gs_step_view: each wave culls a window of 32
primitives and steps its visible rows); --path two_launch times gs_visibility
(mask, index list and count) followed by the masked step (windows of 32)
instead.  The two-launch
path always runs first: it is reported as a variant, and its per-step visible
counts are the fused path's too, since the two end in bit-identical states
(checked after the runs).  Inputs are resident in HBM before timing starts.
The metric is attribute updates per second (visible primitives x 59 per step
/ wall time of the steps).  The JSON line also carries the roofline of the
dominant kernel measured with HIP events on the launch stream, the FP64
oracle timed on the host over a bounded sample of the same workload, and the
other layouts / moment precisions measured the same way ("variants"), and
the streaming ceilings of plain contiguous kernels on the same device
("stream_ceiling": the step's 4-read / 3-write mix, a copy and a read).

Usage: python bench.py [--gpus 1] [--steps 1000] [--warmup 20] [--path view|two_launch]
       [--order morton|index] [--moments f32|bf16] [--no-variants] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

# Launch configuration of the fused step in the benchmark (the full-size
# parity test runs the same one).
STEP_LAUNCH = {"schedule": 2, "unit": 32}           # masked schedule, windows of 32 primitives

N_PRIMS = 3_000_000
MCMC_N = 6_000_000                 # the MCMC-shaped workload's cap
BATCH_SIZE_RANGE = (2e5, 4e6)      # the batched workload's scene sizes (log-uniform)
DEVICE = "cuda:0"
# the unfused comparator is checked against the fused step before it is timed
CHECK_UNFUSED = True
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per visible primitive of the step: theta r/w, g r, m r/w,
# v r/w over 59 elements; t r/w
BYTES_PER_VISIBLE = {"f32": 59 * (4 + 4 + 4 + 4 + 4 + 4 + 4) + 8,          # 1660
                     "bf16": 59 * (4 + 4 + 4 + 2 + 2 + 2 + 2) + 8}         # 1188
# and per primitive of the scene: the masked step reads its mask byte; the
# fused view step reads its mean once more for the cull
BYTES_PER_PRIMITIVE = {"two_launch": 1, "view": 12}
LAMBDA_O, LAMBDA_S, CLIP, REG_NORM = 1e-3, 1e-5, 10.0, 1e5
RSR_EVERY, RSR_P, RSR_A1, RSR_A2 = 100, 0.05, 0.2, 0.04
N_GRAD_SETS = 4
GS_F32, GS_BF16 = 0, 1               # moment dtypes (gs_moment_dtype)
# primitives per wave window in the fused view step: 0 = the library's
# default, 32 on plain steps and 64 on Re-State iterations
VIEW_UNIT = 0
STATE_WARMUP_STEPS = 20                 # discarded steps on a leg's own buffers before its warm-up (state reset after)
# HBM counter summaries per path, and the sources of the kernel each covers
TRAFFIC_FILES = {"view": os.path.join(ROOT, "profiles", "step_view_kernel_3M_traffic.json"),
                 "two_launch": os.path.join(ROOT, "profiles", "step_kernel_3M_traffic.json")}
KERNEL_SOURCES = {"view": ("internal.h", "device_common.h", "predicate.h", "step_view.hip"),
                  "two_launch": ("internal.h", "device_common.h", "step.hip")}


class TimingEvents:
    """Pairs of HIP events for timing kernels on a stream.  They are created
    with hipEventDisableSystemFence: a default timing event writes back and
    invalidates the caches at each record, which costs several microseconds
    between back-to-back kernels and would be charged to the step being
    timed.  Read them only after a device synchronization."""

    FLAGS = 0x20000000            # hipEventDisableSystemFence (hip_runtime_api.h)

    def __init__(self, count: int):
        import ctypes
        import torch  # noqa: F401  (its HIP runtime is the one loaded)
        self._hip = ctypes.CDLL("libamdhip64.so.7")
        self._hip.hipEventCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
        self._hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        self._hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self._hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self._ctypes = ctypes
        self.start, self.end = [], []
        for lst in (self.start, self.end):
            for _ in range(count):
                e = ctypes.c_void_p()
                if self._hip.hipEventCreateWithFlags(ctypes.byref(e), self.FLAGS) != 0:
                    raise RuntimeError("hipEventCreateWithFlags failed")
                lst.append(e)

    def record(self, which: str, slot: int, stream) -> None:
        ev = (self.start if which == "start" else self.end)[slot]
        if self._hip.hipEventRecord(ev, self._ctypes.c_void_p(int(stream.cuda_stream))) != 0:
            raise RuntimeError("hipEventRecord failed")

    def ms(self, slot: int) -> float:
        out = self._ctypes.c_float()
        if self._hip.hipEventElapsedTime(self._ctypes.byref(out), self.start[slot], self.end[slot]) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(out.value)

    def close(self) -> None:
        for e in self.start + self.end:
            self._hip.hipEventDestroy(e)
        self.start, self.end = [], []


def kernel_source_hash(path: str = "view") -> str:
    """Hash of the kernel's sources and of the library's build script (its
    compiler flags shape the machine code too)."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[path]:
        with open(os.path.join(ROOT, "paper_2601_16736_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    with open(os.path.join(ROOT, "paper_2601_16736_amd", "build.py"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(order: str, moments: str, path: str = "view"):
    """HBM bytes per launch of the path's dominant kernel from the committed
    rocprofv3 counter summary, if it was taken on the current kernel source
    and layout."""
    try:
        with open(TRAFFIC_FILES[path]) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if (d.get("source_hash") != kernel_source_hash(path) or d.get("order") != order
            or d.get("moments") != moments):
        return None
    return d.get("bytes_per_launch")


def host_cores() -> int:
    """Host threads the CPU baseline uses: the cores this process may run on,
    at most 16 (one GPU's share of a shared host)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(scene, cams, order, budget_s: float = 12.0, sample_n: int = 0, cores: int = 0):
    """The FP64 oracle, unchanged, on the same scene, cameras and
    hyper-parameters: each step is the visibility predicate of the step's
    view and the AdamW-GS step.  The primitives are split into one
    contiguous shard per host thread (every primitive's step depends only on
    its own rows; each shard passes its rows' scene indices, so the Re-State
    draws are those of the unsharded step), and the threads run the oracle's
    C functions concurrently (ctypes releases the GIL during a call).  Steps
    run until half the budget is spent on all `cores` threads, then until the
    other half is spent on one thread, from where the first run stopped.
    sample_n = 0 takes the whole scene."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    from synth import GROUPS_59
    n = scene.n if sample_n <= 0 else min(sample_n, scene.n)
    cores = cores or host_cores()
    groups = []
    for name, dim, lr, dar in GROUPS_59:
        p = np.ascontiguousarray(scene.params[name][:n], dtype=np.float64)
        groups.append(oracle.Group(p, np.zeros_like(p), np.zeros_like(p), np.zeros_like(p), lr, dar_kind=dar,
                                   dar_lambda=LAMBDA_O if dar == 1 else LAMBDA_S, dar_clip=CLIP))
    t = np.zeros(n, np.int32)
    rng = np.random.default_rng(1234)
    for G in groups:
        G.grad[:] = 1e-3 * rng.standard_normal(G.grad.shape)

    def shards(k):
        bounds = np.linspace(0, n, k + 1).astype(np.int64)
        out = []
        for a, b in zip(bounds[:-1], bounds[1:]):
            if b > a:
                sub = [oracle.Group(G.param[a:b], G.grad[a:b], G.m[a:b], G.v[a:b], G.lr, dar_kind=G.dar_kind,
                                    dar_lambda=G.dar_lambda, dar_clip=G.dar_clip) for G in groups]
                out.append((sub, t[a:b], np.arange(a, b, dtype=np.int64)))
        return out

    def one_shard(sh, cam, cfg):
        sub, ts, ids = sh
        mask = oracle.visibility(sub[0].param.astype(np.float32), cam)
        oracle.adamw_gs_step(sub, len(ids), mask, ts, cfg, ids=ids)
        return int(mask.sum())

    step = 0

    def run(k_threads, budget):
        nonlocal step
        parts = shards(k_threads)
        updates, elapsed, steps = 0, 0.0, 0
        with ThreadPoolExecutor(max_workers=k_threads) as pool:
            while elapsed < budget:
                c = cams[order[step % len(order)]]
                cam = oracle.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far)
                cfg = oracle.Config(reg_norm=REG_NORM, seed=0, iteration=step, rsr_enable=step % RSR_EVERY == 0,
                                    rsr_ratio=RSR_P, rsr_alpha1=RSR_A1, rsr_alpha2=RSR_A2)
                t0 = time.perf_counter()
                vis = sum(pool.map(lambda sh: one_shard(sh, cam, cfg), parts))
                elapsed += time.perf_counter() - t0
                updates += vis * 59
                steps += 1
                step += 1
        return updates / elapsed, steps, elapsed

    v_all, s_all, e_all = run(cores, budget_s / 2)
    v_one, s_one, e_one = run(1, budget_s / 2)
    return {"value": v_all, "unit": "attr-updates/s", "cores": cores, "kind": "oracle",
            "value_1_thread": v_one, "speedup_over_1_thread": v_all / v_one,
            "sample": f"{n} primitives of the scene (index order), visibility + step per step; "
                      f"{s_all} steps in {e_all:.1f} s on {cores} threads (one contiguous shard each), "
                      f"then {s_one} steps in {e_one:.1f} s on 1 thread"}


def calibrate_copy(nbytes: int = 1 << 30, reps: int = 10) -> int:
    """A plain device-to-device copy of known size, for scaling the HBM byte
    counters (FETCH_SIZE, WRITE_SIZE) of a profiled run."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device=DEVICE)
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        y.copy_(x)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps,
                      "copy_GBps_rw": 2 * nbytes / dt / 1e9}), flush=True)
    return 0


PROBE_DEFAULT = (16, 4, 1, 1, 0)          # width, items, nt_load, nt_store, blocks
# nt_load 2: the hint only on the loads of arrays that are written back
PROBE_SHAPES = [(w, it, ntl, nts, b) for w in (16, 8) for it in (2, 4, 8, 16) for ntl in (1, 0, 2) for nts in (1, 0)
                for b in (0, 1024, 2048)]


def stream_ceilings(torch, nbytes: int = 1 << 30, reps: int = 20, shapes=None, stagger: int = 0) -> dict:
    """Bandwidth of plain contiguous kernels on this device (bench_probe):
    the step's 4-read / 3-write mix over four arrays of `nbytes`, a copy and
    a read, each timed with HIP events over `reps` launches after 3 untimed
    ones, for every launch shape in `shapes` (access width, accesses in
    flight per thread, non-temporal hints on loads / stores, one-shot or
    resident grid).  Reports the fixed default shape and the best shape of
    each mix.  Each array is 1 GiB by default, four times the 256 MB
    Infinity Cache: with 256 MiB arrays, an array loaded without the
    non-temporal hint stays partly in that cache from one launch to the
    next, and such shapes then read above what the HBM delivers.
    stagger = 0: four separate allocations;
    > 0: one allocation holding array k at offset k * (nbytes + stagger),
    so the arrays' element i sit at different offsets modulo any power of
    two up to stagger's lowest set bit."""
    import bench_probe
    lib = bench_probe.load()
    vp = __import__("ctypes").c_void_p
    dev = torch.device(DEVICE)
    if stagger > 0:
        if stagger % 16:
            raise ValueError("stagger must be a multiple of 16 bytes")
        pitch = (nbytes + stagger) // 4
        whole = torch.rand(4 * pitch, device=dev)
        arrs = [whole[k * pitch:k * pitch + nbytes // 4] for k in range(4)]
    else:
        arrs = [torch.rand(nbytes // 4, device=dev) for _ in range(4)]
    sink = torch.zeros(4, device=dev)
    n16 = nbytes // 16
    stream = torch.cuda.current_stream()
    sp = vp(stream.cuda_stream)
    ptr = [a.data_ptr() for a in arrs]
    shapes = PROBE_SHAPES if shapes is None else shapes
    if PROBE_DEFAULT not in shapes:
        shapes = [PROBE_DEFAULT] + list(shapes)

    def timed(fn) -> float:
        ev = TimingEvents(reps)
        for _ in range(3):
            if fn() != 0:
                raise RuntimeError("gsprobe launch failed")
        for j in range(reps):
            ev.record("start", j, stream)
            fn()
            ev.record("end", j, stream)
        torch.cuda.synchronize()
        sec = float(np.mean([ev.ms(j) for j in range(reps)])) * 1e-3
        ev.close()
        return sec

    table = {"rmw_4r3w": {}, "copy": {}, "read": {}}
    for (w, it, ntl, nts, b) in shapes:
        key = f"w{w}_i{it}_ntl{ntl}_nts{nts}_b{b}"
        table["rmw_4r3w"][key] = 7 * nbytes / timed(
            lambda: lib.gsprobe_rmw_4r3w_cfg(ptr[0], ptr[1], ptr[2], ptr[3], n16, w, it, ntl, nts, b, sp)) / 1e9
        if ntl == 2:                    # copy and read write back nothing they read
            continue
        table["copy"][key] = 2 * nbytes / timed(
            lambda: lib.gsprobe_copy_cfg(ptr[0], ptr[1], n16, w, it, ntl, nts, b, sp)) / 1e9
        if nts == 1:                    # a read has no stores: one entry per load hint
            table["read"][key] = nbytes / timed(
                lambda: lib.gsprobe_read_cfg(ptr[0], n16, sink.data_ptr(), w, it, ntl, b, sp)) / 1e9
    dkey = "w{}_i{}_ntl{}_nts{}_b{}".format(*PROBE_DEFAULT)
    out = {}
    for mix, t in table.items():
        best = max(t, key=t.get)
        out[f"{mix}_GBps"] = t[dkey]
        out[f"{mix}_best_GBps"] = t[best]
        out[f"{mix}_best_shape"] = best
    out["shapes_timed"] = len(shapes)
    out["default_shape"] = dkey
    out["stagger"] = stagger
    out["array_bytes"] = nbytes
    out["table"] = table
    del arrs, sink
    torch.cuda.empty_cache()
    return out


ROWS_PROBE_SHAPES = [(w, it) for w in (32, 64, 128, 256) for it in (2, 4, 8)]


def rows_ceiling(gs, torch, sd: SceneOnDevice, cams, order, steps: int = 50, warmup: int = 5,
                 shapes=None, moments: str = "f32") -> dict:
    """The masked step's own access pattern with no method arithmetic
    (bench_probe rows_kernel): per step, gs_visibility writes the camera's
    mask (not timed), then the probe reads and writes exactly the rows and
    bytes the masked FP32 step does (the five groups' four arrays, the step
    counters), timed with HIP events, for each launch shape (window of
    primitives per wave, chunk items in flight per lane) in `shapes`, with
    FP32 or BF16 moment arrays.  Same accounting as the step:
    BYTES_PER_VISIBLE per visible row plus 1 B of mask per primitive.  The ratio of a step kernel's bandwidth to the best
    shape's is how close it comes to what its access pattern allows."""
    import ctypes

    import bench_probe
    import synth
    shapes = list(shapes or ROWS_PROBE_SHAPES)
    dev = torch.device(DEVICE)
    lib = bench_probe.load()
    arrs = []
    mdt = torch.bfloat16 if moments == "bf16" else torch.float32
    for (name, dim, lr, dar), p, sets in zip(synth.GROUPS_59, sd.params, sd.grads):
        arrs.append((p.clone(), sets[0], torch.zeros(p.shape, dtype=mdt, device=dev),
                     torch.zeros(p.shape, dtype=mdt, device=dev)))
    t = torch.zeros(N_PRIMS, dtype=torch.int32, device=dev)
    mask = torch.zeros(N_PRIMS, dtype=torch.uint8, device=dev)
    idx = torch.zeros(N_PRIMS, dtype=torch.int32, device=dev)
    total = warmup + steps
    counts = torch.zeros(total, dtype=torch.int32, device=dev)
    ng = len(arrs)
    ptrs = [(ctypes.c_void_p * ng)(*[a[k].data_ptr() for a in arrs]) for k in range(4)]
    dims = (ctypes.c_int32 * ng)(*[a[0].shape[1] for a in arrs])
    gcams = [gs.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far) for c in cams]
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    means = sd.params[0]
    table = {}
    nv = None
    for (win, items) in shapes:
        ev = TimingEvents(steps)
        for k in range(total):
            gs.gs_visibility(means, gcams[order[k % len(order)]], mask=mask, vis_idx=idx,
                             vis_count=counts[k:k + 1], stream=stream)
            j = k - warmup
            if j >= 0:
                ev.record("start", j, stream)
            rc = lib.gsprobe_rows_4r3w_cfg(ctypes.c_void_p(mask.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                           ptrs[0], ptrs[1], ptrs[2], ptrs[3], dims, ng, N_PRIMS, win, items,
                                           int(moments == "bf16"), sp)
            if rc != 0:
                raise RuntimeError(f"gsprobe_rows_4r3w_cfg returned {rc}")
            if j >= 0:
                ev.record("end", j, stream)
        torch.cuda.synchronize()
        durs = np.array([ev.ms(j) for j in range(steps)]) * 1e-3
        ev.close()
        nv = counts.cpu().numpy().astype(np.int64)[warmup:]
        byts = nv * BYTES_PER_VISIBLE[moments] + N_PRIMS * BYTES_PER_PRIMITIVE["two_launch"]
        table[f"win{win}_i{items}"] = {"GBps": float(byts.sum() / durs.sum()) / 1e9, "us": float(durs.mean() * 1e6)}
    del arrs, t, mask, idx
    torch.cuda.empty_cache()
    best = max(table, key=lambda k: table[k]["GBps"])
    step_shape = "win32_i4"
    return {"moments": moments,
            "GBps": table[step_shape]["GBps"] if step_shape in table else None,
            "us": table[step_shape]["us"] if step_shape in table else None,
            "best_GBps": table[best]["GBps"], "best_shape": best, "table": table,
            "visible_mean": float(nv.mean()), "steps": steps,
            "kind": "masked-step access pattern without arithmetic (bench_probe rows_kernel): the five groups' "
                    "attribute, gradient and moment arrays and the step counters; GBps: windows of 32, 4 chunk "
                    "items in flight; best: fastest of windows 32-256 x 2-8 items; "
                    f"{BYTES_PER_VISIBLE[moments]} B per visible + 1 B of mask per primitive"}


def gpu_clocks():
    """Current GPU clock levels from the amdgpu driver's sysfs files (the run
    does not pin them), or None where they cannot be read.  Plain file
    reads: no helper program is started."""
    out = {}
    for path in sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_[sm]clk")):
        try:
            with open(path) as f:
                cur = [line.strip() for line in f if line.strip().endswith("*")]
        except OSError:
            continue
        if cur:
            card = path.split("/")[4]
            out[f"{card}:{os.path.basename(path)[7:]}"] = cur[0].rstrip("* ").split(":", 1)[-1].strip()
    return out or None


class SceneOnDevice:
    """The scene's attributes and gradient sets in HBM, in a chosen order."""

    def __init__(self, gs, torch, scene, order: str):
        import synth
        dev = torch.device(DEVICE)
        self.params = [torch.from_numpy(scene.params[name]).to(dev) for name, *_ in synth.GROUPS_59]
        gen = torch.Generator(device=dev)
        gen.manual_seed(0)
        self.grads = [[torch.randn((N_PRIMS, dim), generator=gen, device=dev) * 1e-3 for _ in range(N_GRAD_SETS)]
                      for _, dim, _, _ in synth.GROUPS_59]
        self.order = order
        if order == "morton":
            perm = torch.empty(N_PRIMS, dtype=torch.int32, device=dev)
            ws = torch.empty(gs.gs_spatial_order_workspace_size(N_PRIMS), dtype=torch.uint8, device=dev)
            gs.gs_spatial_order(self.params[0], perm, ws)
            self.params = gs.apply_spatial_order(self.params, perm)
            self.grads = [gs.apply_spatial_order(sets, perm) for sets in self.grads]
            del ws, perm
        torch.cuda.synchronize()


def device_warmup(gs, torch, sd: SceneOnDevice, cams, seconds: float = 1.0) -> int:
    """Brings the device to its working clocks before anything is timed: the
    fused view step on a scratch copy of the scene's state, stepped through
    the camera rig until `seconds` of wall time have passed.  Nothing it
    computes is kept.  Returns the number of steps taken."""
    import synth
    dev = torch.device(DEVICE)
    groups = [gs.Group(p.clone(), sets[0], torch.zeros_like(p), torch.zeros_like(p), lr, dar_kind=dar,
                       dar_lambda=LAMBDA_O if dar == 1 else (LAMBDA_S if dar == 2 else 0.0), dar_clip=CLIP)
              for (name, dim, lr, dar), p, sets in zip(synth.GROUPS_59, sd.params, sd.grads)]
    t = torch.zeros(N_PRIMS, dtype=torch.int32, device=dev)
    gcams = [gs.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far) for c in cams]
    stream = torch.cuda.current_stream()
    k = 0
    t0 = time.perf_counter()
    while True:
        for _ in range(50):
            cfg = gs.StepConfig(reg_norm=REG_NORM, seed=7, iteration=k, unit=VIEW_UNIT)
            gs.adamw_gs_step_view(groups, N_PRIMS, t, cfg, groups[0].param, gcams[k % len(gcams)], stream=stream)
            k += 1
        torch.cuda.synchronize()
        if time.perf_counter() - t0 >= seconds:
            break
    del groups, t
    return k


def run_steps(gs, torch, sd: SceneOnDevice, cams, order, moments: str, steps: int, warmup: int,
              path: str = "two_launch", counts_from=None, keep_state: bool = False):
    """Times `steps` whole steps (after `warmup`) on fresh optimizer state.
    path "two_launch": gs_visibility (mask, index list and count) then the
    masked step; "view": adamw_gs_step_view, visibility fused into the step (one
    launch, the library's default windows).  The fused path writes no count, so its visible
    counts are taken from a two-launch run on the same cameras (`counts_from`),
    whose results are bit-identical."""
    import synth
    dev = torch.device(DEVICE)
    mdt = torch.bfloat16 if moments == "bf16" else torch.float32
    groups = []
    for (name, dim, lr, dar), p, sets in zip(synth.GROUPS_59, sd.params, sd.grads):
        groups.append(gs.Group(p.clone(), sets[0], torch.zeros((N_PRIMS, dim), dtype=mdt, device=dev),
                               torch.zeros((N_PRIMS, dim), dtype=mdt, device=dev), lr, dar_kind=dar,
                               dar_lambda=LAMBDA_O if dar == 1 else (LAMBDA_S if dar == 2 else 0.0),
                               dar_clip=CLIP))
    total = warmup + steps
    t = torch.zeros(N_PRIMS, dtype=torch.int32, device=dev)
    mask = torch.zeros(N_PRIMS, dtype=torch.uint8, device=dev)
    idx = torch.zeros(N_PRIMS, dtype=torch.int32, device=dev)
    counts = torch.zeros(total, dtype=torch.int32, device=dev)
    gcams = [gs.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far) for c in cams]
    means = groups[0].param
    stream = torch.cuda.current_stream()
    ev = TimingEvents(1 if path == "view" else steps)
    mom = gs.GS_MOMENT_BF16 if moments == "bf16" else gs.GS_MOMENT_F32

    def one_step(k: int, slot: int = -1):
        cnt = counts[k:k + 1]
        gs.gs_visibility(means, gcams[order[k % len(order)]], mask=mask, vis_idx=idx, vis_count=cnt, stream=stream)
        for G, sets in zip(groups, sd.grads):
            G.grad = sets[k % N_GRAD_SETS]
        cfg = gs.StepConfig(reg_norm=REG_NORM, seed=0, iteration=k, rsr_enable=(k % RSR_EVERY == 0),
                            rsr_ratio=RSR_P, rsr_alpha1=RSR_A1, rsr_alpha2=RSR_A2, moment_dtype=mom,
                            stochastic_round=True, **STEP_LAUNCH)
        if slot >= 0:
            ev.record("start", slot, stream)
        gs.adamw_gs_step(groups, N_PRIMS, t, cfg, visible=mask, vis_idx=idx, vis_count=cnt, stream=stream)
        if slot >= 0:
            ev.record("end", slot, stream)

    def one_view_step(k: int, slot: int = -1):
        for G, sets in zip(groups, sd.grads):
            G.grad = sets[k % N_GRAD_SETS]
        cfg = gs.StepConfig(reg_norm=REG_NORM, seed=0, iteration=k, rsr_enable=(k % RSR_EVERY == 0),
                            rsr_ratio=RSR_P, rsr_alpha1=RSR_A1, rsr_alpha2=RSR_A2, moment_dtype=mom,
                            stochastic_round=True, unit=VIEW_UNIT)
        if slot >= 0:
            ev.record("start", slot, stream)
        gs.adamw_gs_step_view(groups, N_PRIMS, t, cfg, means, gcams[order[k % len(order)]], stream=stream)
        if slot >= 0:
            ev.record("end", slot, stream)

    if path == "view":
        if counts_from is None:
            raise ValueError("the fused path needs the visible counts of a two-launch run")
        one_step = one_view_step  # noqa: F811

    region = path == "view"
    if region:
        # each timed step's arguments are packed on the host first, before
        # the warm-up (adamw_gs_step_view marshals tens of microseconds of
        # Python per call; in a loop that runs ahead of the device this
        # overlaps the previous step, but the first call after the timer's
        # synchronization would leave the device idle that long, and packing
        # them all between the warm-up and the timer would idle it longer
        # still, letting its clocks fall)
        launches = []
        for j in range(steps):
            k = warmup + j
            for G, sets in zip(groups, sd.grads):
                G.grad = sets[k % N_GRAD_SETS]
            cfg = gs.StepConfig(reg_norm=REG_NORM, seed=0, iteration=k, rsr_enable=(k % RSR_EVERY == 0),
                                rsr_ratio=RSR_P, rsr_alpha1=RSR_A1, rsr_alpha2=RSR_A2, moment_dtype=mom,
                                stochastic_round=True, unit=VIEW_UNIT)
            launches.append(gs.prepare_step_view(groups, N_PRIMS, t, cfg, means, gcams[order[k % len(order)]],
                                                 stream=stream))
    # The leg's own buffers first take STATE_WARMUP_STEPS discarded steps
    # (device clocks fall while the host sets the leg up, and take about 20
    # steps to come back), then the state is reset by copies: the warm-up and
    # timed steps below start from exactly the state they would without it.
    for k in range(STATE_WARMUP_STEPS):
        one_step(k % total)
    for G, p in zip(groups, sd.params):
        G.param.copy_(p)
        G.exp_avg.zero_()
        G.exp_avg_sq.zero_()
    t.zero_()
    for k in range(warmup):
        one_step(k)
    torch.cuda.synchronize()
    # The fused path launches one kernel per step, so one pair of events
    # around the timed steps gives its average launch duration: a pair per
    # step would put an event record between every two launches (about 8 us
    # of idle each) into the very time being measured.  The two-launch path
    # brackets its step kernel in every step, apart from the visibility
    # launches.
    t0 = time.perf_counter()
    if region:
        ev.record("start", 0, stream)
        for launch in launches:
            launch()
        ev.record("end", 0, stream)
    else:
        for j in range(steps):
            one_step(warmup + j, j)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    all_counts = counts.cpu().numpy().astype(np.int64) if path != "view" else np.asarray(counts_from)
    nv = all_counts[warmup:warmup + steps]
    spread = None
    if region:
        durs = np.full(steps, ev.ms(0) * 1e-3 / steps)
        plain = np.ones(steps, dtype=bool)      # Re-State steps included (their extra rows not counted)
        # the per-step spread, from a separate pass over the same steps (cameras, iterations, gradient
        # sets) on a copy of the state, with a pair of events around each launch; not part of the timing
        # above, and the state compared with the two-launch path is untouched
        copies = [gs.Group(G.param.clone(), G.grad, G.exp_avg.clone(), G.exp_avg_sq.clone(), G.lr,
                           dar_kind=G.dar_kind, dar_lambda=G.dar_lambda, dar_clip=G.dar_clip) for G in groups]
        t_copy = t.clone()
        ev2 = TimingEvents(steps)
        for j in range(steps):
            k = warmup + j
            for G, sets in zip(copies, sd.grads):
                G.grad = sets[k % N_GRAD_SETS]
            cfg = gs.StepConfig(reg_norm=REG_NORM, seed=0, iteration=k, rsr_enable=(k % RSR_EVERY == 0),
                                rsr_ratio=RSR_P, rsr_alpha1=RSR_A1, rsr_alpha2=RSR_A2, moment_dtype=mom,
                                stochastic_round=True, unit=VIEW_UNIT)
            ev2.record("start", j, stream)
            gs.adamw_gs_step_view(copies, N_PRIMS, t_copy, cfg, copies[0].param, gcams[order[k % len(order)]],
                                  stream=stream)
            ev2.record("end", j, stream)
        torch.cuda.synchronize()
        each = np.array([ev2.ms(j) for j in range(steps)]) * 1e3
        ev2.close()
        keep = np.array([(warmup + j) % RSR_EVERY != 0 for j in range(steps)])
        spread = [float(x) for x in np.percentile(each[keep] if keep.any() else each, [10, 50, 90])]
        del copies, t_copy
    else:
        durs = np.array([ev.ms(j) for j in range(steps)]) * 1e-3
        plain = np.array([(warmup + j) % RSR_EVERY != 0 for j in range(steps)])
    ev.close()
    step_bytes = nv[plain] * BYTES_PER_VISIBLE[moments] + N_PRIMS * BYTES_PER_PRIMITIVE[path]
    achieved = float(step_bytes.sum() / durs[plain].sum()) / 1e9 if plain.any() else float("nan")
    state = (groups, t) if keep_state else None
    del groups, t, mask, idx
    torch.cuda.empty_cache()
    return {
        "state": state,
        "value": int(nv.sum()) * 59 / wall,
        "ms_per_step": wall / steps * 1e3,
        "visible_mean": float(nv.mean()),
        "achieved_GBps": achieved,
        "step_kernel_us": float(durs[plain].mean() * 1e6) if plain.any() else float("nan"),
        # per launch, plain steps: from the per-step events of the timed loop (two-launch path), or of the
        # separate per-step pass (fused path; each figure then includes its launch's dispatch gap)
        "step_kernel_us_p10_p50_p90": (spread if region else
                                       [float(x) for x in np.percentile(durs[plain] * 1e6, [10, 50, 90])]
                                       if plain.any() else None),
        "counts": all_counts,
    }


def run_unfused(gs, torch, sd: SceneOnDevice, cams, steps: int = 100, warmup: int = 5):
    """What fusion buys: the same AdamW-GS step written as one-op-per-pass
    PyTorch eager kernels over the compacted visible rows.  The library's
    gs_visibility gives the index list; its count is read to the host, as an
    eager implementation must, to size the gathers.  Per group: gather the
    theta, g, m and v rows; moment updates, bias correction, Adam direction,
    DAR term and parameter update one op at a time; scatter theta, m and v
    back.  Re-State iterations rescale m and v of a Bernoulli sample drawn
    with torch's generator.  FP32 moments.  A comparator, not part of the
    library: before it is timed, three steps of it are checked against the
    fused step from the same state.  The camera order is the leg's own,
    sized to its own steps."""
    import synth
    dev = torch.device(DEVICE)
    order = synth.camera_order(len(cams), warmup + steps, seed=0)
    b1, b2, eps = 0.9, 0.999, 1e-15
    gcams = [gs.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far) for c in cams]
    mask = torch.zeros(N_PRIMS, dtype=torch.uint8, device=dev)
    idx = torch.zeros(N_PRIMS, dtype=torch.int32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int32, device=dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)

    def fresh():
        out = []
        for (name, dim, lr, dar), p, sets in zip(synth.GROUPS_59, sd.params, sd.grads):
            lam = LAMBDA_O if dar == 1 else (LAMBDA_S if dar == 2 else 0.0)
            out.append(gs.Group(p.clone(), sets[0], torch.zeros_like(p), torch.zeros_like(p), lr, dar_kind=dar,
                                dar_lambda=lam, dar_clip=CLIP))
        return out, torch.zeros(N_PRIMS, dtype=torch.int32, device=dev)

    def eager_step(groups, t, k):
        for G, sets in zip(groups, sd.grads):
            G.grad = sets[k % N_GRAD_SETS]
        gs.gs_visibility(groups[0].param, gcams[order[k % len(order)]], mask=mask, vis_idx=idx, vis_count=cnt)
        if k % RSR_EVERY == 0:
            picked = torch.nonzero(torch.rand(N_PRIMS, generator=gen, device=dev) < RSR_P).squeeze(1)
            for G in groups:
                G.exp_avg[picked] = G.exp_avg[picked] * RSR_A1
                G.exp_avg_sq[picked] = G.exp_avg_sq[picked] * RSR_A2
        rows = idx[:int(cnt.item())].long()
        tv = t[rows] + 1
        t[rows] = tv
        tf = tv.to(torch.float32)
        bc1 = (1.0 - torch.pow(b1, tf)).unsqueeze(1)
        bc2 = (1.0 - torch.pow(b2, tf)).unsqueeze(1)
        for G in groups:
            th, g = G.param[rows], G.grad[rows]
            m, v = G.exp_avg[rows], G.exp_avg_sq[rows]
            m.mul_(b1).add_(g, alpha=1.0 - b1)
            v.mul_(b2).addcmul_(g, g, value=1.0 - b2)
            d = (v / bc2).sqrt_().add_(eps)
            u = (m / bc1) / d
            if G.dar_kind == 1:
                e = torch.exp(-th.abs())
                u += torch.clamp(G.dar_lambda / REG_NORM * (e / ((1.0 + e) * (1.0 + e))) / d, max=G.dar_clip)
            elif G.dar_kind == 2:
                u += torch.clamp(G.dar_lambda / REG_NORM * torch.exp(th) / d, max=G.dar_clip)
            G.param[rows] = th - G.lr * u
            G.exp_avg[rows] = m
            G.exp_avg_sq[rows] = v

    worst = moved = rows_checked = None
    if CHECK_UNFUSED:
        # the comparator computes the same step: three steps from the same state
        ref, t_ref = fresh()
        mine, t_mine = fresh()
        for k in (1, 2, 3):
            for G, sets in zip(ref, sd.grads):
                G.grad = sets[k % N_GRAD_SETS]
            gs.gs_visibility(ref[0].param, gcams[order[k % len(order)]], mask=mask, vis_idx=idx, vis_count=cnt)
            gs.adamw_gs_step(ref, N_PRIMS, t_ref, gs.StepConfig(reg_norm=REG_NORM, seed=0, iteration=k, **STEP_LAUNCH),
                             visible=mask, vis_idx=idx, vis_count=cnt)
            eager_step(mine, t_mine, k)
        torch.cuda.synchronize()
        worst = max(float(((A.param - B.param).abs() / B.param.abs().clamp(min=1.0)).max()) for A, B in zip(mine, ref))
        moved = max(float((B.param - p).abs().max()) for B, p in zip(ref, sd.params))
        rows_checked = int((t_ref > 0).sum())
        if not torch.equal(t_mine, t_ref) or worst > 1e-5 or moved == 0.0 or rows_checked == 0:
            raise RuntimeError(f"the unfused comparator does not reproduce the fused step (max err {worst:.3g}, "
                               f"fused step moved theta by up to {moved:.3g}, {rows_checked} rows stepped)")
        del ref, t_ref, mine, t_mine

    groups, t = fresh()
    total = warmup + steps
    for k in range(warmup):
        eager_step(groups, t, k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    nv = 0
    for k in range(warmup, total):
        eager_step(groups, t, k)
        nv += int(cnt.item())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    del groups, t
    torch.cuda.empty_cache()
    return {"path": "unfused eager PyTorch (gs_visibility + one op per pass)", "value": nv * 59 / wall,
            "ms_per_step": wall / steps * 1e3, "steps": steps, "check_max_err_3_steps": worst,
            "check_rows_stepped": rows_checked, "check_max_theta_move": moved}


def run_config1(gs, torch, steps: int = 20, warmup: int = 5, n: int = 100_000) -> dict:
    """The small plain workload: 100k Gaussians of 59 FP32 attributes, all
    drawn N(0, 1); per step a Bernoulli(0.3) visibility mask (seed 0) and
    gradients N(0, 1e-3) on the visible rows only, as synth draws them; RSR
    off (its 100-step interval exceeds the run).  Every step's mask and
    gradients are uploaded before timing.  The step is adamw_gs_step with
    the mask (masked windows of 32), timed per launch with HIP events on the
    launch stream.  The optimizer state (94 MB) fits in the 256 MB Infinity
    Cache, so this figure is cache-resident, not an HBM figure."""
    import synth
    dev = torch.device(DEVICE)
    g0 = synth.rng(0, 1)
    params = {name: g0.standard_normal((n, dim)).astype(np.float32) for name, dim, _, _ in synth.GROUPS_59}
    masks, grads = [], []
    for k in range(warmup + steps):
        m = synth.bernoulli_mask(n, 0.3, seed=0, step=k)
        gk = synth.grads(n, synth.GROUPS_59, m, seed=0, step=k)
        masks.append(torch.from_numpy(m).to(dev))
        grads.append([torch.from_numpy(gk[name]).to(dev) for name, *_ in synth.GROUPS_59])
    groups = [gs.Group(torch.from_numpy(params[name]).to(dev), grads[0][j], torch.zeros((n, dim), device=dev),
                       torch.zeros((n, dim), device=dev), lr, dar_kind=dar,
                       dar_lambda=LAMBDA_O if dar == 1 else (LAMBDA_S if dar == 2 else 0.0), dar_clip=CLIP)
              for j, (name, dim, lr, dar) in enumerate(synth.GROUPS_59)]
    t = torch.zeros(n, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    ev = TimingEvents(steps)
    torch.cuda.synchronize()
    t0 = 0.0
    for k in range(warmup + steps):
        if k == warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        for G, gk in zip(groups, grads[k]):
            G.grad = gk
        cfg = gs.StepConfig(reg_norm=REG_NORM, seed=0, iteration=k, **STEP_LAUNCH)
        j = k - warmup
        if j >= 0:
            ev.record("start", j, stream)
        gs.adamw_gs_step(groups, n, t, cfg, visible=masks[k], stream=stream)
        if j >= 0:
            ev.record("end", j, stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    d = np.array([ev.ms(j) for j in range(steps)]) * 1e-3
    ev.close()
    nv = np.array([int(masks[k].sum().item()) for k in range(warmup, warmup + steps)], np.int64)
    byts = nv * BYTES_PER_VISIBLE["f32"] + n * BYTES_PER_PRIMITIVE["two_launch"]
    del groups, t, masks, grads
    torch.cuda.empty_cache()
    return {"workload": "100k Gaussians x 59 FP32 attributes, Bernoulli(0.3) visibility per step, "
                        "gradients N(0, 1e-3) on visible rows, masked step (windows of 32); cache-resident",
            "steps": steps, "value": float(nv.sum() * 59 / wall), "ms_per_step": wall / steps * 1e3,
            "kernel_attr_updates_per_s": float(nv.sum() * 59 / d.sum()),
            "step_kernel_us": float(d.mean() * 1e6), "visible_mean": float(nv.mean()),
            "achieved_GBps_cache_resident": float(byts.sum() / d.sum() / 1e9)}


def guarded(name: str, fn, *args, **kwargs):
    """Runs one variant leg; a failure becomes {"error": ...} in the JSON
    line instead of ending the run (the headline, its roofline and the CPU
    baseline are printed whatever the variants do)."""
    import traceback
    print(f"bench: variant {name}", file=sys.stderr, flush=True)
    try:
        return fn(*args, **kwargs)
    except Exception as e:  # noqa: BLE001  (any failure of a context leg)
        tb = traceback.format_exc(limit=4)
        print(f"bench: variant {name} failed: {e!r}\n{tb}", file=sys.stderr, flush=True)
        try:
            import torch
            torch.cuda.synchronize()
            torch.cuda.empty_cache()
        except Exception:  # noqa: BLE001
            pass
        return {"error": f"{type(e).__name__}: {e}"}


# position-noise and AIU settings of the widened-row measurements (the paper
# defers lambda_mu, lambda_t and eta_{R_o} to the 3DGS-MCMC settings and gives
# Pro_AIU / eta_AIU only per table; these are those defaults and round values)
NOISE_KW = dict(noise_enable=True, noise_groups=(0, 1, 2, 3), noise_lr=5e5, noise_k=100.0, noise_t=0.005)
AIU_RATIO, AIU_SCALE = 0.05, 1.0


def run_next_rows(gs, torch, sd: SceneOnDevice, cams, steps: int = 200, warmup: int = 10) -> dict:
    """The widened rows on the 3M Morton scene with FP32 moments, each timed
    with HIP events on the launch stream and read against its algorithmic
    bytes:
    - position noise: the fused view step with the noise term on the means,
      with the scene's N(0, 1) log-scales and with small ones (N(ln 0.01,
      0.5), beside the plain step on the same scales);
    - AIU every step (Pro_AIU 0.05): the fused view step, whose waves also
      move their windows' sampled invisible rows with t > 0;
    - four cameras per step: the fused view step over the union of four views;
    - eight views' visibility in one pass (gs_visibility_multi);
    - pruning 10 % of the primitives (gs_prune) and appending 5 % as clones
      (gs_append).
    The view steps also write their mask (1 B per primitive, counted), from
    which the visible counts are read outside the timed region.  The camera
    order is the leg's own, sized to its own steps."""
    import synth
    dev = torch.device(DEVICE)
    order = synth.camera_order(len(cams), warmup + steps, seed=0)
    gcams = [gs.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far) for c in cams]
    stream = torch.cuda.current_stream()
    n = N_PRIMS

    def fresh():
        groups = [gs.Group(p.clone(), sets[0], torch.zeros_like(p), torch.zeros_like(p), lr, dar_kind=dar,
                           dar_lambda=LAMBDA_O if dar == 1 else (LAMBDA_S if dar == 2 else 0.0), dar_clip=CLIP)
                  for (name, dim, lr, dar), p, sets in zip(synth.GROUPS_59, sd.params, sd.grads)]
        return groups, torch.zeros(n, dtype=torch.int32, device=dev)

    def view_steps(extra, n_cams=1, aiu=False, small_scales=False):
        groups, t = fresh()
        if small_scales:
            # log-scales ~ N(ln 0.01, 0.5), the size of a trained scene's
            # Gaussians: the noise displacement stays small, so the means keep
            # their Morton runs and the time is the noise computation's
            gen = torch.Generator(device=dev)
            gen.manual_seed(29)
            groups[1].param.copy_(torch.randn(groups[1].param.shape, generator=gen, device=dev) * 0.5 - 4.6)
        mask = torch.zeros(n, dtype=torch.uint8, device=dev)
        ev = TimingEvents(steps)
        vis, aiu_rows = [], []
        for k in range(warmup + steps):
            for G, sets in zip(groups, sd.grads):
                G.grad = sets[k % N_GRAD_SETS]
            # windows: the library's default (32; 64 with position noise)
            cfg = gs.StepConfig(reg_norm=REG_NORM, seed=0, iteration=k, rsr_enable=(k % RSR_EVERY == 0),
                                rsr_ratio=RSR_P, rsr_alpha1=RSR_A1, rsr_alpha2=RSR_A2, **extra)
            view = [gcams[order[(k + 53 * j) % len(order)]] for j in range(n_cams)] if n_cams > 1 \
                else gcams[order[k % len(order)]]
            if aiu and k >= warmup:
                # expected AIU rows of this step: p x (invisible rows with t > 0), t before the step
                aiu_t = (t > 0)
            j = k - warmup
            if j >= 0:
                ev.record("start", j, stream)
            gs.adamw_gs_step_view(groups, n, t, cfg, groups[0].param, view, visible_out=mask, stream=stream)
            if j >= 0:
                ev.record("end", j, stream)
                vis.append(mask.sum(dtype=torch.int64))
                if aiu:
                    aiu_rows.append((aiu_t & (mask == 0)).sum(dtype=torch.int64))
        torch.cuda.synchronize()
        d = np.array([ev.ms(j) for j in range(steps)]) * 1e-3
        ev.close()
        nv = np.array([int(x.item()) for x in vis], np.int64)
        plain = np.array([(warmup + j) % RSR_EVERY != 0 for j in range(steps)])
        byts = nv * BYTES_PER_VISIBLE["f32"] + n * (BYTES_PER_PRIMITIVE["view"] + 1)
        if aiu:
            byts = byts + AIU_RATIO * np.array([int(x.item()) for x in aiu_rows], np.float64) * 948
        # the cached blocks stay with torch, so every row runs on the same memory
        del groups, t, mask
        ach = float(byts[plain].sum() / d[plain].sum() / 1e9)
        return {"step_kernel_us": float(d[plain].mean() * 1e6), "visible_mean": float(nv.mean()),
                "achieved_GBps": ach, "frac": ach / HBM_PEAK_GBS}

    view_steps({})                     # discarded: brings the device to its working clocks
    out = {"plain_view": view_steps({})}
    out["position_noise"] = view_steps(dict(NOISE_KW))
    out["position_noise_small_scales"] = view_steps(dict(NOISE_KW), small_scales=True)
    out["plain_view_small_scales"] = view_steps({}, small_scales=True)
    out["aiu_every_step"] = view_steps(dict(aiu_enable=True, aiu_ratio=AIU_RATIO, aiu_scale=AIU_SCALE), aiu=True)
    out["aiu_every_step"]["bytes_note"] = "948 B per expected AIU row (p x invisible rows with t > 0) added"
    out["four_views_union"] = view_steps({}, n_cams=4)

    # eight views' visibility in one pass
    means = sd.params[0]
    mask = torch.zeros(n, dtype=torch.uint8, device=dev)
    bits = torch.zeros(n, dtype=torch.int32, device=dev)
    idx = torch.zeros(n, dtype=torch.int32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int32, device=dev)
    views = [gcams[order[53 * j % len(order)]] for j in range(8)]
    reps = 50
    ev = TimingEvents(reps)
    for j in range(reps + 3):
        if j >= 3:
            ev.record("start", j - 3, stream)
        gs.gs_visibility_multi(means, views, mask=mask, view_bits=bits, vis_idx=idx, vis_count=cnt, stream=stream)
        if j >= 3:
            ev.record("end", j - 3, stream)
    torch.cuda.synchronize()
    us = float(np.mean([ev.ms(j) for j in range(reps)]) * 1e3)
    ev.close()
    nu = int(cnt.item())
    mb = n * (12 + 1 + 4) + nu * 4
    out["visibility_8_views"] = {"kernel_us": us, "union_visible": nu, "achieved_GBps": mb / us / 1e3,
                                 "frac": mb / us / 1e3 / HBM_PEAK_GBS,
                                 "bytes": "12 B means + 1 B mask + 4 B view bits per primitive, 4 B per union index"}
    del mask, bits, idx, cnt

    # pruning 10 % and appending 5 %, on a state that has taken a few steps
    src, t = fresh()
    m0 = torch.zeros(n, dtype=torch.uint8, device=dev)
    for k in range(3):
        gs.adamw_gs_step_view(src, n, t, gs.StepConfig(reg_norm=REG_NORM, iteration=k, unit=VIEW_UNIT),
                              src[0].param, gcams[order[k % len(order)]], visible_out=m0)
    gen = torch.Generator(device=dev)
    gen.manual_seed(17)
    keep = (torch.rand(n, generator=gen, device=dev) < 0.9).to(torch.uint8)
    dst = [gs.Group(torch.empty_like(g.param), None, torch.empty_like(g.exp_avg), torch.empty_like(g.exp_avg_sq), g.lr)
           for g in src]
    t_dst = torch.empty_like(t)
    kept = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = torch.empty(gs.gs_prune_workspace_size(n), dtype=torch.uint8, device=dev)
    ev = TimingEvents(20)
    for j in range(23):
        if j >= 3:
            ev.record("start", j - 3, stream)
        gs.gs_prune(keep, src, dst, gs.GS_MOMENT_F32, t, t_dst, kept, ws, stream=stream)
        if j >= 3:
            ev.record("end", j - 3, stream)
    torch.cuda.synchronize()
    us = float(np.mean([ev.ms(j) for j in range(20)]) * 1e3)
    ev.close()
    nk = int(kept.item())
    mb = nk * (59 * 3 * 8 + 8) + n
    out["prune_10pct"] = {"kernel_us": us, "kept": nk, "achieved_GBps": mb / us / 1e3, "frac": mb / us / 1e3 / HBM_PEAK_GBS,
                          "bytes": "per kept row theta, m, v read + written (59 x 3 x 8 B) and t (8 B); 1 B of keep per primitive"}
    del dst, t_dst, ws
    k_new = n // 20
    grown = [gs.Group(torch.cat([g.param, torch.zeros((k_new, g.param.shape[1]), device=dev)]), None,
                      torch.cat([g.exp_avg, torch.zeros((k_new, g.param.shape[1]), device=dev)]),
                      torch.cat([g.exp_avg_sq, torch.zeros((k_new, g.param.shape[1]), device=dev)]), g.lr)
             for g in src]
    t_grown = torch.cat([t, torch.zeros(k_new, dtype=torch.int32, device=dev)])
    src_idx = torch.randint(0, n, (k_new,), generator=gen, device=dev, dtype=torch.int32)
    ev = TimingEvents(20)
    for j in range(23):
        if j >= 3:
            ev.record("start", j - 3, stream)
        gs.gs_append(grown, gs.GS_MOMENT_F32, n, src_idx, t_grown, stream=stream)
        if j >= 3:
            ev.record("end", j - 3, stream)
    torch.cuda.synchronize()
    us = float(np.mean([ev.ms(j) for j in range(20)]) * 1e3)
    ev.close()
    mb = k_new * 948 + k_new * 4
    out["append_5pct"] = {"kernel_us": us, "appended": k_new, "achieved_GBps": mb / us / 1e3,
                          "frac": mb / us / 1e3 / HBM_PEAK_GBS,
                          "bytes": "per new row theta read + written (59 x 8 B), m and v written (59 x 8 B), t written; 4 B of index"}
    del src, grown, t, t_grown
    torch.cuda.empty_cache()
    return out


def run_sweep(gs, torch, steps: int = 100, warmup: int = 10, only_n: int = 0) -> list:
    """The fused view step (FP32, windows of 32, Morton order) over
    scene sizes 1M-24M at the rig's z_far 17.5, and over visible fractions
    (z_far 15, 17.5, 20, 25, infinity) at 3M.  Scenes are drawn on the
    device (means U[-10, 10]^3, other attributes N(0, 1), one gradient set
    N(0, 1e-3)).  The step writes its mask, whose counts, read outside the
    timed region, give the algorithmic bytes (1660 B per visible + 13 B per
    primitive)."""
    import synth
    dev = torch.device(DEVICE)
    stream = torch.cuda.current_stream()
    out = []

    def one(n, z_far):
        gen = torch.Generator(device=dev)
        gen.manual_seed(n)
        means = torch.rand((n, 3), generator=gen, device=dev) * 20.0 - 10.0
        perm = torch.empty(n, dtype=torch.int32, device=dev)
        ws = torch.empty(gs.gs_spatial_order_workspace_size(n), dtype=torch.uint8, device=dev)
        gs.gs_spatial_order(means, perm, ws)
        means = gs.apply_spatial_order([means], perm)[0]
        del perm, ws
        groups = []
        for k, (name, d, lr, dar) in enumerate(synth.GROUPS_59):
            p = means if k == 0 else torch.randn((n, d), generator=gen, device=dev)
            g = torch.randn((n, d), generator=gen, device=dev) * 1e-3
            groups.append(gs.Group(p, g, torch.zeros_like(p), torch.zeros_like(p), lr, dar_kind=dar,
                                   dar_lambda=LAMBDA_O if dar == 1 else (LAMBDA_S if dar == 2 else 0.0),
                                   dar_clip=CLIP))
        t = torch.zeros(n, dtype=torch.int32, device=dev)
        mask = torch.zeros(n, dtype=torch.uint8, device=dev)
        cams = synth.camera_rig(z_far=z_far)
        gcams = [gs.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far) for c in cams]
        order = synth.camera_order(len(cams), warmup + steps, seed=1)
        ev = TimingEvents(steps)
        vis = []
        for k in range(warmup + steps):
            cfg = gs.StepConfig(reg_norm=REG_NORM, seed=0, iteration=k + 1, unit=VIEW_UNIT)
            j = k - warmup
            if j >= 0:
                ev.record("start", j, stream)
            gs.adamw_gs_step_view(groups, n, t, cfg, groups[0].param, gcams[order[k % len(order)]], visible_out=mask,
                                  stream=stream)
            if j >= 0:
                ev.record("end", j, stream)
                vis.append(mask.sum(dtype=torch.int64))
        torch.cuda.synchronize()
        d = np.array([ev.ms(j) for j in range(steps)]) * 1e-3
        ev.close()
        nv = np.array([int(x.item()) for x in vis], np.int64)
        byts = nv * BYTES_PER_VISIBLE["f32"] + n * (BYTES_PER_PRIMITIVE["view"] + 1)
        ach = float(byts.sum() / d.sum() / 1e9)
        del groups, t, mask, means
        torch.cuda.empty_cache()
        return {"n": n, "z_far": z_far, "visible_frac": float(nv.mean() / n), "step_kernel_us": float(d.mean() * 1e6),
                "attr_updates_per_s": float(nv.sum() * 59 / d.sum()), "achieved_GBps": ach, "frac": ach / HBM_PEAK_GBS}

    one(1_000_000, 17.5)                  # discarded: brings the device to its working clocks
    if only_n > 0:
        return [one(only_n, 17.5)]
    for n in (1_000_000, 3_000_000, 6_000_000, 12_000_000, 24_000_000):
        out.append(one(n, 17.5))
        print(f"bench: sweep n={n} done", file=sys.stderr, flush=True)
    for z_far in (15.0, 20.0, 25.0, float("inf")):
        out.append(one(3_000_000, z_far))
        print(f"bench: sweep z_far={z_far} done", file=sys.stderr, flush=True)
    return out


def run_profile_set(gs, torch, reps: int = 10) -> dict:
    """A short, fixed sequence of launches for counter runs (rocprofv3
    --pmc): on the 3M scene (means U[-10, 10]^3 drawn on the device, Morton
    order, other attributes N(0, 1), z_far 17.5) `reps` fused view steps with
    FP32 moments, `reps` with BF16 moments, `reps` / 2 dense steps (every
    primitive visible, windows of 64) with FP32 moments, `reps` two-launch
    steps (visibility, then the masked step in windows of 32) with FP32
    moments; the rows probe on the same cameras' masks (FP32 moments in the
    step's shape and in 8 items in flight, BF16 in the step's shape), `reps`
    each; then the streaming probes' 4-read / 3-write mix in its default and
    best swept shapes and the copy in its best shape, `reps` launches each
    over 4 x 1 GiB.  Each kernel is told apart by its name (template
    arguments) in the trace."""
    import ctypes

    import bench_probe
    import synth
    dev = torch.device(DEVICE)
    n = N_PRIMS
    gen = torch.Generator(device=dev)
    gen.manual_seed(n)
    means = torch.rand((n, 3), generator=gen, device=dev) * 20.0 - 10.0
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    ws = torch.empty(gs.gs_spatial_order_workspace_size(n), dtype=torch.uint8, device=dev)
    gs.gs_spatial_order(means, perm, ws)
    means = gs.apply_spatial_order([means], perm)[0]
    del perm, ws
    params = [means] + [torch.randn((n, d), generator=gen, device=dev) for _, d, _, _ in synth.GROUPS_59[1:]]
    grads = [torch.randn((n, d), generator=gen, device=dev) * 1e-3 for _, d, _, _ in synth.GROUPS_59]
    cams = synth.camera_rig(z_far=17.5)
    gcams = [gs.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far) for c in cams]
    order = synth.camera_order(len(cams), 4 * reps, seed=1)
    stream = torch.cuda.current_stream()
    out = {}
    mask = torch.zeros(n, dtype=torch.uint8, device=dev)
    idx = torch.zeros(n, dtype=torch.int32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int32, device=dev)
    for label, mdt, mom, sched, count in (("view_f32", torch.float32, GS_F32, None, reps),
                                          ("view_bf16", torch.bfloat16, GS_BF16, None, reps),
                                          ("dense_f32", torch.float32, GS_F32, 3, max(reps // 2, 1)),
                                          ("masked_f32", torch.float32, GS_F32, 2, reps)):
        groups = [gs.Group(p.clone(), g, torch.zeros(p.shape, dtype=mdt, device=dev),
                           torch.zeros(p.shape, dtype=mdt, device=dev), lr, dar_kind=dar,
                           dar_lambda=LAMBDA_O if dar == 1 else (LAMBDA_S if dar == 2 else 0.0), dar_clip=CLIP)
                  for (name, d, lr, dar), p, g in zip(synth.GROUPS_59, params, grads)]
        t = torch.zeros(n, dtype=torch.int32, device=dev)
        for k in range(count):
            cfg = gs.StepConfig(reg_norm=REG_NORM, seed=0, iteration=k + 1, moment_dtype=mom,
                                **({} if sched is None else {"schedule": sched}))
            if sched is None:
                gs.adamw_gs_step_view(groups, n, t, cfg, groups[0].param, gcams[order[k % len(order)]],
                                      stream=stream)
            elif sched == 2:
                gs.gs_visibility(groups[0].param, gcams[order[k % len(order)]], mask=mask, vis_idx=idx,
                                 vis_count=cnt, stream=stream)
                cfg = gs.StepConfig(reg_norm=REG_NORM, seed=0, iteration=k + 1, moment_dtype=mom, **STEP_LAUNCH)
                gs.adamw_gs_step(groups, n, t, cfg, visible=mask, vis_idx=idx, vis_count=cnt, stream=stream)
            else:
                gs.adamw_gs_step(groups, n, t, cfg, stream=stream)
        torch.cuda.synchronize()
        out[label] = count
        del groups, t
    lib = bench_probe.load()
    sp = ctypes.c_void_p(stream.cuda_stream)
    dims = (ctypes.c_int32 * len(params))(*[p.shape[1] for p in params])
    for label, mdt, bf16, win, items in (("rows_f32", torch.float32, 0, 32, 4), ("rows_f32_i8", torch.float32, 0, 32, 8),
                                         ("rows_bf16", torch.bfloat16, 1, 32, 4)):
        arrs = [(p.clone(), g, torch.zeros(p.shape, dtype=mdt, device=dev), torch.zeros(p.shape, dtype=mdt, device=dev))
                for p, g in zip(params, grads)]
        ptrs = [(ctypes.c_void_p * len(arrs))(*[a[j].data_ptr() for a in arrs]) for j in range(4)]
        t = torch.zeros(n, dtype=torch.int32, device=dev)
        for k in range(reps):
            gs.gs_visibility(params[0], gcams[order[k % len(order)]], mask=mask, vis_idx=idx, vis_count=cnt,
                             stream=stream)
            rc = lib.gsprobe_rows_4r3w_cfg(ctypes.c_void_p(mask.data_ptr()), ctypes.c_void_p(t.data_ptr()), ptrs[0],
                                           ptrs[1], ptrs[2], ptrs[3], dims, len(arrs), n, win, items, bf16, sp)
            if rc != 0:
                raise RuntimeError(f"gsprobe_rows_4r3w_cfg returned {rc}")
        torch.cuda.synchronize()
        out[label] = reps
        del arrs, t
    del params, grads, means, mask, idx, cnt
    torch.cuda.empty_cache()
    nbytes = 1 << 30
    arrs = [torch.rand(nbytes // 4, device=dev) for _ in range(4)]
    ptr = [a.data_ptr() for a in arrs]
    for (w, it, ntl, nts) in ((16, 4, 1, 1), (8, 2, 1, 1)):
        for _ in range(reps):
            lib.gsprobe_rmw_4r3w_cfg(ptr[0], ptr[1], ptr[2], ptr[3], nbytes // 16, w, it, ntl, nts, 0, sp)
    for _ in range(reps):
        lib.gsprobe_copy_cfg(ptr[0], ptr[1], nbytes // 16, 8, 2, 1, 1, 0, sp)
    torch.cuda.synchronize()
    out["probe"] = reps
    return out


def same_state(torch, a, b) -> bool:
    """Bit equality of two (groups, step counts) end states."""
    (ga, ta), (gb, tb) = a, b
    def bits(x):
        return x.view(torch.int16) if x.dtype == torch.bfloat16 else x
    return torch.equal(ta, tb) and all(
        torch.equal(x.param, y.param) and torch.equal(bits(x.exp_avg), bits(y.exp_avg))
        and torch.equal(bits(x.exp_avg_sq), bits(y.exp_avg_sq)) for x, y in zip(ga, gb))


# The packed layout of the batched workload: the five attribute groups as
# column ranges of one [n][64] array per role (attributes, gradients, each
# moment), 16-byte aligned where their rows allow vector access.
PACKED_WIDTH = 64
PACKED_COLUMNS = {"sh": 0, "quats": 48, "means": 52, "scales": 55, "opacity": 58}


def run_tuner(gs, torch, sd: SceneOnDevice, cams, steps: int = 20, z_fars=(17.5, 10.0)) -> dict:
    """The schedule tuner on the 3M Morton scene with FP32 moments: gs_tune_mask
    with the first camera's own visibility mask against gs_tune at that mask's
    visible fraction (a synthetic i.i.d. mask), at the rig's far plane and at
    a nearer one (fewer visible primitives).  Each choice's step is then timed
    on that camera's mask: HIP events around `steps` launches, after 3 untimed
    ones; the visibility and compaction run once beforehand.  Algorithmic
    bytes: 1660 B per visible, plus 1 B of mask per primitive (masked) or 4 B
    of index per visible (compacted)."""
    import synth
    dev = torch.device(DEVICE)
    mask = torch.zeros(N_PRIMS, dtype=torch.uint8, device=dev)
    idx = torch.zeros(N_PRIMS, dtype=torch.int32, device=dev)
    cnt = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    dims = [d for _, d, _, _ in synth.GROUPS_59]
    groups = [gs.Group(p.clone(), sets[0], torch.zeros_like(p), torch.zeros_like(p), lr, dar_kind=dar,
                       dar_lambda=LAMBDA_O if dar == 1 else (LAMBDA_S if dar == 2 else 0.0), dar_clip=CLIP)
              for (name, dim, lr, dar), p, sets in zip(synth.GROUPS_59, sd.params, sd.grads)]
    t = torch.zeros(N_PRIMS, dtype=torch.int32, device=dev)
    names = {gs.GS_SCHED_COMPACTED: "compacted", gs.GS_SCHED_MASKED: "masked"}
    out = {"workload": "3M-primitive scene, Morton order, FP32, one camera's mask", "cases": []}
    c = cams[0]
    for z_far in z_fars:
        cam = gs.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, z_far)
        gs.gs_visibility(sd.params[0], cam, mask=mask, vis_idx=idx, vis_count=cnt, stream=stream)
        torch.cuda.synchronize()
        vis = int(cnt.item())
        gs.gs_tune_clear()
        choices = {"own_mask": gs.gs_tune_mask(N_PRIMS, dims, mask),
                   "iid_mask": gs.gs_tune(N_PRIMS, dims, max(vis, 1) / N_PRIMS)}
        gs.gs_tune_clear()
        case = {"z_far": z_far, "visible": vis}
        for label, (sched, unit) in choices.items():
            cfg = gs.StepConfig(reg_norm=REG_NORM, iteration=1, schedule=sched, unit=unit)
            for _ in range(3):
                gs.adamw_gs_step(groups, N_PRIMS, t, cfg, visible=mask, vis_idx=idx, vis_count=cnt, stream=stream)
            ev = TimingEvents(1)
            ev.record("start", 0, stream)
            for _ in range(steps):
                gs.adamw_gs_step(groups, N_PRIMS, t, cfg, visible=mask, vis_idx=idx, vis_count=cnt, stream=stream)
            ev.record("end", 0, stream)
            torch.cuda.synchronize()
            us = ev.ms(0) * 1e3 / steps
            ev.close()
            alg = vis * BYTES_PER_VISIBLE["f32"] + (N_PRIMS if sched == gs.GS_SCHED_MASKED else 4 * vis)
            case[label] = {"schedule": names.get(sched, str(sched)), "unit": unit, "step_kernel_us": us,
                           "achieved_GBps": alg / us / 1e3}
        out["cases"].append(case)
    del groups, t
    torch.cuda.empty_cache()
    return out


def run_batched(gs, torch, steps: int = 300, warmup: int = 10, n_masks: int = 8,
                forms=("batched_bf16", "batched_bf16_packed", "batched_bf16_resident", "per_scene_bf16",
                       "per_scene_f32"), rows_probe: bool = True):
    """Many-scene workload: 16 scenes with sizes log-uniform in [2e5, 4e6] and
    visible ratios U[0.02, 0.60] (Bernoulli visibility, 8 pre-drawn masks per
    scene used in turn), 59 attributes each.  Times three forms of the same
    steps: the BF16-moment plan (one persistent launch per step from a HIP
    graph, schedules picked by the tuner; one plan per mask set), and
    per-scene adamw_gs_step calls with FP32 and with BF16 moments.  The
    "packed" form keeps each scene's groups as column ranges of one [n][64]
    array per role (PACKED_COLUMNS), so that an isolated visible primitive
    reads and writes whole 128-byte lines; its algorithmic bytes are the same
    (the 5 padding floats per row are not counted).  Every form includes
    the compaction of the compacted scenes' masks."""
    import synth
    dev = torch.device(DEVICE)
    sizes, ratios = synth.batch_scene_sizes(16, *BATCH_SIZE_RANGE, seed=0)
    dims = [d for _, d, _, _ in synth.GROUPS_59]
    gen = torch.Generator(device=dev)
    gen.manual_seed(5)
    scenes = []
    for n, p in zip(sizes.tolist(), ratios.tolist()):
        sched, unit = gs.gs_tune(n, dims, float(p), gs.GS_MOMENT_BF16)
        scenes.append(dict(
            n=n, p=p, sched=sched,
            params=[torch.randn((n, d), generator=gen, device=dev) for d in dims],
            grads=[torch.randn((n, d), generator=gen, device=dev) * 1e-3 for d in dims],
            masks=[(torch.rand(n, generator=gen, device=dev) < p).to(torch.uint8) for _ in range(n_masks)],
            idx=[torch.zeros(n, dtype=torch.int32, device=dev) for _ in range(n_masks)],
            cnt=[torch.zeros(1, dtype=torch.int32, device=dev) for _ in range(n_masks)]))
    stream = torch.cuda.current_stream()

    def make_groups(sc, mdt, packed=False):
        lam = {1: LAMBDA_O, 2: LAMBDA_S}
        if not packed:
            return [gs.Group(p.clone(), g, torch.zeros(p.shape, dtype=mdt, device=dev),
                             torch.zeros(p.shape, dtype=mdt, device=dev), lr, dar_kind=dar,
                             dar_lambda=lam.get(dar, 0.0), dar_clip=CLIP)
                    for (name, d, lr, dar), p, g in zip(synth.GROUPS_59, sc["params"], sc["grads"])]
        # one [n][64] array per role: each primitive's state fills whole lines
        n = sc["n"]
        pk = {"p": torch.zeros((n, PACKED_WIDTH), device=dev), "g": torch.zeros((n, PACKED_WIDTH), device=dev),
              "m": torch.zeros((n, PACKED_WIDTH), dtype=mdt, device=dev),
              "v": torch.zeros((n, PACKED_WIDTH), dtype=mdt, device=dev)}
        out = []
        for (name, d, lr, dar), p, g in zip(synth.GROUPS_59, sc["params"], sc["grads"]):
            c = PACKED_COLUMNS[name]
            pk["p"][:, c:c + d] = p
            pk["g"][:, c:c + d] = g
            out.append(gs.Group(pk["p"][:, c:c + d], pk["g"][:, c:c + d], pk["m"][:, c:c + d], pk["v"][:, c:c + d],
                                lr, dar_kind=dar, dar_lambda=lam.get(dar, 0.0), dar_clip=CLIP))
        return out

    def timed(form):
        bf16 = form != "per_scene_f32"
        mdt = torch.bfloat16 if bf16 else torch.float32
        mom = gs.GS_MOMENT_BF16 if bf16 else gs.GS_MOMENT_F32
        packed = form.endswith("packed")
        state = [dict(groups=make_groups(sc, mdt, packed), t=torch.zeros(sc["n"], dtype=torch.int32, device=dev))
                 for sc in scenes]
        plans = []
        if form.startswith("batched_bf16"):
            for r in range(n_masks):
                plans.append(gs.Batch([gs.Scene(groups=st["groups"], n=sc["n"], step_count=st["t"],
                                                visible=sc["masks"][r], vis_idx=sc["idx"][r],
                                                vis_count=sc["cnt"][r], schedule=sc["sched"],
                                                visible_hint=sc["p"]) for sc, st in zip(scenes, state)],
                                      moment_dtype=mom))
                plans[-1].set_resident(form.endswith("resident"))

        def one(k):
            r = k % n_masks
            for sc in scenes:
                if sc["sched"] == gs.GS_SCHED_COMPACTED:
                    gs.gs_compact(sc["masks"][r], sc["idx"][r], sc["cnt"][r], stream=stream)
            cfg = dict(reg_norm=REG_NORM, seed=0, iteration=k, rsr_enable=(k % RSR_EVERY == 0), rsr_ratio=RSR_P,
                       rsr_alpha1=RSR_A1, rsr_alpha2=RSR_A2, moment_dtype=mom, stochastic_round=True)
            if plans:
                plans[r].step(gs.StepConfig(**cfg), stream=stream)
            else:
                for s, (sc, st) in enumerate(zip(scenes, state)):
                    gs.adamw_gs_step(st["groups"], sc["n"], st["t"],
                                     gs.StepConfig(**dict(cfg, seed=s, schedule=sc["sched"])),
                                     visible=sc["masks"][r], vis_idx=sc["idx"][r], vis_count=sc["cnt"][r],
                                     stream=stream)

        for k in range(warmup):
            one(k)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(warmup, warmup + steps):
            one(k)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        for b in plans:
            b.close()
        del state, plans
        torch.cuda.empty_cache()
        return wall

    vis_per_mask = [sum(int(sc["masks"][r].sum().item()) for sc in scenes) for r in range(n_masks)]
    vis_total = sum(vis_per_mask[k % n_masks] for k in range(warmup, warmup + steps))
    out = {"workload": "16 scenes, N log-uniform in [2e5, 4e6] (sum %d), visible 2-60 %%, 59 attributes, %d steps"
                       % (int(sizes.sum()), steps),
           "schedules": {"compacted": sum(sc["sched"] == gs.GS_SCHED_COMPACTED for sc in scenes),
                         "masked": sum(sc["sched"] == gs.GS_SCHED_MASKED for sc in scenes)},
           "visible_per_step": vis_total / steps,
           "algorithmic_bytes_per_step_bf16": vis_total / steps * BYTES_PER_VISIBLE["bf16"] + int(sizes.sum())}
    for form in forms:
        wall = timed(form)
        out[form] = {"value": vis_total * 59 / wall, "ms_per_step": wall / steps * 1e3}
    if rows_probe:
        rp = guarded("batched rows probe", batched_rows_ceiling, torch, scenes, n_masks, min(steps, 40))
        if "error" not in rp:
            rp["alg_GBps"] = {k: out["algorithmic_bytes_per_step_bf16"] / (v * 1e-3) / 1e9
                              for k, v in rp["kernel_ms_per_step"].items()}
        out["rows_probe_bf16"] = rp
        rp = guarded("batched rows probe, packed", batched_rows_ceiling, torch, scenes, n_masks, min(steps, 40),
                     shapes=((128, 2), (128, 4), (64, 2), (64, 4), (32, 4), (128, 8)), packed=True)
        if "error" not in rp:
            rp["alg_GBps"] = {k: out["algorithmic_bytes_per_step_bf16"] / (v * 1e-3) / 1e9
                              for k, v in rp["kernel_ms_per_step"].items()}
        out["rows_probe_bf16_packed"] = rp
    scenes.clear()
    torch.cuda.empty_cache()
    return out


def batched_rows_ceiling(torch, scenes, n_masks: int, steps: int,
                         shapes=((32, 4), (64, 4), (128, 4), (32, 8), (64, 8), (128, 8)), packed: bool = False) -> dict:
    """The rows probe (the masked step's access pattern, no arithmetic; BF16
    moments) over each scene of the batch with its own masks, one launch per
    scene, each launch timed with HIP events; the sum over the scenes of a
    step is that step's kernel time.  Per launch shape (window, chunk items
    in flight), the mean over `steps` steps.  packed: each scene's state as
    one [n][PACKED_WIDTH] array per role (the packed plan's rows, padding
    included), instead of one array per group."""
    import ctypes

    import bench_probe
    import synth
    dev = torch.device(DEVICE)
    lib = bench_probe.load()
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    dims = [PACKED_WIDTH] if packed else [d for _, d, _, _ in synth.GROUPS_59]
    ng = len(dims)
    cd = (ctypes.c_int32 * ng)(*dims)
    res = {}
    for (win, items) in shapes:
        total_ms = 0.0
        for sc in scenes:
            n = sc["n"]
            if packed:
                arrs = [(torch.randn((n, PACKED_WIDTH), device=dev), torch.randn((n, PACKED_WIDTH), device=dev) * 1e-3,
                         torch.zeros((n, PACKED_WIDTH), dtype=torch.bfloat16, device=dev),
                         torch.zeros((n, PACKED_WIDTH), dtype=torch.bfloat16, device=dev))]
            else:
                arrs = [(p.clone(), g, torch.zeros(p.shape, dtype=torch.bfloat16, device=dev),
                         torch.zeros(p.shape, dtype=torch.bfloat16, device=dev))
                        for p, g in zip(sc["params"], sc["grads"])]
            t = torch.zeros(n, dtype=torch.int32, device=dev)
            ptrs = [(ctypes.c_void_p * ng)(*[a[k].data_ptr() for a in arrs]) for k in range(4)]
            ev = TimingEvents(steps)
            for k in range(steps + 2):
                j = k - 2
                if j >= 0:
                    ev.record("start", j, stream)
                rc = lib.gsprobe_rows_4r3w_cfg(ctypes.c_void_p(sc["masks"][k % n_masks].data_ptr()),
                                               ctypes.c_void_p(t.data_ptr()), ptrs[0], ptrs[1], ptrs[2], ptrs[3],
                                               cd, ng, n, win, items, 1, sp)
                if rc != 0:
                    raise RuntimeError(f"gsprobe_rows_4r3w_cfg returned {rc}")
                if j >= 0:
                    ev.record("end", j, stream)
            torch.cuda.synchronize()
            total_ms += float(np.mean([ev.ms(j) for j in range(steps)]))
            ev.close()
            del arrs, t
        res[f"win{win}_i{items}"] = total_ms
    torch.cuda.empty_cache()
    best = min(res, key=res.get)
    return {"kernel_ms_per_step": res, "best_shape": best, "best_kernel_ms_per_step": res[best],
            "kind": "rows probe (masked-step access pattern, BF16 moments, no arithmetic) per scene with the "
                    "scene's own masks; per step: sum of the scenes' kernel times"
                    + (f"; packed rows: one [n][{PACKED_WIDTH}] array per role" if packed else "")}


def run_mcmc(gs, torch, cams, steps: int = 500, warmup: int = 10, path: str = "two_launch", counts_from=None):
    """3DGS-MCMC-shaped workload: 6M primitives (the cap), means from an
    equal-weight mixture of 64 isotropic Gaussians (sigma 1.5), other
    attributes N(0, 1), opacity and scale regularisation weights 0.01, and
    every step the 1 % lowest opacity logits (60 000) get their state reset
    (relocation).  Morton layout, FP32 moments.  One step = the AdamW-GS step
    ("two_launch": visibility + compaction, then the masked step; "view": the
    fused view step) and the relocation select + reset.  The fused path
    writes no count: its visible counts come from a two-launch run
    (`counts_from`), whose end state it must reproduce bit for bit (the
    returned digest)."""
    import synth
    dev = torch.device(DEVICE)
    n = MCMC_N
    k_reloc = n // 100
    means = synth.scene_clustered(n, seed=0, groups=[("means", 3, 0.0, 0)]).params["means"]
    gen = torch.Generator(device=dev)
    gen.manual_seed(6)
    params = [torch.from_numpy(means).to(dev)] + [torch.randn((n, d), generator=gen, device=dev)
                                                   for _, d, _, _ in synth.GROUPS_59[1:]]
    grads = [[torch.randn((n, d), generator=gen, device=dev) * 1e-3 for _ in range(2)]
             for _, d, _, _ in synth.GROUPS_59]
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    ws = torch.empty(gs.gs_spatial_order_workspace_size(n), dtype=torch.uint8, device=dev)
    gs.gs_spatial_order(params[0], perm, ws)
    params = gs.apply_spatial_order(params, perm)
    grads = [gs.apply_spatial_order(sets, perm) for sets in grads]
    del ws, perm
    groups = [gs.Group(p, sets[0], torch.zeros_like(p), torch.zeros_like(p), lr, dar_kind=dar,
                       dar_lambda=0.01 if dar else 0.0, dar_clip=CLIP)
              for (name, d, lr, dar), p, sets in zip(synth.GROUPS_59, params, grads)]
    opacity = groups[3].param
    t = torch.zeros(n, dtype=torch.int32, device=dev)
    mask = torch.zeros(n, dtype=torch.uint8, device=dev)
    idx = torch.zeros(n, dtype=torch.int32, device=dev)
    counts = torch.zeros(warmup + steps, dtype=torch.int32, device=dev)
    rws = torch.empty(gs.gs_relocate_workspace_size(n), dtype=torch.uint8, device=dev)
    order = synth.camera_order(len(cams), warmup + steps, seed=3)
    gcams = [gs.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far) for c in cams]
    stream = torch.cuda.current_stream()
    ev = TimingEvents(steps)

    def one(k, slot=-1):
        cnt = counts[k:k + 1]
        for G, sets in zip(groups, grads):
            G.grad = sets[k % 2]
        common = dict(reg_norm=REG_NORM, seed=0, iteration=k, rsr_enable=(k % RSR_EVERY == 0), rsr_ratio=RSR_P,
                      rsr_alpha1=RSR_A1, rsr_alpha2=RSR_A2)
        if path == "view":
            gs.adamw_gs_step_view(groups, n, t, gs.StepConfig(**common, unit=VIEW_UNIT), groups[0].param,
                                  gcams[order[k % len(order)]], stream=stream)
        else:
            gs.gs_visibility(groups[0].param, gcams[order[k % len(order)]], mask=mask, vis_idx=idx, vis_count=cnt, stream=stream)
            gs.adamw_gs_step(groups, n, t, gs.StepConfig(**common, **STEP_LAUNCH), visible=mask, vis_idx=idx,
                             vis_count=cnt, stream=stream)
        if slot >= 0:
            ev.record("start", slot, stream)
        gs.gs_relocate_reset(opacity, k_reloc, groups, gs.GS_MOMENT_F32, t, True, rws, stream=stream)
        if slot >= 0:
            ev.record("end", slot, stream)

    for k in range(warmup):
        one(k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(steps):
        one(warmup + j, j)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if path == "view":
        if counts_from is None:
            raise ValueError("the fused path needs the visible counts of a two-launch run")
        all_counts = np.asarray(counts_from)
    else:
        all_counts = counts.cpu().numpy().astype(np.int64)
    nv = all_counts[warmup:]
    reloc_us = float(np.mean([ev.ms(j) for j in range(steps)]) * 1e3)
    ev.close()
    # exact digest of the end state: integer sums of the bit patterns
    digest = [int(t.to(torch.int64).sum().item())]
    for G in groups:
        for a in (G.param, G.exp_avg, G.exp_avg_sq):
            digest.append(int(a.view(torch.int32).to(torch.int64).sum().item()))
    del groups, params, grads, t, mask, idx, rws
    torch.cuda.empty_cache()
    return {"workload": "6M primitives, 64-cluster mixture means (sigma 1.5), lambda_o = lambda_s = 0.01, "
                        "1 %% lowest opacity reset every step, Morton order, FP32, %d steps" % steps,
            "path": path, "value": int(nv.sum()) * 59 / wall, "ms_per_step": wall / steps * 1e3,
            "visible_frac": float(nv.mean() / n), "relocation_us": reloc_us, "counts": all_counts,
            "digest": digest}


def run_mcmc_both(gs, torch, cams, steps: int = 500, warmup: int = 10):
    """The MCMC-shaped workload on both paths; the fused run must end in the
    two-launch run's state."""
    two = run_mcmc(gs, torch, cams, steps, warmup, "two_launch")
    view = run_mcmc(gs, torch, cams, steps, warmup, "view", counts_from=two["counts"])
    view["same_state_as_two_launch"] = view["digest"] == two["digest"]
    out = []
    for r in (view, two):
        r = dict(r)
        r.pop("counts")
        r.pop("digest")
        out.append(r)
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--order", choices=["morton", "index"], default="morton")
    ap.add_argument("--moments", choices=["f32", "bf16"], default="f32")
    ap.add_argument("--path", choices=["view", "two_launch"], default="view",
                    help="view: visibility fused into the step (one launch); two_launch: gs_visibility + step")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--device-warmup", type=float, default=1.0,
                    help="seconds of discarded fused steps before anything is timed (device clocks)")
    ap.add_argument("--rows-probe", action="store_true",
                    help="only the two-launch FP32 step and the rows probe (its access pattern, no arithmetic)")
    ap.add_argument("--probe-trips", action="store_true",
                    help="only the streaming probe's 4-read / 3-write mix with 1 to 256 tiles per block")
    ap.add_argument("--probe-mib", type=int, default=1024,
                    help="with --probe-sweep: MiB per probe array (4 arrays; the Infinity Cache holds 256 MB)")
    ap.add_argument("--profile-set", action="store_true",
                    help="only a short fixed sequence of step and probe launches, for counter runs")
    ap.add_argument("--probe-sweep", action="store_true",
                    help="only time the streaming probes over every launch shape, for separate and for staggered "
                         "arrays (one JSON line with the table per array layout)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy 10 times (counter calibration)")
    ap.add_argument("--mcmc-only", action="store_true",
                    help="only run the 6M MCMC-shaped workload with relocation (for profiling)")
    ap.add_argument("--unfused-only", action="store_true",
                    help="only run the unfused eager comparator on the 3M Morton scene")
    ap.add_argument("--sweep", action="store_true",
                    help="only run the fused view step over scene sizes 1M-24M and visible fractions (z_far)")
    ap.add_argument("--sweep-n", type=int, default=0,
                    help="with --sweep: only this scene size (at z_far 17.5), e.g. for a profiled run")
    ap.add_argument("--next-only", action="store_true",
                    help="only run the widened rows (noise, AIU, multi-view, prune/append) on the 3M Morton scene")
    ap.add_argument("--tuner-only", action="store_true",
                    help="only run the schedule tuner on the 3M Morton scene's own mask against an i.i.d. one")
    ap.add_argument("--batched-only", action="store_true",
                    help="only run the 16-scene batched workload (for profiling)")
    ap.add_argument("--batched-steps", type=int, default=300,
                    help="timed steps of the batched workload (default 300)")
    ap.add_argument("--batched-forms",
                    default="batched_bf16,batched_bf16_packed,batched_bf16_resident,per_scene_bf16,per_scene_f32",
                    help="comma-separated forms of the batched workload to time")
    args = ap.parse_args(argv)
    if args.calibrate_copy:
        return calibrate_copy()
    if args.profile_set:
        import torch
        import paper_2601_16736_amd as gs
        print(json.dumps(run_profile_set(gs, torch)), flush=True)
        return 0
    if args.rows_probe:
        import torch
        import paper_2601_16736_amd as gs
        import synth
        scene = synth.scene_uniform(N_PRIMS, seed=0, groups=synth.GROUPS_59)
        cams = synth.camera_rig()
        order = synth.camera_order(len(cams), args.warmup + args.steps, seed=0)
        sd = SceneOnDevice(gs, torch, scene, args.order)
        device_warmup(gs, torch, sd, cams, seconds=args.device_warmup)
        two = run_steps(gs, torch, sd, cams, order, "f32", args.steps, args.warmup)
        two.pop("counts")
        two.pop("state")
        rows = rows_ceiling(gs, torch, sd, cams, order, steps=args.steps, warmup=args.warmup)
        rows["two_launch_step_GBps"] = two["achieved_GBps"]
        rows["two_launch_step_us"] = two["step_kernel_us"]
        rows["two_launch_step_frac_of_best"] = two["achieved_GBps"] / rows["best_GBps"]
        print(json.dumps(rows), flush=True)
        two = run_steps(gs, torch, sd, cams, order, "bf16", args.steps, args.warmup)
        two.pop("counts")
        two.pop("state")
        rows = rows_ceiling(gs, torch, sd, cams, order, steps=args.steps, warmup=args.warmup, moments="bf16")
        rows["two_launch_step_GBps"] = two["achieved_GBps"]
        rows["two_launch_step_us"] = two["step_kernel_us"]
        rows["two_launch_step_frac_of_best"] = two["achieved_GBps"] / rows["best_GBps"]
        print(json.dumps(rows), flush=True)
        return 0
    if args.probe_trips:
        import torch
        # the step's mix in its best shapes, with each block taking 1, 2, 4, ...
        # tiles one after another (one-shot grid = 1 tile per block)
        nbytes = args.probe_mib << 20
        shapes = []
        for (w, it) in ((8, 2), (16, 4)):
            tiles = (nbytes // w) // (256 * it)
            shapes += [(w, it, 1, 1, 0)] + [(w, it, 1, 1, tiles // k) for k in (2, 4, 8, 16, 64, 256)]
        out = stream_ceilings(torch, nbytes=nbytes, shapes=shapes)
        out["tiles_per_block"] = {f"w{w}_i{it}_b{b}": (1 if b == 0 else ((nbytes // w) // (256 * it)) // b)
                                  for (w, it, _, _, b) in shapes}
        print(json.dumps(out), flush=True)
        return 0
    if args.probe_sweep:
        import torch
        nbytes = args.probe_mib << 20
        for stagger in (0, 4096 + 256, 1 << 20):
            print(json.dumps(stream_ceilings(torch, nbytes=nbytes, stagger=stagger)), flush=True)
        return 0
    if args.batched_only:
        import torch
        import paper_2601_16736_amd as gs
        print(json.dumps(run_batched(gs, torch, steps=args.batched_steps,
                                     forms=tuple(args.batched_forms.split(",")))), flush=True)
        return 0
    if args.mcmc_only:
        import torch
        import paper_2601_16736_amd as gs
        import synth
        for r in run_mcmc_both(gs, torch, synth.camera_rig(), steps=args.steps, warmup=args.warmup):
            print(json.dumps(r), flush=True)
        return 0
    if args.sweep:
        import torch
        import paper_2601_16736_amd as gs
        for r in run_sweep(gs, torch, only_n=args.sweep_n):
            print(json.dumps(r), flush=True)
        return 0
    if args.next_only:
        import torch
        import paper_2601_16736_amd as gs
        import synth
        scene = synth.scene_uniform(N_PRIMS, seed=0, groups=synth.GROUPS_59)
        cams = synth.camera_rig()
        print(json.dumps(run_next_rows(gs, torch, SceneOnDevice(gs, torch, scene, "morton"), cams)), flush=True)
        return 0
    if args.tuner_only:
        import torch
        import paper_2601_16736_amd as gs
        import synth
        scene = synth.scene_uniform(N_PRIMS, seed=0, groups=synth.GROUPS_59)
        print(json.dumps(run_tuner(gs, torch, SceneOnDevice(gs, torch, scene, "morton"), synth.camera_rig())), flush=True)
        return 0
    if args.unfused_only:
        import torch
        import paper_2601_16736_amd as gs
        import synth
        scene = synth.scene_uniform(N_PRIMS, seed=0, groups=synth.GROUPS_59)
        cams = synth.camera_rig()
        print(json.dumps(run_unfused(gs, torch, SceneOnDevice(gs, torch, scene, "morton"), cams)), flush=True)
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the AdamW-GS step has no cross-GPU exchange to measure "
              f"(--gpus {args.gpus} requested)", file=sys.stderr)
        return 2

    import torch

    import paper_2601_16736_amd as gs
    import synth

    torch.cuda.set_device(0)
    print(f"bench: generating the {N_PRIMS}-primitive scene", file=sys.stderr, flush=True)
    scene = synth.scene_uniform(N_PRIMS, seed=0, groups=synth.GROUPS_59)
    cams = synth.camera_rig()
    order = synth.camera_order(len(cams), args.warmup + args.steps, seed=0)

    layouts = {args.order: SceneOnDevice(gs, torch, scene, args.order)}
    layouts_head = layouts[args.order]
    print(f"bench: device warm-up ({args.device_warmup:.1f} s of discarded steps)", file=sys.stderr, flush=True)
    warm_steps = device_warmup(gs, torch, layouts[args.order], cams, seconds=args.device_warmup)
    # the two-launch path (gs_visibility, then the masked step) always runs
    # first: it is a variant line, and its per-step visible counts are the
    # fused path's too, since both produce the same bits (checked below)
    print(f"bench: {args.order} order, {args.moments} moments, two launches: {args.steps} steps",
          file=sys.stderr, flush=True)
    two = run_steps(gs, torch, layouts[args.order], cams, order, args.moments, args.steps, args.warmup,
                    path="two_launch", keep_state=args.path == "view")
    two_counts = two.pop("counts")
    two_frac_src = two
    variants = []
    same_as_two_launch = None
    if args.path == "view":
        print(f"bench: {args.order} order, {args.moments} moments, visibility fused into the step: "
              f"{args.steps} steps", file=sys.stderr, flush=True)
        head = run_steps(gs, torch, layouts[args.order], cams, order, args.moments, args.steps, args.warmup,
                         path="view", counts_from=two_counts, keep_state=True)
        head.pop("counts")
        same_as_two_launch = same_state(torch, two.pop("state"), head.pop("state"))
        torch.cuda.empty_cache()
        if not same_as_two_launch:
            print("bench: WARNING: the fused and two-launch paths ended in different states", file=sys.stderr,
                  flush=True)
        two.update({"order": args.order, "moments": args.moments, "path": "two_launch",
                    "frac": two["achieved_GBps"] / HBM_PEAK_GBS})
        variants.append(two)
    else:
        two.pop("state")
        head = two
    if not args.no_variants:
        def layout_leg(o, mo):
            if o not in layouts:
                layouts[o] = SceneOnDevice(gs, torch, scene, o)
            fused_too = o == "morton"
            r = run_steps(gs, torch, layouts[o], cams, order, mo, args.steps, args.warmup, keep_state=fused_too)
            counts = r.pop("counts")
            r.update({"order": o, "moments": mo, "path": "two_launch", "frac": r["achieved_GBps"] / HBM_PEAK_GBS})
            out = [r]
            if fused_too:
                f = run_steps(gs, torch, layouts[o], cams, order, mo, args.steps, args.warmup, path="view",
                              counts_from=counts, keep_state=True)
                f.pop("counts")
                f["same_state_as_two_launch"] = same_state(torch, r.pop("state"), f.pop("state"))
                torch.cuda.empty_cache()
                f.update({"order": o, "moments": mo, "path": "view", "frac": f["achieved_GBps"] / HBM_PEAK_GBS})
                out.insert(0, f)
            else:
                r.pop("state")
            return out

        for o, mo in (("index", "f32"), ("morton", "f32"), ("morton", "bf16"), ("index", "bf16")):
            if (o, mo) == (args.order, args.moments):
                continue
            r = guarded(f"{o} order, {mo} moments", layout_leg, o, mo)
            variants.extend(r if isinstance(r, list) else [dict(r, order=o, moments=mo)])
        if "morton" in layouts:
            variants.append({"next_rows": guarded("widened rows (noise, AIU, multi-view, prune/append)",
                                                  run_next_rows, gs, torch, layouts["morton"], cams)})
            unf = guarded("unfused eager comparator", run_unfused, gs, torch, layouts["morton"], cams)
            fused_ms = head["ms_per_step"] if (args.order, args.moments) == ("morton", "f32") else None
            if "error" not in unf:
                unf["fused_speedup"] = unf["ms_per_step"] / fused_ms if fused_ms else None
            variants.append({"unfused_comparator": unf})
            variants.append({"tuner_3m": guarded("tuner on the scene's own mask", run_tuner, gs, torch,
                                                 layouts["morton"], cams)})
        del layouts
        torch.cuda.empty_cache()
        variants.append({"config1_100k": guarded("100k plain (cache-resident)", run_config1, gs, torch)})
        variants.append({"batched": guarded("batched 16 scenes", run_batched, gs, torch)})
        mc = guarded("MCMC-shaped 6M with relocation", run_mcmc_both, gs, torch, cams)
        if isinstance(mc, list):
            variants.append({"mcmc_6m": mc[0]})
            variants.append({"mcmc_6m_two_launch": mc[1]})
        else:
            variants.append({"mcmc_6m": mc})

    traffic = measured_traffic(args.order, args.moments, args.path)
    out = {
        "metric": "primitive-attr updates/s + % HBM roofline, fused AdamW-GS vs plain, 3M Gaussians",
        "value": head["value"],
        "unit": "attr-updates/s",
        "visible_updates_per_s": head["value"] / 59,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.moments == "f32" else "f32 (bf16 moment storage)",
        "data": "synthetic",
        "config": {
            "workload": "3M-primitive scene, 59 FP32 attributes per Gaussian, 200-camera rig (z_far 17.5), "
                        + ("visibility + RSR + Sparse-Adam/DAR step in one launch" if args.path == "view" else
                           "visibility (mask + compaction), then RSR + fused Sparse-Adam/DAR step"),
            "n_primitives": N_PRIMS,
            "primitive_order": args.order,
            "moments": args.moments,
            "visible_mean": head["visible_mean"],
            "visible_frac": head["visible_mean"] / N_PRIMS,
            "path": args.path,
            "schedule": "view windows" if args.path == "view" else "masked windows",
            "unit": ("32 (64 on Re-State iterations)" if VIEW_UNIT == 0 else VIEW_UNIT) if args.path == "view"
                    else STEP_LAUNCH["unit"],
            "same_state_as_two_launch": same_as_two_launch,
            "device_warmup_steps": warm_steps,
            "state_warmup_steps": STATE_WARMUP_STEPS,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": ("step_view_kernel (visibility + Sparse-Adam + DAR, one launch)" if args.path == "view"
                       else "step_kernel (fused Sparse-Adam + DAR)"),
            "achieved": head["achieved_GBps"],
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": head["achieved_GBps"] / HBM_PEAK_GBS,
            "traffic": traffic,
            "traffic_GBps": traffic / (head["step_kernel_us"] * 1e3) if traffic else None,
            "traffic_frac": traffic / (head["step_kernel_us"] * 1e3) / HBM_PEAK_GBS if traffic else None,
            "step_kernel_us": head["step_kernel_us"],
            "step_kernel_us_p10_p50_p90": head["step_kernel_us_p10_p50_p90"],
            "bytes_per_visible": BYTES_PER_VISIBLE[args.moments],
            "bytes_per_primitive": BYTES_PER_PRIMITIVE[args.path],
        },
        "cpu_baseline": None,
        "variants": variants,
    }
    ceil = guarded("streaming ceilings", stream_ceilings, torch)
    if "error" not in ceil:
        ceil.pop("table")
        ceil["step_frac_of_rmw_4r3w"] = head["achieved_GBps"] / ceil["rmw_4r3w_GBps"]
        ceil["step_frac_of_rmw_4r3w_best"] = head["achieved_GBps"] / ceil["rmw_4r3w_best_GBps"]
        ceil["kind"] = ("plain contiguous kernels over 4 x 1 GiB arrays (bench_probe); *_GBps: 16-byte "
                        "non-temporal accesses, 4 in flight per thread, one tile per block; *_best_GBps: the "
                        "fastest of the swept launch shapes (width, in flight, hints, grid form)")
    # the rows probe in both moment precisions, beside the step lines of the
    # same order and precision
    for mo in ("f32", "bf16"):
        rows = guarded(f"rows probe ({mo} moments)", rows_ceiling, gs, torch, layouts_head, cams, order,
                       moments=mo)
        if "error" not in rows:
            for line in [dict(head, path=args.path, moments=args.moments, order=args.order)] + \
                    [v for v in variants if isinstance(v, dict) and "achieved_GBps" in v]:
                if line.get("moments") == mo and line.get("order") == args.order:
                    rows[f"{line['path']}_step_frac_of_best"] = line["achieved_GBps"] / rows["best_GBps"]
        if isinstance(ceil, dict):
            ceil[f"rows_{mo}"] = rows
    out["stream_ceiling"] = ceil
    out["gpu_clocks"] = gpu_clocks()
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = guarded("CPU oracle baseline", cpu_baseline, scene, cams, order,
                                      budget_s=args.cpu_budget)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
