"""FP64 CPU oracle for the AdamW-GS optimizer step -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It binds ``gsoracle.c`` (plain C,
FP64, one primitive and one element at a time) with ctypes over numpy arrays
and shares nothing with the HIP library in ``paper_2601_16736_amd``.

Paper: "A Step to Decouple Optimization in 3DGS" (arXiv 2601.16736).
Each wrapper names the passage its C function follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsoracle.c")
_LIB = os.path.join(_HERE, "libgsoracle.so")

# Plain IEEE arithmetic: no contraction into FMA, no fast-math, SSE (not x87)
# on x86-64, so every binary32 operation of the visibility predicate is one
# correctly rounded step.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
          "-fno-fast-math", "-fno-unsafe-math-optimizations", "-Wall"]

DAR_NONE, DAR_OPACITY_SIGMOID, DAR_LOGSCALE_EXP = 0, 1, 2
REG_ADAPTIVE, REG_CONSTANT, REG_CONSTANT_CLIPPED = 0, 1, 2
TAG_RSR = 1


def build(force: bool = True) -> str:
    """Compile gsoracle.c into libgsoracle.so next to it (gcc)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Camera(ctypes.Structure):
    _fields_ = [("view", ctypes.c_float * 12), ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("z_near", ctypes.c_float), ("z_far", ctypes.c_float),
                ("r_min", ctypes.c_float)]


class _Group(ctypes.Structure):
    _fields_ = [("param", ctypes.c_void_p), ("grad", ctypes.c_void_p), ("m", ctypes.c_void_p),
                ("v", ctypes.c_void_p), ("dim", ctypes.c_int32), ("lr", ctypes.c_double),
                ("dar_kind", ctypes.c_int32), ("dar_lambda", ctypes.c_double),
                ("dar_clip", ctypes.c_double), ("reg_mode", ctypes.c_int32)]


class _Config(ctypes.Structure):
    _fields_ = [("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("reg_norm", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("iteration", ctypes.c_int64), ("rsr_enable", ctypes.c_int32),
                ("rsr_alpha1", ctypes.c_double), ("rsr_alpha2", ctypes.c_double),
                ("rsr_ratio", ctypes.c_double), ("noise_enable", ctypes.c_int32),
                ("noise_groups", ctypes.c_int32 * 4), ("noise_lr", ctypes.c_double),
                ("noise_k", ctypes.c_double), ("noise_t", ctypes.c_double),
                ("aiu_enable", ctypes.c_int32), ("aiu_ratio", ctypes.c_double), ("aiu_scale", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        u64, i64, i32, vp = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p
        L.orc_mix64.restype = u64; L.orc_mix64.argtypes = [u64]
        L.orc_splitmix_output.restype = u64; L.orc_splitmix_output.argtypes = [u64, u64]
        L.orc_stream_state.restype = u64; L.orc_stream_state.argtypes = [u64, u64, i64]
        L.orc_draw.restype = u64; L.orc_draw.argtypes = [u64, u64, i64, u64]
        L.orc_rsr_threshold.restype = u64; L.orc_rsr_threshold.argtypes = [ctypes.c_double]
        L.orc_rsr_sampled.restype = ctypes.c_int; L.orc_rsr_sampled.argtypes = [u64, i64, i64, ctypes.c_double]
        L.orc_rsr_sample_mask.restype = None
        L.orc_rsr_sample_mask.argtypes = [u64, i64, vp, i64, ctypes.c_double, vp]
        L.orc_aiu_sample_mask.restype = None
        L.orc_aiu_sample_mask.argtypes = [u64, i64, vp, i64, ctypes.c_double, vp]
        L.orc_reg_norm.restype = ctypes.c_double; L.orc_reg_norm.argtypes = [ctypes.c_double]
        L.orc_visible_f32.restype = ctypes.c_int; L.orc_visible_f32.argtypes = [vp, vp, vp]
        L.orc_visibility.restype = None; L.orc_visibility.argtypes = [vp, vp, i64, vp, vp]
        L.orc_visibility_f64.restype = None; L.orc_visibility_f64.argtypes = [vp, vp, i64, vp, vp]
        L.orc_visibility_multi.restype = None; L.orc_visibility_multi.argtypes = [vp, vp, i64, vp, i32, vp, vp]
        L.orc_compact.restype = i64; L.orc_compact.argtypes = [vp, i64, vp]
        L.orc_adamw_gs_step.restype = None; L.orc_adamw_gs_step.argtypes = [vp, i32, i64, vp, vp, vp]
        L.orc_adamw_gs_step_rows.restype = None
        L.orc_adamw_gs_step_rows.argtypes = [vp, i32, i64, vp, vp, vp, vp]
        L.orc_noise_gamma.restype = None; L.orc_noise_gamma.argtypes = [u64, i64, i64, vp]
        L.orc_noise_displacement.restype = None
        L.orc_noise_displacement.argtypes = [vp, vp, ctypes.c_double, ctypes.c_double, vp, vp, vp]
        L.orc_select_smallest.restype = None; L.orc_select_smallest.argtypes = [vp, i64, i64, vp]
        L.orc_reset_state.restype = None; L.orc_reset_state.argtypes = [vp, i32, vp, i64, vp, i32]
        L.orc_prune.restype = i64; L.orc_prune.argtypes = [vp, vp, i32, i64, vp, vp, vp]
        L.orc_append.restype = None; L.orc_append.argtypes = [vp, i32, i64, vp, i64, vp]
        L.orc_bf16_rne.restype = ctypes.c_uint16; L.orc_bf16_rne.argtypes = [ctypes.c_float]
        L.orc_bf16_sr.restype = ctypes.c_uint16; L.orc_bf16_sr.argtypes = [ctypes.c_float, ctypes.c_uint32]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


def _need(a: np.ndarray, dtype) -> np.ndarray:
    if a.dtype != dtype or not a.flags.c_contiguous:
        raise TypeError(f"oracle expects C-contiguous {np.dtype(dtype)} arrays, got {a.dtype}")
    return a


# --------------------------------------------------------------------------
# random draws (SplitMix64, Steele, Lea & Flood 2014)
# --------------------------------------------------------------------------
def mix64(z: int) -> int:
    return int(lib().orc_mix64(z & (2**64 - 1)))


def splitmix_output(state: int, k: int) -> int:
    return int(lib().orc_splitmix_output(state & (2**64 - 1), k & (2**64 - 1)))


def stream_state(seed: int, tag: int, iteration: int) -> int:
    return int(lib().orc_stream_state(seed & (2**64 - 1), tag, iteration))


def draw(seed: int, tag: int, iteration: int, element: int) -> int:
    return int(lib().orc_draw(seed & (2**64 - 1), tag, iteration, element))


def rsr_threshold(ratio: float) -> int:
    return int(lib().orc_rsr_threshold(float(ratio)))


def rsr_sampled(seed: int, iteration: int, i: int, ratio: float) -> bool:
    return bool(lib().orc_rsr_sampled(seed & (2**64 - 1), iteration, i, float(ratio)))


def rsr_sample_mask(seed: int, iteration: int, n: int, ratio: float,
                    ids: Optional[np.ndarray] = None) -> np.ndarray:
    """Re-State sample flags (bool) of primitives 0..n-1, or of ``ids``."""
    if ids is not None:
        ids = _need(np.ascontiguousarray(ids), np.int64)
        n = ids.shape[0]
    out = np.zeros(n, np.uint8)
    lib().orc_rsr_sample_mask(seed & (2**64 - 1), iteration, _ptr(ids), n, float(ratio), _ptr(out))
    return out.astype(bool)


def aiu_sample_mask(seed: int, iteration: int, n: int, ratio: float,
                    ids: Optional[np.ndarray] = None) -> np.ndarray:
    """AIU sample flags (bool) of primitives 0..n-1, or of ``ids``."""
    if ids is not None:
        ids = _need(np.ascontiguousarray(ids), np.int64)
        n = ids.shape[0]
    out = np.zeros(n, np.uint8)
    lib().orc_aiu_sample_mask(seed & (2**64 - 1), iteration, _ptr(ids), n, float(ratio), _ptr(out))
    return out.astype(bool)


def reg_norm(n_pixels: float) -> float:
    """N_I' of the DAR paragraph in Sec. "Hyperparameter Selection"."""
    return float(lib().orc_reg_norm(float(n_pixels)))


# --------------------------------------------------------------------------
# visibility
# --------------------------------------------------------------------------
@dataclass
class Camera:
    view: np.ndarray            # (3, 4) float32, world -> camera [R|t]
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    z_near: float = 0.2
    z_far: float = float("inf")
    r_min: float = 0.0

    def _c(self) -> _Camera:
        c = _Camera()
        v = np.ascontiguousarray(self.view, dtype=np.float32).reshape(12)
        for k in range(12):
            c.view[k] = float(v[k])
        c.fx, c.fy, c.cx, c.cy = (float(np.float32(x)) for x in (self.fx, self.fy, self.cx, self.cy))
        c.width, c.height = int(self.width), int(self.height)
        c.z_near, c.z_far, c.r_min = (float(np.float32(x)) for x in (self.z_near, self.z_far, self.r_min))
        return c


def visibility(means: np.ndarray, cam: Camera, radius: Optional[np.ndarray] = None) -> np.ndarray:
    """FP32 frustum/radius predicate per primitive (uint8 mask)."""
    means = _need(np.ascontiguousarray(means), np.float32)
    n = means.shape[0]
    if radius is not None:
        radius = _need(np.ascontiguousarray(radius), np.float32)
    mask = np.zeros(n, np.uint8)
    c = cam._c()
    lib().orc_visibility(_ptr(means), _ptr(radius), n, ctypes.addressof(c), _ptr(mask))
    return mask


def visibility_multi(means: np.ndarray, cams: List[Camera], radius: Optional[np.ndarray] = None):
    """(union mask uint8, per-view bits uint32) over up to 32 views."""
    means = _need(np.ascontiguousarray(means), np.float32)
    n = means.shape[0]
    if radius is not None:
        radius = _need(np.ascontiguousarray(radius), np.float32)
    if not 1 <= len(cams) <= 32:
        raise ValueError("1..32 views")
    arr = (type(cams[0]._c()) * len(cams))(*[c._c() for c in cams])
    mask = np.zeros(n, np.uint8)
    bits = np.zeros(n, np.uint32)
    lib().orc_visibility_multi(_ptr(means), _ptr(radius), n, ctypes.addressof(arr), len(cams), _ptr(mask),
                               _ptr(bits))
    return mask, bits


def visibility_f64(means: np.ndarray, cam: Camera, radius: Optional[np.ndarray] = None) -> np.ndarray:
    means = _need(np.ascontiguousarray(means), np.float32)
    n = means.shape[0]
    if radius is not None:
        radius = _need(np.ascontiguousarray(radius), np.float32)
    mask = np.zeros(n, np.uint8)
    c = cam._c()
    lib().orc_visibility_f64(_ptr(means), _ptr(radius), n, ctypes.addressof(c), _ptr(mask))
    return mask


def compact(mask: np.ndarray) -> np.ndarray:
    mask = _need(np.ascontiguousarray(mask), np.uint8)
    idx = np.zeros(mask.shape[0], np.int32)
    k = lib().orc_compact(_ptr(mask), mask.shape[0], _ptr(idx))
    return idx[:k].copy()


# --------------------------------------------------------------------------
# the step
# --------------------------------------------------------------------------
@dataclass
class Group:
    """One attribute group: arrays are float64 [n, dim], updated in place."""
    param: np.ndarray
    grad: np.ndarray
    m: np.ndarray
    v: np.ndarray
    lr: float
    dar_kind: int = DAR_NONE
    dar_lambda: float = 0.0
    dar_clip: float = 0.0
    reg_mode: int = REG_ADAPTIVE

    @property
    def dim(self) -> int:
        return int(self.param.shape[1])


@dataclass
class Config:
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-15
    reg_norm: float = 1e5
    seed: int = 0
    iteration: int = 0
    rsr_enable: bool = False
    rsr_alpha1: float = 0.2
    rsr_alpha2: float = 0.04
    rsr_ratio: float = 0.0
    noise_enable: bool = False
    noise_groups: tuple = (0, 1, 2, 3)     # mean, log-scale, quaternion, opacity-logit groups
    noise_lr: float = 0.0                  # eta_{R_o}
    noise_k: float = 100.0                 # lambda_mu
    noise_t: float = 0.005                 # lambda_t
    aiu_enable: bool = False
    aiu_ratio: float = 0.0                 # Pro_AIU
    aiu_scale: float = 0.0                 # eta_AIU


def _groups_struct(groups: List[Group]):
    arr = (_Group * len(groups))()
    for k, g in enumerate(groups):
        for a in (g.param, g.grad, g.m, g.v):
            _need(a, np.float64)
            if a.ndim != 2 or a.shape != g.param.shape:
                raise ValueError("group arrays must share one [n, dim] shape")
        arr[k].param, arr[k].grad, arr[k].m, arr[k].v = (_ptr(g.param), _ptr(g.grad), _ptr(g.m), _ptr(g.v))
        arr[k].dim = g.dim
        arr[k].lr = float(g.lr)
        arr[k].dar_kind = int(g.dar_kind)
        arr[k].dar_lambda = float(g.dar_lambda)
        arr[k].dar_clip = float(g.dar_clip)
        arr[k].reg_mode = int(g.reg_mode)
    return arr


def _config_struct(cfg: Config) -> _Config:
    c = _Config()
    c.beta1, c.beta2, c.eps, c.reg_norm = cfg.beta1, cfg.beta2, cfg.eps, cfg.reg_norm
    c.seed = cfg.seed & (2**64 - 1)
    c.iteration = cfg.iteration
    c.rsr_enable = int(bool(cfg.rsr_enable))
    c.rsr_alpha1, c.rsr_alpha2, c.rsr_ratio = cfg.rsr_alpha1, cfg.rsr_alpha2, cfg.rsr_ratio
    c.noise_enable = int(bool(cfg.noise_enable))
    for k in range(4):
        c.noise_groups[k] = int(cfg.noise_groups[k])
    c.noise_lr, c.noise_k, c.noise_t = cfg.noise_lr, cfg.noise_k, cfg.noise_t
    c.aiu_enable = int(bool(cfg.aiu_enable))
    c.aiu_ratio, c.aiu_scale = cfg.aiu_ratio, cfg.aiu_scale
    return c


def noise_gamma(seed: int, iteration: int, i: int) -> np.ndarray:
    """gamma ~ N(0, I3) of primitive i (Box-Muller on the counter draws)."""
    g = np.zeros(3)
    lib().orc_noise_gamma(seed & (2**64 - 1), iteration, i, _ptr(g))
    return g


def noise_displacement(q, kappa, tau: float, lr_mu: float, cfg: Config, gamma) -> np.ndarray:
    """eta_{R_o} R_mu of one primitive (position equations, Implementation Details)."""
    q = np.ascontiguousarray(q, np.float64)
    kappa = np.ascontiguousarray(kappa, np.float64)
    gamma = np.ascontiguousarray(gamma, np.float64)
    out = np.zeros(3)
    c = _config_struct(cfg)
    lib().orc_noise_displacement(_ptr(q), _ptr(kappa), float(tau), float(lr_mu), ctypes.addressof(c), _ptr(gamma),
                                 _ptr(out))
    return out


def adamw_gs_step(groups: List[Group], n: int, visible: Optional[np.ndarray], t: np.ndarray,
                  cfg: Config, ids: Optional[np.ndarray] = None) -> None:
    """One AdamW-GS step (Sec. "Recoupling: AdamW-GS"; Eqs. of the sparse
    beta, Re-State, decoupled moments and DAR update), in place.
    ``visible=None`` is V = 1 everywhere (synchronous Adam).  ``ids`` (int64,
    optional) gives each row's primitive index in its scene when the rows are
    a subset; it keys the Re-State draw."""
    _need(t, np.int32)
    if visible is not None:
        _need(visible, np.uint8)
    if ids is not None:
        _need(ids, np.int64)
        if ids.shape[0] != n:
            raise ValueError("ids must have n entries")
    for g in groups:
        if g.param.shape[0] != n:
            raise ValueError("group row count differs from n")
    arr = _groups_struct(groups)
    c = _config_struct(cfg)
    lib().orc_adamw_gs_step_rows(ctypes.addressof(arr), len(groups), n, _ptr(ids), _ptr(visible), _ptr(t),
                                 ctypes.addressof(c))


def select_smallest(key: np.ndarray, k: int) -> np.ndarray:
    """Indices (ascending) of the k smallest keys, ties to the lower index."""
    key = _need(np.ascontiguousarray(key), np.float32)
    sel = np.zeros(max(k, 0), np.int64)
    lib().orc_select_smallest(_ptr(key), key.shape[0], k, _ptr(sel))
    return sel


def reset_state(groups: List[Group], sel: np.ndarray, t: Optional[np.ndarray], reset_t: bool) -> None:
    sel = _need(np.ascontiguousarray(sel), np.int64)
    arr = _groups_struct(groups)
    lib().orc_reset_state(ctypes.addressof(arr), len(groups), _ptr(sel), sel.shape[0], _ptr(t),
                          int(bool(reset_t)))


def prune(src: List[Group], keep: np.ndarray, t: np.ndarray):
    """Order-preserving compaction of theta, m, v and t by ``keep``; returns
    (groups of the kept rows, their step counts)."""
    keep = _need(np.ascontiguousarray(keep), np.uint8)
    _need(t, np.int32)
    n = keep.shape[0]
    k = int(np.count_nonzero(keep))
    dst = [Group(np.zeros((max(k, 1), g.dim)), np.zeros((max(k, 1), g.dim)), np.zeros((max(k, 1), g.dim)),
                 np.zeros((max(k, 1), g.dim)), g.lr, g.dar_kind, g.dar_lambda, g.dar_clip, g.reg_mode) for g in src]
    t_dst = np.zeros(max(k, 1), np.int32)
    a, b = _groups_struct(src), _groups_struct(dst)
    w = lib().orc_prune(ctypes.addressof(a), ctypes.addressof(b), len(src), n, _ptr(keep), _ptr(t), _ptr(t_dst))
    assert w == k
    for g in dst:
        g.param, g.grad, g.m, g.v = g.param[:k], g.grad[:k], g.m[:k], g.v[:k]
    return dst, t_dst[:k]


def append(groups: List[Group], n: int, src_idx: np.ndarray, t: np.ndarray) -> None:
    """Rows n .. n+k-1 (the arrays hold at least n+k rows) become clones of
    rows src_idx with zero state, in place."""
    src_idx = _need(np.ascontiguousarray(src_idx), np.int64)
    _need(t, np.int32)
    k = src_idx.shape[0]
    for g in groups:
        if g.param.shape[0] < n + k or t.shape[0] < n + k:
            raise ValueError("arrays must hold n + k rows")
        if k and (src_idx.min() < 0 or src_idx.max() >= n):
            raise ValueError("source rows must be below n")
    arr = _groups_struct(groups)
    lib().orc_append(ctypes.addressof(arr), len(groups), n, _ptr(src_idx), k, _ptr(t))


def bf16_rne(x: float) -> int:
    return int(lib().orc_bf16_rne(float(x)))


def bf16_sr(x: float, r16: int) -> int:
    return int(lib().orc_bf16_sr(float(x), int(r16) & 0xFFFF))
