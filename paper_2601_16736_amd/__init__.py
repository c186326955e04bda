"""Python binding of libgsopt, the gfx950 AdamW-GS optimizer-step library.

Argument marshalling only: every step of the path runs in the HIP kernels
of ``libgsopt.so`` (built from ``csrc/`` by ``build.py``).  The names and
arguments mirror the C ABI in ``include/gsopt.h``; tensors are passed as
device pointers and streams as HIP stream handles.  There is no fallback:
if the library is not built, importing this package raises.

Method: "A Step to Decouple Optimization in 3DGS" (arXiv 2601.16736),
Sec. "Recoupling: AdamW-GS" and Sec. "Implementation Details / AdamW-GS".
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsopt.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2601_16736_amd.build` "
                      "(or __graft_entry__.build()) first")

# torch ships its own HIP runtime (soname libamdhip64.so.7, loaded by another
# file name).  Loading torch first makes this library's libamdhip64.so.7
# dependency resolve to that already-loaded runtime, so tensors, streams and
# these kernels share one runtime; loading this library first would bring in
# a second runtime that finds no device.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

GS_OK, GS_EINVAL, GS_EHIP, GS_ENOMEM, GS_EUNSUPPORTED = 0, 1, 2, 3, 4
GS_DAR_NONE, GS_DAR_OPACITY_SIGMOID, GS_DAR_LOGSCALE_EXP = 0, 1, 2
GS_REG_ADAPTIVE, GS_REG_CONSTANT, GS_REG_CONSTANT_CLIPPED = 0, 1, 2
GS_MOMENT_F32, GS_MOMENT_BF16 = 0, 1
GS_SCHED_AUTO, GS_SCHED_COMPACTED, GS_SCHED_MASKED, GS_SCHED_DENSE = 0, 1, 2, 3
GS_MAX_GROUPS = 8

_STATUS = {0: "GS_OK", 1: "GS_EINVAL", 2: "GS_EHIP", 3: "GS_ENOMEM", 4: "GS_EUNSUPPORTED"}


class GsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class gs_camera(ctypes.Structure):
    _fields_ = [("view", ctypes.c_float * 12), ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("z_near", ctypes.c_float), ("z_far", ctypes.c_float),
                ("r_min_px", ctypes.c_float)]


class gs_group(ctypes.Structure):
    _fields_ = [("param", ctypes.c_void_p), ("grad", ctypes.c_void_p), ("exp_avg", ctypes.c_void_p),
                ("exp_avg_sq", ctypes.c_void_p), ("dim", ctypes.c_int32), ("dar_kind", ctypes.c_int32),
                ("reg_mode", ctypes.c_int32), ("row_stride", ctypes.c_int32), ("lr", ctypes.c_double),
                ("dar_lambda", ctypes.c_double), ("dar_clip", ctypes.c_double)]


class gs_step_config(ctypes.Structure):
    _fields_ = [("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("reg_norm", ctypes.c_double), ("seed", ctypes.c_uint64), ("iteration", ctypes.c_int64),
                ("moment_dtype", ctypes.c_int32), ("stochastic_round", ctypes.c_int32),
                ("rsr_enable", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("rsr_alpha1", ctypes.c_double), ("rsr_alpha2", ctypes.c_double),
                ("rsr_ratio", ctypes.c_double), ("visible_hint", ctypes.c_float), ("unit", ctypes.c_int32),
                ("noise_enable", ctypes.c_int32), ("noise_groups", ctypes.c_int32 * 4), ("noise_lr", ctypes.c_double),
                ("noise_k", ctypes.c_double), ("noise_t", ctypes.c_double),
                ("aiu_enable", ctypes.c_int32), ("aiu_ratio", ctypes.c_double), ("aiu_scale", ctypes.c_double)]


class gs_scene(ctypes.Structure):
    _fields_ = [("groups", ctypes.POINTER(gs_group)), ("n_groups", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("n", ctypes.c_int64), ("visible", ctypes.c_void_p),
                ("vis_idx", ctypes.c_void_p), ("vis_count", ctypes.c_void_p),
                ("step_count", ctypes.c_void_p), ("visible_hint", ctypes.c_float),
                ("reserved", ctypes.c_int32)]


_i32, _i64, _u64, _vp, _sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_size_t
_lib.gs_last_error.restype = ctypes.c_char_p
_lib.gs_last_error.argtypes = []
_lib.gs_version.restype = _i32
_lib.gs_reg_norm.restype = ctypes.c_double
_lib.gs_reg_norm.argtypes = [ctypes.c_double]
_lib.gs_visibility.restype = _i32
_lib.gs_visibility.argtypes = [_vp, _i64, _vp, _i64, ctypes.POINTER(gs_camera), _vp, _vp, _vp, _vp]
_lib.adamw_gs_step_view.restype = _i32
_lib.adamw_gs_step_view.argtypes = [ctypes.POINTER(gs_group), _i32, _i64, _vp, _i64, _vp, ctypes.POINTER(gs_camera),
                                    _i32, _vp, _vp, ctypes.POINTER(gs_step_config), _vp]
_lib.gs_visibility_multi.restype = _i32
_lib.gs_visibility_multi.argtypes = [_vp, _i64, _vp, _i64, ctypes.POINTER(gs_camera), _i32, _vp, _vp, _vp, _vp,
                                     _vp]
_lib.gs_compact.restype = _i32
_lib.gs_compact.argtypes = [_vp, _i64, _vp, _vp, _vp]
_lib.adamw_gs_step.restype = _i32
_lib.adamw_gs_step.argtypes = [ctypes.POINTER(gs_group), _i32, _i64, _vp, _vp, _vp, _vp,
                               ctypes.POINTER(gs_step_config), _vp]
_lib.gs_batch_create.restype = _i32
_lib.gs_batch_create.argtypes = [ctypes.POINTER(gs_scene), _i32, _i32, ctypes.POINTER(_vp)]
_lib.adamw_gs_step_batched.restype = _i32
_lib.adamw_gs_step_batched.argtypes = [_vp, ctypes.POINTER(gs_step_config), _vp]
_lib.gs_batch_set_resident.restype = _i32
_lib.gs_batch_set_resident.argtypes = [_vp, _i32]
_lib.gs_batch_scene_schedule.restype = _i32
_lib.gs_batch_scene_schedule.argtypes = [_vp, _i32]
_lib.gs_batch_destroy.restype = _i32
_lib.gs_batch_destroy.argtypes = [_vp]
_lib.gs_relocate_workspace_size.restype = _sz
_lib.gs_relocate_workspace_size.argtypes = [_i64]
_lib.gs_relocate_reset.restype = _i32
_lib.gs_relocate_reset.argtypes = [_vp, _i64, _i64, _i64, ctypes.POINTER(gs_group), _i32, _i32, _vp, _i32, _vp,
                                   _vp, _sz, _vp]
_lib.gs_relocate_reset_noalloc.restype = _i32
_lib.gs_relocate_reset_noalloc.argtypes = [_vp, _i64, _i64, _i64, ctypes.POINTER(gs_group), _i32, _i32, _vp, _i32,
                                           _vp, _vp]
_lib.gs_tune.restype = _i32
_lib.gs_tune.argtypes = [_i64, ctypes.POINTER(_i32), _i32, ctypes.c_float, _i32, ctypes.POINTER(_i32),
                         ctypes.POINTER(_i32)]
_lib.gs_tune_mask.restype = _i32
_lib.gs_tune_mask.argtypes = [_i64, ctypes.POINTER(_i32), _i32, _vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]
_lib.gs_tune_clear.restype = None
_lib.gs_tune_clear.argtypes = []
_lib.gs_spatial_order_workspace_size.restype = _sz
_lib.gs_spatial_order_workspace_size.argtypes = [_i64]
_lib.gs_spatial_order.restype = _i32
_lib.gs_spatial_order.argtypes = [_vp, _i64, _i64, _vp, _vp, _sz, _vp]
_lib.gs_gather_rows.restype = _i32
_lib.gs_gather_rows.argtypes = [_vp, _vp, _vp, _i64, _i64, _vp]
_lib.gs_prune_workspace_size.restype = _sz
_lib.gs_prune_workspace_size.argtypes = [_i64]
_lib.gs_prune.restype = _i32
_lib.gs_prune.argtypes = [_vp, _i64, ctypes.POINTER(gs_group), ctypes.POINTER(gs_group), _i32, _i32, _vp, _vp, _vp,
                          _vp, _sz, _vp]
_lib.gs_append.restype = _i32
_lib.gs_append.argtypes = [ctypes.POINTER(gs_group), _i32, _i32, _i64, _vp, _i64, _vp, _vp]

EXPORTED = ["gs_last_error", "gs_version", "gs_reg_norm", "gs_visibility", "gs_visibility_multi", "gs_compact",
            "adamw_gs_step", "adamw_gs_step_view", "gs_batch_create", "adamw_gs_step_batched", "gs_batch_set_resident", "gs_batch_scene_schedule",
            "gs_batch_destroy",
            "gs_relocate_workspace_size", "gs_relocate_reset", "gs_relocate_reset_noalloc", "gs_tune", "gs_tune_mask", "gs_tune_clear",
            "gs_spatial_order_workspace_size", "gs_spatial_order", "gs_gather_rows", "gs_prune_workspace_size",
            "gs_prune", "gs_append"]


def _check(status: int) -> None:
    if status != GS_OK:
        raise GsError(status, _lib.gs_last_error().decode())


def _ptr(x) -> Optional[int]:
    """Device pointer of a tensor (or an int address, or None)."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


def _stream(stream) -> Optional[int]:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


def last_error() -> str:
    return _lib.gs_last_error().decode()


def _row_stride(t, dim: int) -> int:
    """Elements from one row of t to the next, 0 when the rows are contiguous
    (dim elements apart).  t is [n][dim] (or [n] for dim 1), possibly a
    column slice of a wider packed tensor; objects without strides (plain
    addresses) count as contiguous."""
    if t is None or isinstance(t, int):
        return 0
    try:
        shape, st = t.shape, t.stride()
    except AttributeError:
        return 0
    if len(shape) == 2:
        if shape[0] <= 1 or shape[1] == 0:
            return 0                    # no second row: the stride is never used
        if shape[1] > 1 and st[1] != 1:
            raise ValueError("attribute rows must have unit element stride")
    elif len(shape) != 1 or shape[0] <= 1:
        return 0
    s = int(st[0])
    return 0 if s == dim else s


def version() -> int:
    return int(_lib.gs_version())


def gs_reg_norm(n_pixels: float) -> float:
    """N_I' (DAR paragraph of Sec. "Hyperparameter Selection")."""
    return float(_lib.gs_reg_norm(float(n_pixels)))


# --------------------------------------------------------------------------
@dataclass
class Camera:
    view: Sequence[float]      # 12 floats, row-major 3x4 [R|t] world -> camera
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    z_near: float = 0.2
    z_far: float = math.inf
    r_min_px: float = 0.0

    def to_c(self) -> gs_camera:
        c = gs_camera()
        flat = [float(v) for v in (self.view.reshape(-1) if hasattr(self.view, "reshape") else self.view)]
        if len(flat) != 12:
            raise ValueError("camera view must hold 12 values")
        for k, v in enumerate(flat):
            c.view[k] = v
        c.fx, c.fy, c.cx, c.cy = float(self.fx), float(self.fy), float(self.cx), float(self.cy)
        c.width, c.height = int(self.width), int(self.height)
        c.z_near, c.z_far, c.r_min_px = float(self.z_near), float(self.z_far), float(self.r_min_px)
        return c


def gs_visibility(means, cam: Camera, mask=None, vis_idx=None, vis_count=None, radius=None, stream=None) -> None:
    n = int(means.shape[0])
    c = cam.to_c()
    _check(_lib.gs_visibility(_ptr(means), _row_stride(means, 3), _ptr(radius), n, ctypes.byref(c), _ptr(mask),
                              _ptr(vis_idx), _ptr(vis_count), _stream(stream)))


def gs_visibility_multi(means, cams: Sequence[Camera], mask=None, view_bits=None, vis_idx=None, vis_count=None,
                        radius=None, stream=None) -> None:
    """Up to 32 views at once: per-view bits (uint32 as int32 tensor), union mask, union indices."""
    n = int(means.shape[0])
    arr = (gs_camera * max(len(cams), 1))(*[c.to_c() for c in cams])
    _check(_lib.gs_visibility_multi(_ptr(means), _row_stride(means, 3), _ptr(radius), n, arr, len(cams), _ptr(mask),
                                    _ptr(view_bits), _ptr(vis_idx), _ptr(vis_count), _stream(stream)))


def gs_compact(mask, vis_idx, vis_count, stream=None) -> None:
    _check(_lib.gs_compact(_ptr(mask), int(mask.shape[0]), _ptr(vis_idx), _ptr(vis_count), _stream(stream)))


# --------------------------------------------------------------------------
@dataclass
class Group:
    param: object              # [n, dim] float32 device tensor
    grad: object
    exp_avg: object            # float32 or bfloat16 (per StepConfig.moment_dtype)
    exp_avg_sq: object
    lr: float
    dar_kind: int = GS_DAR_NONE
    dar_lambda: float = 0.0
    dar_clip: float = 0.0
    reg_mode: int = GS_REG_ADAPTIVE
    row_stride: Optional[int] = None   # None: from the tensors' strides

    @property
    def dim(self) -> int:
        return int(self.param.shape[1]) if len(self.param.shape) > 1 else 1

    def stride(self) -> int:
        """The group's row stride (gs_group.row_stride): row_stride if set,
        else read from the tensors, which must then agree."""
        if self.row_stride is not None:
            return int(self.row_stride)
        dim = self.dim
        found = {_row_stride(t, dim) for t in (self.param, self.grad, self.exp_avg, self.exp_avg_sq)
                 if t is not None and hasattr(t, "stride")}
        if len(found) > 1:
            raise ValueError(f"param, grad and moments of a group need one row stride, got {sorted(found)}")
        return found.pop() if found else 0

    def to_c(self) -> gs_group:
        g = gs_group()
        g.param, g.grad, g.exp_avg, g.exp_avg_sq = (_ptr(self.param), _ptr(self.grad), _ptr(self.exp_avg),
                                                    _ptr(self.exp_avg_sq))
        g.dim = self.dim
        g.dar_kind, g.reg_mode, g.row_stride = int(self.dar_kind), int(self.reg_mode), self.stride()
        g.lr, g.dar_lambda, g.dar_clip = float(self.lr), float(self.dar_lambda), float(self.dar_clip)
        return g


@dataclass
class StepConfig:
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-15
    reg_norm: float = 1e5
    seed: int = 0
    iteration: int = 0
    moment_dtype: int = GS_MOMENT_F32
    stochastic_round: bool = True
    rsr_enable: bool = False
    schedule: int = GS_SCHED_AUTO
    rsr_alpha1: float = 0.2
    rsr_alpha2: float = 0.04
    rsr_ratio: float = 0.0
    visible_hint: float = 0.0
    unit: int = 0
    noise_enable: bool = False
    noise_groups: tuple = (0, 1, 2, 3)      # mean, log-scale, quaternion, opacity-logit groups
    noise_lr: float = 0.0                   # eta_{R_o}
    noise_k: float = 100.0                  # lambda_mu
    noise_t: float = 0.005                  # lambda_t
    aiu_enable: bool = False                # Artificial Implicit Update of sampled invisible rows
    aiu_ratio: float = 0.0                  # Pro_AIU
    aiu_scale: float = 0.0                  # eta_AIU

    def to_c(self) -> gs_step_config:
        c = gs_step_config()
        c.beta1, c.beta2, c.eps, c.reg_norm = self.beta1, self.beta2, self.eps, self.reg_norm
        c.seed = int(self.seed) & (2**64 - 1)
        c.iteration = int(self.iteration)
        c.moment_dtype = int(self.moment_dtype)
        c.stochastic_round = int(bool(self.stochastic_round))
        c.rsr_enable = int(bool(self.rsr_enable))
        c.schedule = int(self.schedule)
        c.rsr_alpha1, c.rsr_alpha2, c.rsr_ratio = self.rsr_alpha1, self.rsr_alpha2, self.rsr_ratio
        c.visible_hint = float(self.visible_hint)
        c.unit = int(self.unit)
        c.noise_enable = int(bool(self.noise_enable))
        for k in range(4):
            c.noise_groups[k] = int(self.noise_groups[k])
        c.noise_lr, c.noise_k, c.noise_t = float(self.noise_lr), float(self.noise_k), float(self.noise_t)
        c.aiu_enable = int(bool(self.aiu_enable))
        c.aiu_ratio, c.aiu_scale = float(self.aiu_ratio), float(self.aiu_scale)
        return c


def _groups_c(groups: Sequence[Group]):
    arr = (gs_group * max(len(groups), 1))()
    for k, g in enumerate(groups):
        arr[k] = g.to_c()
    return arr


def adamw_gs_step(groups: Sequence[Group], n: int, step_count, cfg: StepConfig, visible=None, vis_idx=None,
                  vis_count=None, stream=None) -> None:
    """One AdamW-GS step (see include/gsopt.h for the exact contract)."""
    arr = _groups_c(groups)
    c = cfg.to_c()
    _check(_lib.adamw_gs_step(arr, len(groups), int(n), _ptr(visible), _ptr(vis_idx), _ptr(vis_count),
                              _ptr(step_count), ctypes.byref(c), _stream(stream)))


def adamw_gs_step_view(groups: Sequence[Group], n: int, step_count, cfg: StepConfig, means, cams,
                       radius=None, visible_out=None, stream=None) -> None:
    """Visibility and step in one launch (see include/gsopt.h).  ``cams`` is a
    Camera or a sequence of up to 32 (their union decides V)."""
    prepare_step_view(groups, n, step_count, cfg, means, cams, radius, visible_out, stream)()


def prepare_step_view(groups: Sequence[Group], n: int, step_count, cfg: StepConfig, means, cams,
                      radius=None, visible_out=None, stream=None):
    """The arguments of one adamw_gs_step_view call, marshalled now: returns a
    function without arguments that makes that call.  The host-side packing
    (tens of microseconds per call) can then be done ahead of time, e.g.
    for a loop whose launches should follow one another without host gaps.
    The returned function keeps the argument objects alive; the tensors'
    addresses, shapes and the groups' fields are read here, so changing them
    afterwards does not affect the prepared call."""
    cams = [cams] if isinstance(cams, Camera) else list(cams)
    arr = _groups_c(groups)
    c = cfg.to_c()
    cc = (gs_camera * max(len(cams), 1))(*[x.to_c() for x in cams])
    args = (arr, len(groups), int(n), _ptr(means), _row_stride(means, 3), _ptr(radius), cc, len(cams),
            _ptr(visible_out), _ptr(step_count), ctypes.byref(c), _stream(stream))
    keep = (list(groups), [G.grad for G in groups], step_count, means, radius, visible_out, c)

    def launch() -> None:
        _check(_lib.adamw_gs_step_view(*args))

    launch.keep = keep          # the argument objects live as long as the call
    return launch


# --------------------------------------------------------------------------
@dataclass
class Scene:
    groups: List[Group]
    n: int
    step_count: object
    visible: object = None
    vis_idx: object = None
    vis_count: object = None
    schedule: int = GS_SCHED_AUTO
    visible_hint: float = 0.0


class Batch:
    """Plan for stepping many scenes in one launch."""

    def __init__(self, scenes: Sequence[Scene], moment_dtype: int = GS_MOMENT_F32):
        self._scenes = list(scenes)              # keeps tensors alive
        self.moment_dtype = int(moment_dtype)
        self._garr = [_groups_c(s.groups) for s in self._scenes]
        sarr = (gs_scene * len(self._scenes))()
        for k, s in enumerate(self._scenes):
            sarr[k].groups = ctypes.cast(self._garr[k], ctypes.POINTER(gs_group))
            sarr[k].n_groups = len(s.groups)
            sarr[k].schedule = int(s.schedule)
            sarr[k].n = int(s.n)
            sarr[k].visible, sarr[k].vis_idx, sarr[k].vis_count = (_ptr(s.visible), _ptr(s.vis_idx),
                                                                   _ptr(s.vis_count))
            sarr[k].step_count = _ptr(s.step_count)
            sarr[k].visible_hint = float(s.visible_hint)
            sarr[k].reserved = 0
        h = _vp()
        _check(_lib.gs_batch_create(sarr, len(self._scenes), self.moment_dtype, ctypes.byref(h)))
        self._h = h

    def schedule(self, s: int) -> int:
        return int(_lib.gs_batch_scene_schedule(self._h, s))

    def set_resident(self, resident: bool) -> None:
        """Persistent grid (True) or one wave per unit (False, the default)."""
        _check(_lib.gs_batch_set_resident(self._h, int(bool(resident))))

    def step(self, cfg: StepConfig, stream=None) -> None:
        adamw_gs_step_batched(self, cfg, stream)

    def close(self) -> None:
        if getattr(self, "_h", None):
            _check(_lib.gs_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gs_batch_create(scenes: Sequence[Scene], moment_dtype: int = GS_MOMENT_F32) -> Batch:
    return Batch(scenes, moment_dtype)


def adamw_gs_step_batched(batch: Batch, cfg: StepConfig, stream=None) -> None:
    c = cfg.to_c()
    _check(_lib.adamw_gs_step_batched(batch._h, ctypes.byref(c), _stream(stream)))


def gs_batch_destroy(batch: Batch) -> None:
    batch.close()


# --------------------------------------------------------------------------
def gs_relocate_workspace_size(n: int) -> int:
    return int(_lib.gs_relocate_workspace_size(int(n)))


def gs_relocate_reset(key, k: int, groups: Sequence[Group], moment_dtype: int, step_count, reset_t: bool,
                      workspace, selected=None, stream=None) -> None:
    arr = _groups_c(groups)
    n = int(key.shape[0])
    ws_bytes = int(workspace.numel() * workspace.element_size())
    _check(_lib.gs_relocate_reset(_ptr(key), _row_stride(key, 1), n, int(k), arr, len(groups), int(moment_dtype),
                                  _ptr(step_count), int(bool(reset_t)), _ptr(selected), _ptr(workspace), ws_bytes,
                                  _stream(stream)))


# largest n gs_relocate_reset_noalloc serves (GS_RELOCATE_NOALLOC_MAX_N in gsopt.h)
GS_RELOCATE_NOALLOC_MAX_N = 1 << 27


def gs_relocate_reset_noalloc(key, k: int, groups: Sequence[Group], moment_dtype: int, step_count,
                              reset_t: bool, selected=None, stream=None) -> None:
    """gs_relocate_reset on the library's own fixed device workspace: no
    allocation, n <= GS_RELOCATE_NOALLOC_MAX_N (see include/gsopt.h)."""
    arr = _groups_c(groups)
    n = int(key.shape[0])
    _check(_lib.gs_relocate_reset_noalloc(_ptr(key), _row_stride(key, 1), n, int(k), arr, len(groups),
                                          int(moment_dtype), _ptr(step_count), int(bool(reset_t)), _ptr(selected),
                                          _stream(stream)))


def gs_tune(n: int, dims: Sequence[int], visible_fraction: float, moment_dtype: int = GS_MOMENT_F32):
    """Times the schedules on synthetic buffers; returns (schedule, unit)."""
    d = (ctypes.c_int32 * len(dims))(*[int(x) for x in dims])
    s, u = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(_lib.gs_tune(int(n), d, len(dims), float(visible_fraction), int(moment_dtype), ctypes.byref(s),
                        ctypes.byref(u)))
    return int(s.value), int(u.value)


def gs_tune_mask(n: int, dims: Sequence[int], mask, moment_dtype: int = GS_MOMENT_F32):
    """Times the schedules with the caller's visibility mask (device uint8
    tensor or address); returns (schedule, unit)."""
    d = (ctypes.c_int32 * len(dims))(*[int(x) for x in dims])
    s, u = ctypes.c_int32(0), ctypes.c_int32(0)
    _check(_lib.gs_tune_mask(int(n), d, len(dims), _ptr(mask), int(moment_dtype), ctypes.byref(s),
                             ctypes.byref(u)))
    return int(s.value), int(u.value)


def gs_tune_clear() -> None:
    _lib.gs_tune_clear()


# --------------------------------------------------------------------------
def gs_spatial_order_workspace_size(n: int) -> int:
    return int(_lib.gs_spatial_order_workspace_size(int(n)))


def gs_spatial_order(means, perm, workspace, stream=None) -> None:
    """perm <- primitive indices in Morton order of their means."""
    ws_bytes = int(workspace.numel() * workspace.element_size())
    _check(_lib.gs_spatial_order(_ptr(means), _row_stride(means, 3), int(means.shape[0]), _ptr(perm),
                                 _ptr(workspace), ws_bytes, _stream(stream)))


def gs_gather_rows(src, dst, perm, stream=None) -> None:
    """dst[i] = src[perm[i]] row by row (rows = leading dimension)."""
    n = int(src.shape[0])
    row_bytes = int(src[0].numel() * src.element_size()) if n else 1
    _check(_lib.gs_gather_rows(_ptr(src), _ptr(dst), _ptr(perm), n, row_bytes, _stream(stream)))


def apply_spatial_order(tensors, perm, stream=None):
    """Returns copies of the given per-primitive tensors permuted by perm."""
    out = []
    for t in tensors:
        d = t.new_empty(t.shape)
        gs_gather_rows(t.contiguous(), d, perm, stream)
        out.append(d)
    return out


# --------------------------------------------------------------------------
def gs_prune_workspace_size(n: int) -> int:
    return int(_lib.gs_prune_workspace_size(int(n)))


def gs_prune(keep, src: Sequence[Group], dst: Sequence[Group], moment_dtype: int, t_src, t_dst, kept_count,
             workspace, stream=None) -> None:
    """Order-preserving compaction of theta, m, v and t by ``keep`` into dst."""
    if len(src) != len(dst):
        raise ValueError("src and dst need the same groups")
    a, b = _groups_c(src), _groups_c(dst)
    n = int(keep.shape[0])
    ws_bytes = int(workspace.numel() * workspace.element_size()) if workspace is not None else 0
    _check(_lib.gs_prune(_ptr(keep), n, a, b, len(src), int(moment_dtype), _ptr(t_src), _ptr(t_dst),
                         _ptr(kept_count), _ptr(workspace), ws_bytes, _stream(stream)))


def gs_append(groups: Sequence[Group], moment_dtype: int, n: int, src_idx, step_count, stream=None) -> None:
    """Rows n .. n+k-1 become clones of rows src_idx with zero state."""
    arr = _groups_c(groups)
    k = int(src_idx.shape[0]) if src_idx is not None else 0
    _check(_lib.gs_append(arr, len(groups), int(moment_dtype), int(n), _ptr(src_idx), k, _ptr(step_count),
                          _stream(stream)))
