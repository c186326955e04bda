"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/gsopt.h declares, and rejects invalid arguments with
GS_EINVAL before anything is enqueued (no call here reaches a launch)."""
import ctypes
import os
import re

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gsopt.h")

gs = pytest.importorskip("paper_2601_16736_amd", reason="libgsopt.so not built")

# These calls pass fake device addresses and rely on validation failing
# before any launch.  Where a GPU is present a call that validation let
# through would launch on them, so the module runs only on GPU-less hosts
# (counting devices does not initialise the runtime).
import torch  # noqa: E402

if torch.cuda.device_count() > 0:
    pytest.skip("host-side ABI checks use fake device pointers; run them where no GPU is present",
                allow_module_level=True)

FAKE = 0x7F0000000000          # an aligned address that is never dereferenced


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_library_exports_every_declared_function():
    names = declared_functions()
    assert len(names) >= 14
    lib = ctypes.CDLL(gs.LIB_PATH)
    for n in names:
        assert hasattr(lib, n), f"{n} declared in gsopt.h but not exported"
    assert set(gs.EXPORTED) == set(names)


def test_version_and_reg_norm():
    assert gs.version() == 2
    for n_i in (1e6, 1089480, 404301, 999999, 10, 7, 0.5):
        assert gs.gs_reg_norm(n_i) == oracle.reg_norm(n_i)


def _group(**kw):
    d = dict(param=FAKE, grad=FAKE + 4096, exp_avg=FAKE + 8192, exp_avg_sq=FAKE + 12288, lr=1e-3)
    d.update(kw)
    return gs.Group(**d)


class _Fake:
    """Stands in for a tensor: only shape and data_ptr are read."""

    def __init__(self, addr, shape):
        self._a, self.shape = addr, shape

    def data_ptr(self):
        return self._a


def _step(groups=None, n=10, cfg=None, **kw):
    groups = [_group(param=_Fake(FAKE, (n, 3)))] if groups is None else groups
    cfg = cfg or gs.StepConfig(schedule=gs.GS_SCHED_DENSE)
    with pytest.raises(gs.GsError) as e:
        gs.adamw_gs_step(groups, n, kw.pop("t", FAKE + 65536), cfg, stream=0, **kw)
    return e.value


@pytest.mark.parametrize("cfg", [
    gs.StepConfig(beta1=1.0, schedule=gs.GS_SCHED_DENSE),
    gs.StepConfig(beta1=-0.1, schedule=gs.GS_SCHED_DENSE),
    gs.StepConfig(beta2=1.0, schedule=gs.GS_SCHED_DENSE),
    gs.StepConfig(eps=0.0, schedule=gs.GS_SCHED_DENSE),
    gs.StepConfig(eps=1e-60, schedule=gs.GS_SCHED_DENSE),      # rounds to 0 in FP32
    gs.StepConfig(eps=float("nan"), schedule=gs.GS_SCHED_DENSE),
    gs.StepConfig(moment_dtype=5, schedule=gs.GS_SCHED_DENSE),
    gs.StepConfig(rsr_enable=True, rsr_alpha1=1.0, schedule=gs.GS_SCHED_DENSE),
    gs.StepConfig(rsr_enable=True, rsr_alpha2=-0.5, schedule=gs.GS_SCHED_DENSE),
    gs.StepConfig(rsr_enable=True, rsr_ratio=1.5, schedule=gs.GS_SCHED_DENSE),
    gs.StepConfig(schedule=9),
    gs.StepConfig(schedule=gs.GS_SCHED_COMPACTED),             # no vis_idx
    gs.StepConfig(schedule=gs.GS_SCHED_MASKED),                # no mask
    gs.StepConfig(schedule=gs.GS_SCHED_DENSE, unit=100),       # unknown unit
    gs.StepConfig(schedule=gs.GS_SCHED_DENSE, iteration=-1),
    gs.StepConfig(schedule=gs.GS_SCHED_DENSE, aiu_enable=True, aiu_ratio=1.5),
    gs.StepConfig(schedule=gs.GS_SCHED_DENSE, aiu_enable=True, aiu_ratio=0.5, aiu_scale=-1.0),
    gs.StepConfig(schedule=gs.GS_SCHED_DENSE, aiu_enable=True, aiu_ratio=0.5, aiu_scale=float("inf")),
])
def test_step_rejects_bad_config(cfg):
    e = _step(cfg=cfg)
    assert e.status == gs.GS_EINVAL, str(e)


def test_step_rejects_bad_groups_and_sizes():
    assert _step(n=-1).status == gs.GS_EINVAL
    assert _step(n=2**31).status == gs.GS_EINVAL
    assert _step(groups=[]).status == gs.GS_EINVAL
    assert _step(groups=[_group(param=_Fake(FAKE, (10, 3)))] * 9).status == gs.GS_EINVAL
    assert _step(groups=[_group(param=_Fake(FAKE + 2, (10, 3)))]).status == gs.GS_EINVAL   # misaligned
    assert _step(groups=[_group(param=_Fake(0, (10, 3)))]).status == gs.GS_EINVAL          # NULL
    assert _step(groups=[_group(param=_Fake(FAKE, (10, 3)), dar_kind=7)]).status == gs.GS_EINVAL
    assert _step(groups=[_group(param=_Fake(FAKE, (10, 3)), reg_mode=3)]).status == gs.GS_EINVAL
    assert _step(groups=[_group(param=_Fake(FAKE, (10, 3)), lr=float("inf"))]).status == gs.GS_EINVAL
    assert _step(groups=[_group(param=_Fake(FAKE, (10, 3)), dar_lambda=-1.0)]).status == gs.GS_EINVAL
    assert _step(groups=[_group(param=_Fake(FAKE, (10, 3)), dar_kind=1)],
                 cfg=gs.StepConfig(reg_norm=0.0, schedule=gs.GS_SCHED_DENSE)).status == gs.GS_EINVAL
    assert _step(t=0).status == gs.GS_EINVAL                                             # step_count NULL
    e = _step(n=-5)
    assert "n = -5" in str(e) and gs.last_error() in str(e)


def test_visibility_rejects_bad_arguments():
    cam = gs.Camera([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 15], 866.0, 866.0, 500, 500, 1000, 1000)
    means = _Fake(FAKE, (10, 3))
    cases = [
        dict(mask=None, vis_idx=None),                          # no output
        dict(mask=FAKE + 4096, vis_idx=FAKE + 8192),            # idx without count
        dict(mask=FAKE + 4097),                                 # fine: mask is bytes -> next case
    ]
    with pytest.raises(gs.GsError):
        gs.gs_visibility(means, cam, stream=0, **cases[0])
    with pytest.raises(gs.GsError):
        gs.gs_visibility(means, cam, stream=0, **cases[1])
    bad = gs.Camera([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 15], 866.0, 866.0, 500, 500, 0, 1000)
    with pytest.raises(gs.GsError):
        gs.gs_visibility(means, bad, mask=FAKE + 4096, stream=0)
    bad = gs.Camera([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 15], 866.0, 866.0, 500, 500, 1000, 1000, z_near=5, z_far=5)
    with pytest.raises(gs.GsError):
        gs.gs_visibility(means, bad, mask=FAKE + 4096, stream=0)
    bad = gs.Camera([float("nan")] + [0] * 11, 866.0, 866.0, 500, 500, 1000, 1000)
    with pytest.raises(gs.GsError):
        gs.gs_visibility(means, bad, mask=FAKE + 4096, stream=0)
    with pytest.raises(gs.GsError):
        gs.gs_visibility(_Fake(FAKE + 1, (10, 3)), cam, mask=FAKE + 4096, stream=0)
    with pytest.raises(gs.GsError):
        gs.gs_compact(_Fake(FAKE, (10,)), FAKE + 4096, None, stream=0)


def test_tune_rejects_bad_arguments():
    for args in ((0, [3], 0.3), (100, [], 0.3), (100, [3], 0.0), (100, [3], 1.5), (100, [0], 0.3)):
        with pytest.raises(gs.GsError):
            gs.gs_tune(*args)
    for args in ((0, [3], FAKE), (100, [], FAKE), (100, [0], FAKE), (100, [3], None)):
        with pytest.raises(gs.GsError):
            gs.gs_tune_mask(*args)
    with pytest.raises(gs.GsError):
        gs.gs_tune_mask(100, [3], FAKE, moment_dtype=7)


def test_struct_layouts_match_the_header(tmp_path):
    """The binding's ctypes mirrors have the C header's sizes and offsets
    (a C program built against include/gsopt.h prints them)."""
    import subprocess
    structs = {"gs_camera": gs.gs_camera, "gs_group": gs.gs_group, "gs_step_config": gs.gs_step_config,
               "gs_scene": gs.gs_scene}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "gsopt.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for f in cls._fields_:
            lines.append(f'printf("{name} {f[0]} %zu\\n", offsetof({name}, {f[0]}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                           "-I", "/opt/rocm/include", str(src), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split("\n")
    for row in filter(None, out):
        name, field, val = row.split()
        cls = structs[name]
        got = ctypes.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert got == int(val), f"{name}.{field}: ctypes {got}, C {val}"


def test_visibility_multi_rejects_bad_arguments():
    """Every call here fails validation before any launch."""
    cam = gs.Camera([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 15], 866.0, 866.0, 500, 500, 1000, 1000)
    bad = gs.Camera([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 15], 866.0, 866.0, 500, 500, 1000, 1000, z_near=5, z_far=5)
    means = _Fake(FAKE, (10, 3))
    for cams, kw in (([cam], {}),                                            # no output
                     ([], dict(mask=FAKE + 4096)),                           # no view
                     ([cam] * 33, dict(mask=FAKE + 4096)),                   # too many views
                     ([cam], dict(vis_idx=FAKE + 8192)),                     # idx without count
                     ([cam], dict(view_bits=FAKE + 4098)),                   # misaligned bits
                     ([cam, bad], dict(mask=FAKE + 4096))):                  # second view invalid
        with pytest.raises(gs.GsError) as e:
            gs.gs_visibility_multi(means, cams, stream=0, **kw)
        assert e.value.status == gs.GS_EINVAL
    with pytest.raises(gs.GsError) as e:
        gs.gs_visibility_multi(means, [cam, bad], mask=FAKE + 4096, stream=0)
    assert "view 1" in str(e.value)


def test_view_step_rejects_bad_arguments():
    """Every call here fails validation before any launch."""
    cam = gs.Camera([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 15], 866.0, 866.0, 500, 500, 1000, 1000)
    bad = gs.Camera([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 15], 866.0, 866.0, 500, 500, 1000, 1000, z_near=5, z_far=5)
    groups = [_group(param=_Fake(FAKE, (10, 3)))]
    cases = [dict(n=-1), dict(means=None), dict(t=None), dict(cam=bad), dict(unit=512), dict(unit=16),
             dict(means=FAKE + 2), dict(beta1=1.0), dict(cam=[]), dict(cam=[cam] * 33), dict(cam=[cam, bad])]
    for c in cases:
        n = c.get("n", 10)
        cfg = gs.StepConfig(unit=c.get("unit", 0), beta1=c.get("beta1", 0.9))
        with pytest.raises(gs.GsError) as e:
            gs.adamw_gs_step_view(groups, n, c.get("t", FAKE + 65536), cfg, c.get("means", FAKE + 131072),
                                  c.get("cam", cam), stream=0)
        assert e.value.status == gs.GS_EINVAL, c


def _prune(n=10, src=None, dst=None, dtype=0, keep=FAKE + 65536, t_src=FAKE + 131072, t_dst=FAKE + 196608,
           cnt=FAKE + 262144, ws=None):
    src = [_group(param=_Fake(FAKE, (n, 3)))] if src is None else src
    dst = [_group(param=_Fake(FAKE + 1 << 20, (n, 3)), grad=None)] if dst is None else dst
    with pytest.raises(gs.GsError) as e:
        gs.gs_prune(_Fake(keep, (n,)), src, dst, dtype, t_src, t_dst, cnt, ws, stream=0)
    return e.value


def test_prune_rejects_bad_arguments():
    """Every call here fails validation before any launch."""
    assert _prune(n=-1).status == gs.GS_EINVAL
    assert _prune(n=2**31).status == gs.GS_EINVAL
    assert _prune(dtype=3).status == gs.GS_EINVAL
    assert _prune(cnt=0).status == gs.GS_EINVAL                        # kept_count NULL
    assert _prune(cnt=FAKE + 2).status == gs.GS_EINVAL                 # misaligned
    assert _prune(keep=0).status == gs.GS_EINVAL
    assert _prune(t_dst=FAKE + 6).status == gs.GS_EINVAL
    assert _prune(ws=None).status == gs.GS_EINVAL                      # workspace too small
    small = _Fake(FAKE + (1 << 22), (8,))
    small.numel, small.element_size = (lambda: 8), (lambda: 1)
    assert _prune(ws=small).status == gs.GS_EINVAL
    assert _prune(dst=[_group(param=_Fake(FAKE, (10, 4)))]).status == gs.GS_EINVAL      # dims differ
    assert _prune(src=[_group(param=_Fake(FAKE + 2, (10, 3)))]).status == gs.GS_EINVAL  # misaligned
    assert _prune(src=[_group(param=_Fake(FAKE, (10, 3)))] * 9,
                  dst=[_group(param=_Fake(FAKE, (10, 3)))] * 9).status == gs.GS_EINVAL
    with pytest.raises(ValueError):
        gs.gs_prune(_Fake(FAKE, (10,)), [_group()], [], 0, FAKE, FAKE, FAKE, None, stream=0)
    assert gs.gs_prune_workspace_size(0) == 0
    assert gs.gs_prune_workspace_size(10**6) > 2 * 4 * (10**6 // 512)


def test_append_rejects_bad_arguments():
    def app(n=10, k=4, dtype=0, src=FAKE + 65536, t=FAKE + 131072, groups=None):
        groups = [_group(param=_Fake(FAKE, (n + k, 3)))] if groups is None else groups
        with pytest.raises(gs.GsError) as e:
            gs.gs_append(groups, dtype, n, _Fake(src, (k,)), t, stream=0)
        return e.value
    assert app(n=-1).status == gs.GS_EINVAL
    assert app(n=2**31 - 2, k=4).status == gs.GS_EINVAL
    assert app(dtype=2).status == gs.GS_EINVAL
    assert app(src=0).status == gs.GS_EINVAL
    assert app(t=0).status == gs.GS_EINVAL
    assert app(t=FAKE + 2).status == gs.GS_EINVAL
    assert app(groups=[_group(param=_Fake(FAKE, (14, 3)), exp_avg=FAKE + 1)]).status == gs.GS_EINVAL
    assert app(groups=[]).status == gs.GS_EINVAL


def test_relocate_entry_points_reject_bad_arguments():
    """Both relocation entry points validate the same arguments before any
    launch; the no-allocation one also refuses n above its fixed maximum."""
    ws = _Fake(FAKE + (1 << 24), (1 << 20,))
    ws.numel, ws.element_size = (lambda: 1 << 20), (lambda: 1)

    def with_ws(n=10, k=4, dtype=0, key=FAKE + 65536, t=FAKE + 131072, sel=FAKE + 196608, reset_t=True,
                groups=None, workspace=ws):
        groups = [_group(param=_Fake(FAKE, (n, 3)))] if groups is None else groups
        with pytest.raises(gs.GsError) as e:
            gs.gs_relocate_reset(_Fake(key, (n,)), k, groups, dtype, t, reset_t, workspace, selected=sel, stream=0)
        return e.value.status

    def noalloc(n=10, k=4, dtype=0, key=FAKE + 65536, t=FAKE + 131072, sel=FAKE + 196608, reset_t=True,
                groups=None):
        groups = [_group(param=_Fake(FAKE, (n, 3)))] if groups is None else groups
        with pytest.raises(gs.GsError) as e:
            gs.gs_relocate_reset_noalloc(_Fake(key, (n,)), k, groups, dtype, t, reset_t, selected=sel, stream=0)
        return e.value.status

    for call in (with_ws, noalloc):
        assert call(n=-1) == gs.GS_EINVAL
        assert call(k=-1) == gs.GS_EINVAL
        assert call(k=11) == gs.GS_EINVAL
        assert call(dtype=2) == gs.GS_EINVAL
        assert call(key=0) == gs.GS_EINVAL
        assert call(key=FAKE + 2) == gs.GS_EINVAL
        assert call(sel=FAKE + 1) == gs.GS_EINVAL
        assert call(t=0) == gs.GS_EINVAL                          # reset_t needs step_count
        assert call(groups=[_group(param=_Fake(FAKE, (10, 3)), exp_avg=FAKE + 1)]) == gs.GS_EINVAL
    assert with_ws(n=2**31) == gs.GS_EINVAL
    null_ws = _Fake(0, (1 << 20,))
    null_ws.numel, null_ws.element_size = (lambda: 1 << 20), (lambda: 1)
    assert with_ws(workspace=null_ws) == gs.GS_EINVAL
    odd_ws = _Fake(FAKE + 64, (1 << 20,))
    odd_ws.numel, odd_ws.element_size = (lambda: 1 << 20), (lambda: 1)
    assert with_ws(workspace=odd_ws) == gs.GS_EINVAL              # workspace needs 256-byte alignment
    small = _Fake(FAKE + (1 << 24), (8,))
    small.numel, small.element_size = (lambda: 8), (lambda: 1)
    assert with_ws(workspace=small) == gs.GS_EINVAL
    assert noalloc(n=gs.GS_RELOCATE_NOALLOC_MAX_N + 1) == gs.GS_EINVAL
    assert "GS_RELOCATE_NOALLOC_MAX_N" in gs.last_error()
    # the binding's constant is the header's
    text = open(HEADER).read()
    assert re.search(r"#define GS_RELOCATE_NOALLOC_MAX_N \(\(int64_t\)1 << 27\)", text)
    assert gs.GS_RELOCATE_NOALLOC_MAX_N == 1 << 27
    # n = 0 is a no-op that reads no other argument
    gs.gs_relocate_reset_noalloc(_Fake(0, (0,)), 0, [], 0, 0, False, stream=0)


def test_row_strides_are_validated():
    """Strided rows: a group's row_stride must be 0 (contiguous) or cover its
    dim, within the row-stride limit; a means or key stride must be 0 or
    large enough for its row.  Every call here fails before any launch."""
    for rs in (-1, 2, 65537):
        assert _step(groups=[_group(param=_Fake(FAKE, (10, 3)), row_stride=rs)]).status == gs.GS_EINVAL
    assert _step(groups=[_group(param=_Fake(FAKE, (10, 3)), row_stride=2**16)], n=2**25).status == gs.GS_EINVAL
    cam = gs.Camera([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 15], 866.0, 866.0, 500, 500, 1000, 1000)

    class Strided(_Fake):
        def __init__(self, addr, shape, strides):
            super().__init__(addr, shape)
            self._s = strides

        def stride(self, i=None):
            return self._s if i is None else self._s[i]

    for bad in ((2, 1), (70000, 1)):
        means = Strided(FAKE, (10, 3), bad)
        with pytest.raises(gs.GsError) as e:
            gs.gs_visibility(means, cam, mask=FAKE + 4096, stream=0)
        assert e.value.status == gs.GS_EINVAL and "means_stride" in str(e.value)
        with pytest.raises(gs.GsError):
            gs.adamw_gs_step_view([_group(param=_Fake(FAKE, (10, 3)))], 10, FAKE + 65536, gs.StepConfig(), means,
                                  cam, stream=0)
        with pytest.raises(gs.GsError):
            gs.gs_visibility_multi(means, [cam], mask=FAKE + 4096, stream=0)
    with pytest.raises(ValueError):                     # rows must have unit element stride
        gs.gs_visibility(Strided(FAKE, (10, 3), (6, 2)), cam, mask=FAKE + 4096, stream=0)
    ws = _Fake(FAKE + (1 << 24), (1 << 20,))
    ws.numel, ws.element_size = (lambda: 1 << 20), (lambda: 1)
    with pytest.raises(gs.GsError) as e:
        gs.gs_spatial_order(Strided(FAKE, (10, 3), (2, 1)), FAKE + 65536, ws, stream=0)
    assert e.value.status == gs.GS_EINVAL
    with pytest.raises(gs.GsError) as e:
        gs.gs_relocate_reset(Strided(FAKE, (10,), (70000,)), 1, [_group(param=_Fake(FAKE, (10, 3)))], 0,
                             FAKE + 65536, True, ws, stream=0)
    assert e.value.status == gs.GS_EINVAL
    # a group's tensors must agree on their row stride
    g = gs.Group(Strided(FAKE, (10, 3), (64, 1)), Strided(FAKE + 4096, (10, 3), (3, 1)), FAKE + 8192,
                 FAKE + 12288, 1e-3)
    with pytest.raises(ValueError):
        g.to_c()
    assert gs.Group(Strided(FAKE, (10, 3), (64, 1)), Strided(FAKE + 4096, (10, 3), (64, 1)), FAKE + 8192,
                    FAKE + 12288, 1e-3).to_c().row_stride == 64


def test_prepared_view_step_makes_the_same_call(monkeypatch):
    """prepare_step_view packs the arguments at once and its launch passes
    exactly what adamw_gs_step_view passes; a group changed after the
    packing does not change the prepared call.  The library entry point is
    replaced by a recorder, so nothing is launched."""
    calls = []

    class _Rec:
        def adamw_gs_step_view(self, *args):
            calls.append([bytes(a._obj) if type(a).__name__ == "CArgObject" else
                          (bytes(a) if isinstance(a, ctypes.Array) else a) for a in args])
            return gs.GS_OK

    monkeypatch.setattr(gs, "_lib", _Rec())
    cam = gs.Camera([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 15], 866.0, 866.0, 500, 500, 1000, 1000)
    groups = [_group(param=_Fake(FAKE, (10, 3)), grad=_Fake(FAKE + 4096, (10, 3))),
              _group(param=_Fake(FAKE + 65536, (10, 48)), grad=_Fake(FAKE + 69632, (10, 48)), dar_kind=1,
                     dar_lambda=0.01, dar_clip=2.0)]
    cfg = gs.StepConfig(iteration=7, rsr_enable=True, rsr_ratio=0.1, unit=64)
    launch = gs.prepare_step_view(groups, 10, FAKE + 1 << 20, cfg, _Fake(FAKE, (10, 3)), cam, stream=3)
    gs.adamw_gs_step_view(groups, 10, FAKE + 1 << 20, cfg, _Fake(FAKE, (10, 3)), cam, stream=3)
    launch()
    assert calls[0] == calls[1]
    groups[1].grad = _Fake(FAKE + 131072, (10, 48))
    launch()
    assert calls[2] == calls[0]
    gs.adamw_gs_step_view(groups, 10, FAKE + 1 << 20, cfg, _Fake(FAKE, (10, 3)), cam, stream=3)
    assert calls[3] != calls[0]
