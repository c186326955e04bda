"""Packed layout: the attribute groups as column ranges of one [n][64] array
per role (attributes, gradients, each moment), so a primitive's state fills
whole 128-byte lines (gs_group.row_stride, means_stride, key_stride).  The
kernels only address the rows differently, so every result must equal, bit
for bit, that of the same scene in the contiguous one-tensor-per-group
layout (itself checked against the FP64 oracle in the other parity tests),
and the padding columns must never be written.  One case is also checked
against the oracle directly."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

gs = pytest.importorskip("paper_2601_16736_amd")
from _gpu_util import DEV, TOL_THETA, oracle_config, theta_err  # noqa: E402

# column ranges of the packed row: SH first (16-byte aligned rows of 48),
# the quaternion at 48 (aligned), then the 3-float and 1-float groups
COLS = {"sh": 0, "quats": 48, "means": 52, "scales": 55, "opacity": 58}
WIDTH = 64
SPEC = [s for s in synth.GROUPS_59]       # means, scales, quats, opacity, sh
PAD = 1.5e38                               # value of the padding columns


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)


class Twin:
    """One scene in both layouts, with identical values."""

    def __init__(self, n, seed, bf16=False):
        r = synth.rng(seed, 300)
        self.n, self.bf16 = n, bf16
        mdt = torch.bfloat16 if bf16 else torch.float32
        self.mdt = mdt
        self.pack = {role: torch.full((n, WIDTH), PAD, dtype=torch.float32 if role in ("p", "g") else mdt,
                                      device=DEV) for role in ("p", "g", "m", "v")}
        self.flat = []
        self.packed = []
        for name, dim, lr, dar in SPEC:
            vals = {"p": r.standard_normal((n, dim), dtype=np.float32),
                    "g": (1e-3 * r.standard_normal((n, dim))).astype(np.float32),
                    "m": (1e-4 * r.standard_normal((n, dim))).astype(np.float32),
                    "v": (1e-6 * r.random((n, dim)) + 1e-9).astype(np.float32)}
            if name == "means":
                vals["p"] = r.uniform(-10, 10, (n, dim)).astype(np.float32)
            c0 = COLS[name]
            flat = {}
            for role, a in vals.items():
                dt = torch.float32 if role in ("p", "g") else mdt
                t = torch.from_numpy(a).to(DEV).to(dt)
                self.pack[role][:, c0:c0 + dim] = t
                flat[role] = t.clone()
            lam = 1e-3 if dar == 1 else 1e-5
            self.flat.append(gs.Group(flat["p"], flat["g"], flat["m"], flat["v"], lr, dar_kind=dar,
                                      dar_lambda=lam if dar else 0.0, dar_clip=10.0))
            view = {role: self.pack[role][:, c0:c0 + dim] for role in self.pack}
            self.packed.append(gs.Group(view["p"], view["g"], view["m"], view["v"], lr, dar_kind=dar,
                                        dar_lambda=lam if dar else 0.0, dar_clip=10.0))
        t0 = torch.from_numpy(r.integers(0, 30, n).astype(np.int32)).to(DEV)
        self.t_flat, self.t_pack = t0.clone(), t0.clone()

    def means(self, packed):
        return self.packed[0].param if packed else self.flat[0].param

    def check_same(self, label=""):
        torch.cuda.synchronize()
        assert torch.equal(self.t_flat, self.t_pack), f"{label}: step counts"
        for (name, dim, *_), F, P in zip(SPEC, self.flat, self.packed):
            for a, b, what in ((F.param, P.param, "param"), (F.exp_avg, P.exp_avg, "m"), (F.exp_avg_sq, P.exp_avg_sq, "v")):
                x, y = (a.view(torch.int16), b.contiguous().view(torch.int16)) if a.dtype == torch.bfloat16 else \
                       (a.view(torch.int32), b.contiguous().view(torch.int32))
                assert torch.equal(x, y), f"{label}: {name}.{what} differs between the layouts"
        for role, t in self.pack.items():
            pad = t[:, 59:].float()
            assert bool((pad == torch.tensor(PAD, dtype=t.dtype).float()).all()), f"{label}: padding of {role} written"


@pytest.mark.parametrize("sched,unit", [(gs.GS_SCHED_MASKED, 32), (gs.GS_SCHED_COMPACTED, 64),
                                        (gs.GS_SCHED_DENSE, 64), (gs.GS_SCHED_MASKED, 256)])
@pytest.mark.parametrize("bf16", [False, True])
def test_step_packed_equals_contiguous(sched, unit, bf16):
    n = 40_009
    tw = Twin(n, 1 + unit + int(bf16), bf16)
    for k in range(3):
        mask = synth.bernoulli_mask(n, 0.3, seed=7, step=k)
        d_mask = torch.from_numpy(mask).to(DEV)
        idx = torch.zeros(n, dtype=torch.int32, device=DEV)
        cnt = torch.zeros(1, dtype=torch.int32, device=DEV)
        gs.gs_compact(d_mask, idx, cnt)
        cfg = gs.StepConfig(iteration=k, schedule=sched, unit=unit, moment_dtype=int(bf16), stochastic_round=True,
                            rsr_enable=k == 1, rsr_ratio=0.2)
        print(f"packed step sched={sched} unit={unit} bf16={bf16} k={k}", flush=True)
        for groups, t in ((tw.flat, tw.t_flat), (tw.packed, tw.t_pack)):
            gs.adamw_gs_step(groups, n, t, cfg, visible=d_mask, vis_idx=idx, vis_count=cnt)
        tw.check_same(f"sched {sched} unit {unit} step {k}")


def test_packed_step_against_oracle():
    n = 20_011
    tw = Twin(n, 5)
    mask = synth.bernoulli_mask(n, 0.4, seed=9, step=0)
    before = {name: {role: tw.pack[role][:, COLS[name]:COLS[name] + dim].float().cpu().numpy().astype(np.float64)
                     for role in tw.pack} for name, dim, *_ in SPEC}
    t_ref = tw.t_pack.cpu().numpy().copy()
    cfg = gs.StepConfig(iteration=4, schedule=gs.GS_SCHED_MASKED, rsr_enable=True, rsr_ratio=0.3)
    gs.adamw_gs_step(tw.packed, n, tw.t_pack, cfg, visible=torch.from_numpy(mask).to(DEV))
    torch.cuda.synchronize()
    og = [oracle.Group(before[name]["p"].copy(), before[name]["g"].copy(), before[name]["m"].copy(),
                       before[name]["v"].copy(), lr, dar_kind=dar, dar_lambda=(1e-3 if dar == 1 else 1e-5) if dar else 0.0,
                       dar_clip=10.0) for name, dim, lr, dar in SPEC]
    oracle.adamw_gs_step(og, n, mask, t_ref, oracle_config(cfg))
    assert np.array_equal(tw.t_pack.cpu().numpy(), t_ref)
    for (name, dim, *_), O in zip(SPEC, og):
        x = tw.pack["p"][:, COLS[name]:COLS[name] + dim].cpu().numpy()
        e = theta_err(x, O.param)
        assert e <= TOL_THETA, f"{name}: {e:.3e}"


@pytest.mark.parametrize("bf16", [False, True])
@pytest.mark.parametrize("extra", [{}, {"rsr_enable": True, "rsr_ratio": 0.1},
                                   {"aiu_enable": True, "aiu_ratio": 0.2, "aiu_scale": 1.0},
                                   {"noise_enable": True, "noise_lr": 5e5, "noise_k": 100.0, "noise_t": 0.005}])
def test_view_step_packed_equals_contiguous(bf16, extra):
    n = 60_013
    tw = Twin(n, 11 + int(bf16), bf16)
    cams = synth.camera_rig(n_cams=6)
    gc = [gs.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far) for c in cams]
    masks = []
    for k in range(3):
        cfg = gs.StepConfig(iteration=k + 2, moment_dtype=int(bf16), **extra)
        print(f"packed view bf16={bf16} extra={sorted(extra)} k={k}", flush=True)
        out = []
        for groups, t, packed in ((tw.flat, tw.t_flat, False), (tw.packed, tw.t_pack, True)):
            vis = torch.zeros(n, dtype=torch.uint8, device=DEV)
            gs.adamw_gs_step_view(groups, n, t, cfg, tw.means(packed), gc[k], visible_out=vis)
            out.append(vis)
        assert torch.equal(out[0], out[1])
        masks.append(int(out[0].sum()))
        tw.check_same(f"view {sorted(extra)} step {k}")
    assert 0 < min(masks) and max(masks) < n


def test_visibility_and_spatial_order_with_strided_means():
    n = 30_001
    tw = Twin(n, 21)
    cams = synth.camera_rig(n_cams=4)
    gc = [gs.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far) for c in cams]
    res = []
    for packed in (False, True):
        mask = torch.zeros(n, dtype=torch.uint8, device=DEV)
        idx = torch.zeros(n, dtype=torch.int32, device=DEV)
        cnt = torch.zeros(1, dtype=torch.int32, device=DEV)
        gs.gs_visibility(tw.means(packed), gc[0], mask=mask, vis_idx=idx, vis_count=cnt)
        mmask = torch.zeros(n, dtype=torch.uint8, device=DEV)
        bits = torch.zeros(n, dtype=torch.int32, device=DEV)
        gs.gs_visibility_multi(tw.means(packed), gc, mask=mmask, view_bits=bits)
        perm = torch.empty(n, dtype=torch.int32, device=DEV)
        ws = torch.empty(gs.gs_spatial_order_workspace_size(n), dtype=torch.uint8, device=DEV)
        gs.gs_spatial_order(tw.means(packed), perm, ws)
        torch.cuda.synchronize()
        k = int(cnt.item())
        res.append((mask.cpu(), np.sort(idx[:k].cpu().numpy()), mmask.cpu(), bits.cpu(), perm.cpu()))
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(np.asarray(a), np.asarray(b))
    ref = oracle.visibility(tw.flat[0].param.cpu().numpy(), oracle.Camera(*[getattr(cams[0], f) for f in
                            ("view", "fx", "fy", "cx", "cy", "width", "height", "z_near", "z_far")]))
    assert np.array_equal(res[1][0].numpy(), ref)


@pytest.mark.parametrize("noalloc", [False, True])
def test_relocation_with_strided_key(noalloc):
    n = 70_001
    tw = Twin(n, 31)
    k = 700
    sels = []
    for groups, t, packed in ((tw.flat, tw.t_flat, False), (tw.packed, tw.t_pack, True)):
        key = groups[3].param if packed else groups[3].param.view(-1)
        if packed:
            key = tw.pack["p"][:, COLS["opacity"]]            # a strided column, not a copy
            assert key.stride(0) == WIDTH
        sel = torch.full((k,), -1, dtype=torch.int32, device=DEV)
        if noalloc:
            gs.gs_relocate_reset_noalloc(key, k, groups, 0, t, True, selected=sel)
        else:
            ws = torch.empty(gs.gs_relocate_workspace_size(n), dtype=torch.uint8, device=DEV)
            gs.gs_relocate_reset(key, k, groups, 0, t, True, ws, selected=sel)
        sels.append(sel)
    tw.check_same("relocation")
    assert torch.equal(sels[0], sels[1])
    ref = oracle.select_smallest(tw.flat[3].param.view(-1).cpu().numpy(), k)
    assert np.array_equal(sels[0].cpu().numpy().astype(np.int64), ref)


def test_prune_and_append_packed():
    n = 20_003
    tw = Twin(n, 41)
    keep = torch.from_numpy((synth.rng(42).random(n) < 0.6).astype(np.uint8)).to(DEV)
    ws = torch.empty(gs.gs_prune_workspace_size(n), dtype=torch.uint8, device=DEV)
    out = []
    for groups, t, packed in ((tw.flat, tw.t_flat, False), (tw.packed, tw.t_pack, True)):
        if packed:
            dpack = {role: torch.full_like(a, 3.0) for role, a in tw.pack.items()}
            dst = [gs.Group(dpack["p"][:, COLS[nm]:COLS[nm] + d], None, dpack["m"][:, COLS[nm]:COLS[nm] + d],
                            dpack["v"][:, COLS[nm]:COLS[nm] + d], g.lr) for (nm, d, *_), g in zip(SPEC, groups)]
        else:
            dst = [gs.Group(torch.full_like(g.param, 3.0), None, torch.full_like(g.exp_avg, 3.0),
                            torch.full_like(g.exp_avg_sq, 3.0), g.lr) for g in groups]
        t_dst = torch.full_like(t, -4)
        cnt = torch.zeros(1, dtype=torch.int32, device=DEV)
        gs.gs_prune(keep, groups, dst, 0, t, t_dst, cnt, ws)
        out.append((dst, t_dst, cnt))
    torch.cuda.synchronize()
    kept = int(out[0][2].item())
    assert kept == int(out[1][2].item()) == int(keep.sum())
    assert torch.equal(out[0][1], out[1][1])
    for F, P in zip(out[0][0], out[1][0]):
        for a, b in ((F.param, P.param), (F.exp_avg, P.exp_avg), (F.exp_avg_sq, P.exp_avg_sq)):
            assert torch.equal(a[:kept], b[:kept].contiguous())
            assert bool((b[kept:] == 3.0).all())
    # appending clones into spare rows of the packed arrays
    k_new = 500
    src = torch.from_numpy(synth.rng(43).integers(0, n - k_new, k_new).astype(np.int32)).to(DEV)
    m = n - k_new                       # the last k_new rows become the new ones
    for groups, t in ((tw.flat, tw.t_flat), (tw.packed, tw.t_pack)):
        gs.gs_append(groups, 0, m, src, t)
    tw.check_same("append")
    assert bool((tw.t_pack[m:] == 0).all())


def test_packed_scenes_take_the_packed_schedule(capfd, monkeypatch):
    """The launch log names the packed-row schedule for a packed scene (its
    results are checked above), and not for the contiguous one."""
    n = 5003
    tw = Twin(n, 51)
    mask = torch.from_numpy(synth.bernoulli_mask(n, 0.3, 51, 0)).to(DEV)
    c = synth.camera_rig()[2]
    cam = gs.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far)
    monkeypatch.setenv("GSOPT_TRACE", "1")
    capfd.readouterr()
    for groups, t, packed in ((tw.flat, tw.t_flat, False), (tw.packed, tw.t_pack, True)):
        gs.adamw_gs_step(groups, n, t, gs.StepConfig(schedule=gs.GS_SCHED_MASKED), visible=mask)
        gs.adamw_gs_step_view(groups, n, t, gs.StepConfig(), tw.means(packed), cam)
        b = gs.Batch([gs.Scene(groups=groups, n=n, step_count=t, visible=mask, schedule=gs.GS_SCHED_MASKED)])
        b.step(gs.StepConfig())
        b.close()
    torch.cuda.synchronize()
    lines = [ln for ln in capfd.readouterr().err.splitlines() if ln.startswith("gsopt:")]
    assert len(lines) == 6
    assert not any("packed64" in ln for ln in lines[:3]) and all(ln.endswith("packed=0") for ln in lines[2:3])
    assert lines[3].endswith("rows=packed64") and lines[4].endswith("rows=packed64") and lines[5].endswith("packed=1")
    tw.check_same("trace")
