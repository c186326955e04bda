"""The fused view step (visibility and step in one launch) against the
two-launch path it replaces and against the oracle, through the C ABI.

Rows are independent, so the fused kernel must reproduce gs_visibility
followed by the masked step bit for bit: attributes, moments, step counts
and the mask, with Re-State, AIU, position noise and the radius cull on or
off, in FP32 and BF16, for every wave unit and ragged sizes; with a batch
of cameras, the union of their views decides V."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

gs = pytest.importorskip("paper_2601_16736_amd")
from _gpu_util import DEV, compare, make_state, oracle_config, oracle_groups, set_grads  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)


def _bits(x):
    return x.view(torch.int16) if x.dtype == torch.bfloat16 else x


def _clone(st):
    return [gs.Group(g.param.clone(), g.grad.clone(), g.exp_avg.clone(), g.exp_avg_sq.clone(), g.lr,
                     dar_kind=g.dar_kind, dar_lambda=g.dar_lambda, dar_clip=g.dar_clip, reg_mode=g.reg_mode)
            for g in st.groups], st.t.clone()


def _scene(n, seed, bf16):
    st = make_state(gs, n, synth.GROUPS_59, seed, bf16=bf16)
    r = synth.rng(seed, 3)
    st.groups[0].param.copy_(torch.from_numpy(r.uniform(-10, 10, (n, 3)).astype(np.float32)))
    o = r.uniform(1e-4, 0.9, n)
    st.groups[3].param.copy_(torch.from_numpy(np.log(o / (1 - o)).astype(np.float32)[:, None]))
    gr = synth.grads(n, synth.GROUPS_59, np.ones(n, np.uint8), seed, 0)
    for (name, *_), g in zip(synth.GROUPS_59, st.groups):
        g.grad.copy_(torch.from_numpy(gr[name]))
    return st


CASES = [  # (n, unit, bf16, rsr, aiu, noise, radius)
    (1, 128, False, False, False, False, False),
    (31, 32, False, True, True, False, True),
    (20_011, 32, True, True, True, True, False),
    (100_003, 32, False, True, False, True, True),
    (63, 64, True, True, False, False, True),
    (1025, 128, False, True, True, False, False),
    (1025, 256, True, True, True, True, True),
    (20_011, 64, False, False, False, True, False),
    (20_011, 128, True, True, False, False, False),
    (20_011, 256, False, True, True, True, True),
    (100_003, 128, False, True, False, False, False),
    (20_011, 64, True, False, True, False, False),
    (20_011, 64, False, False, True, True, True),
]


@pytest.mark.parametrize("n,unit,bf16,rsr,aiu,noise,radius", CASES)
def test_view_step_equals_visibility_then_step(n, unit, bf16, rsr, aiu, noise, radius):
    st = _scene(n, 40 + n % 97, bf16)
    ref_groups, ref_t = _clone(st)
    rig = synth.camera_rig()
    c = rig[(n * 7) % 200]
    rad = torch.from_numpy((synth.rng(n, 9).random(n) * 0.5).astype(np.float32)).to(DEV) if radius else None
    cam = gs.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far,
                    0.5 if radius else 0.0)
    kw = dict(iteration=17, seed=n, moment_dtype=int(bf16), stochastic_round=bf16, rsr_enable=rsr, rsr_ratio=0.3,
              aiu_enable=aiu, aiu_ratio=0.4, aiu_scale=0.5, noise_enable=noise, noise_lr=0.02 / 1.6e-4,
              noise_t=0.5, unit=unit)
    print(f"view n={n} unit={unit} bf16={bf16} rsr={rsr} aiu={aiu} noise={noise} radius={radius}", flush=True)
    # reference: the two launches
    mask_ref = torch.zeros(n, dtype=torch.uint8, device=DEV)
    gs.gs_visibility(ref_groups[0].param, cam, mask=mask_ref, radius=rad)
    ref_kw = dict(kw, unit=128)          # any window gives the same bits: rows are independent
    gs.adamw_gs_step(ref_groups, n, ref_t, gs.StepConfig(schedule=gs.GS_SCHED_MASKED, **ref_kw), visible=mask_ref)
    # fused
    mask = torch.full((n,), 9, dtype=torch.uint8, device=DEV)
    gs.adamw_gs_step_view(st.groups, n, st.t, gs.StepConfig(**kw), st.groups[0].param, cam, radius=rad,
                          visible_out=mask)
    torch.cuda.synchronize()
    assert torch.equal(mask, mask_ref)
    assert torch.equal(st.t, ref_t)
    for a, b in zip(st.groups, ref_groups):
        assert torch.equal(a.param, b.param)
        assert torch.equal(_bits(a.exp_avg), _bits(b.exp_avg))
        assert torch.equal(_bits(a.exp_avg_sq), _bits(b.exp_avg_sq))


@pytest.mark.parametrize("views,unit,bf16,rsr", [(2, 128, False, True), (5, 64, True, False), (32, 256, False, True),
                                                 (3, 32, False, True)])
def test_view_step_camera_batch_equals_union_then_step(views, unit, bf16, rsr):
    """Several cameras: V is their union, as gs_visibility_multi's mask."""
    n = 40_009
    st = _scene(n, 90 + views, bf16)
    ref_groups, ref_t = _clone(st)
    rig = synth.camera_rig()
    cams = [gs.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far)
            for c in (rig[(11 * v + views) % 200] for v in range(views))]
    kw = dict(iteration=3, seed=views, moment_dtype=int(bf16), stochastic_round=bf16, rsr_enable=rsr, rsr_ratio=0.2,
              unit=unit)
    mask_ref = torch.zeros(n, dtype=torch.uint8, device=DEV)
    gs.gs_visibility_multi(ref_groups[0].param, cams, mask=mask_ref)
    gs.adamw_gs_step(ref_groups, n, ref_t, gs.StepConfig(schedule=gs.GS_SCHED_MASKED, **dict(kw, unit=max(unit, 128))),
                     visible=mask_ref)
    mask = torch.zeros(n, dtype=torch.uint8, device=DEV)
    gs.adamw_gs_step_view(st.groups, n, st.t, gs.StepConfig(**kw), st.groups[0].param, cams, visible_out=mask)
    torch.cuda.synchronize()
    assert torch.equal(mask, mask_ref)
    assert mask.float().mean().item() > 0.3          # the union of several views
    assert torch.equal(st.t, ref_t)
    for a, b in zip(st.groups, ref_groups):
        assert torch.equal(a.param, b.param)
        assert torch.equal(_bits(a.exp_avg), _bits(b.exp_avg))
        assert torch.equal(_bits(a.exp_avg_sq), _bits(b.exp_avg_sq))


def test_view_step_against_oracle():
    """Mask from the oracle's FP32 predicate, then the oracle step."""
    n, spec = 30_000, synth.GROUPS_59
    st = _scene(n, 77, False)
    c = synth.camera_rig()[123]
    cam = gs.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far)
    cfg = gs.StepConfig(iteration=5, seed=3, rsr_enable=True, rsr_ratio=0.2, reg_norm=1e5)
    torch.cuda.synchronize()
    before = st.host()
    mask = torch.zeros(n, dtype=torch.uint8, device=DEV)
    gs.adamw_gs_step_view(st.groups, n, st.t, cfg, st.groups[0].param, cam, visible_out=mask)
    torch.cuda.synchronize()
    ocam = oracle.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far)
    m_ref = oracle.visibility(before["means"]["param"].astype(np.float32), ocam)
    np.testing.assert_array_equal(mask.cpu().numpy(), m_ref)
    og = oracle_groups(before, spec, st.groups)
    t_ref = before["_t"].copy()
    oracle.adamw_gs_step(og, n, m_ref, t_ref, oracle_config(cfg))
    touched = m_ref.astype(bool) | oracle.rsr_sample_mask(cfg.seed, cfg.iteration, n, cfg.rsr_ratio)
    compare(st.host(), before, og, spec, t_ref, touched, False, "view step")


@pytest.mark.parametrize("rsr", [False, True])
@pytest.mark.parametrize("bf16", [False, True])
def test_view_step_full_size_equals_two_launches(bf16, rsr):
    """The benchmark's 3M Morton scene, one step with Re-State, FP32 moments
    or BF16 with stochastic rounding: both paths bit for bit; the mask equals
    the oracle's FP32 predicate over all 3M; sampled visible, invisible and
    Re-State-sampled rows of the fused step match the oracle one by one."""
    import bench
    scene = synth.scene_uniform(bench.N_PRIMS, seed=0)
    sd = bench.SceneOnDevice(gs, torch, scene, "morton")
    n = bench.N_PRIMS
    spec = synth.GROUPS_59
    cams = synth.camera_rig()
    c = cams[11]
    cam = gs.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far)
    mdt = torch.bfloat16 if bf16 else torch.float32
    outs = []
    for fused in (False, True):
        groups = [gs.Group(p.clone(), sets[1], torch.zeros(p.shape, dtype=mdt, device=DEV),
                           torch.zeros(p.shape, dtype=mdt, device=DEV), lr, dar_kind=dar,
                           dar_lambda=1e-3 if dar == 1 else (1e-5 if dar == 2 else 0.0), dar_clip=10.0)
                  for (name, dim, lr, dar), p, sets in zip(spec, sd.params, sd.grads)]
        t = torch.zeros(n, dtype=torch.int32, device=DEV)
        mask = torch.zeros(n, dtype=torch.uint8, device=DEV)
        # the benchmark's windows: 32 on plain steps, 64 on Re-State iterations
        cfg = gs.StepConfig(reg_norm=1e5, iteration=100, rsr_enable=rsr, rsr_ratio=0.05, unit=bench.VIEW_UNIT,
                            moment_dtype=int(bf16), stochastic_round=bf16)
        if fused:
            gs.adamw_gs_step_view(groups, n, t, cfg, groups[0].param, cam, visible_out=mask)
        else:
            gs.gs_visibility(groups[0].param, cam, mask=mask)
            cfg.schedule, cfg.unit = gs.GS_SCHED_MASKED, 128       # any window gives the same bits
            gs.adamw_gs_step(groups, n, t, cfg, visible=mask)
        torch.cuda.synchronize()
        outs.append((groups, t, mask, cfg))
    (ga, ta, ma, _), (gb, tb, mb, cfg) = outs
    assert torch.equal(ma, mb) and torch.equal(ta, tb)
    assert 0.2 < ma.float().mean().item() < 0.4
    for a, b in zip(ga, gb):
        assert torch.equal(a.param, b.param)
        assert torch.equal(a.exp_avg.view(torch.int16) if bf16 else a.exp_avg,
                           b.exp_avg.view(torch.int16) if bf16 else b.exp_avg)
        assert torch.equal(a.exp_avg_sq.view(torch.int16) if bf16 else a.exp_avg_sq,
                           b.exp_avg_sq.view(torch.int16) if bf16 else b.exp_avg_sq)

    ref_mask = oracle.visibility(sd.params[0].cpu().numpy(), oracle.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width,
                                                                          c.height, c.z_near, c.z_far))
    np.testing.assert_array_equal(mb.cpu().numpy(), ref_mask)
    sampled = oracle.rsr_sample_mask(cfg.seed, cfg.iteration, n, cfg.rsr_ratio)
    r = synth.rng(41)
    rows = np.unique(np.concatenate([r.choice(np.flatnonzero(ref_mask), 2000, replace=False),
                                     r.choice(np.flatnonzero(ref_mask == 0), 2000, replace=False),
                                     r.choice(np.flatnonzero(sampled), 1000, replace=False)])).astype(np.int64)
    rows_t = torch.from_numpy(rows).to(DEV)
    before, after = {}, {}
    for (name, dim, *_), p, sets, g in zip(spec, sd.params, sd.grads, gb):
        zero = np.zeros((len(rows), dim))
        before[name] = {"param": p[rows_t].cpu().numpy(), "grad": sets[1][rows_t].cpu().numpy(), "m": zero,
                        "v": zero.copy()}
        after[name] = {"param": g.param[rows_t].cpu().numpy(), "grad": before[name]["grad"],
                       "m": g.exp_avg[rows_t].float().cpu().numpy().astype(np.float64),
                       "v": g.exp_avg_sq[rows_t].float().cpu().numpy().astype(np.float64)}
    before["_t"] = np.zeros(len(rows), np.int32)
    after["_t"] = tb[rows_t].cpu().numpy()
    og = oracle_groups(before, spec, gb)
    t_ref = before["_t"].copy()
    oracle.adamw_gs_step(og, len(rows), ref_mask[rows].copy(), t_ref, oracle_config(cfg), ids=rows)
    touched = ref_mask[rows].astype(bool) | (sampled[rows] if rsr else False)
    compare(after, before, og, spec, t_ref, touched, bf16, "3M fused step")


def test_view_step_rejects_bad_unit_and_camera():
    n = 100
    st = _scene(n, 5, False)
    c = synth.camera_rig()[0]
    cam = gs.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far)
    with pytest.raises(gs.GsError):
        gs.adamw_gs_step_view(st.groups, n, st.t, gs.StepConfig(unit=512), st.groups[0].param, cam)
    with pytest.raises(gs.GsError):
        gs.adamw_gs_step_view(st.groups, n, st.t, gs.StepConfig(unit=16), st.groups[0].param, cam)
    bad = gs.Camera(c.view, c.fx, c.fy, c.cx, c.cy, 0, c.height, c.z_near, c.z_far)
    with pytest.raises(gs.GsError):
        gs.adamw_gs_step_view(st.groups, n, st.t, gs.StepConfig(), st.groups[0].param, bad)
    with pytest.raises(gs.GsError):
        gs.adamw_gs_step_view(st.groups, n, st.t, gs.StepConfig(), st.groups[0].param, [cam, bad])
    with pytest.raises(gs.GsError):
        gs.adamw_gs_step_view(st.groups, n, st.t, gs.StepConfig(), st.groups[0].param, [cam] * 33)
    with pytest.raises(gs.GsError):
        gs.adamw_gs_step_view(st.groups, n, st.t, gs.StepConfig(), st.groups[0].param, [])


@pytest.mark.parametrize("n,unit,bf16,noise", [(20_011, 0, False, False), (20_011, 0, True, False),
                                               (100_003, 0, False, True), (1025, 32, True, True), (1, 0, False, False)])
def test_view_step_aiu_with_and_without_mask_out(n, unit, bf16, noise):
    """AIU without Re-State at the default windows, with and without
    visible_out: both equal the two-launch path bit for bit, over three
    steps (AIU rows need t > 0, so later steps sample more of them)."""
    st = _scene(n, 60 + n % 89, bf16)
    a_groups, a_t = _clone(st)
    ref_groups, ref_t = _clone(st)
    rig = synth.camera_rig()
    for it in range(3):
        c = rig[(n * 3 + 41 * it) % 200]
        cam = gs.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far)
        kw = dict(iteration=20 + it, seed=n, moment_dtype=int(bf16), stochastic_round=bf16, aiu_enable=True,
                  aiu_ratio=0.3, aiu_scale=0.7, noise_enable=noise, noise_lr=0.02 / 1.6e-4, noise_t=0.5, unit=unit)
        print(f"view aiu n={n} unit={unit} bf16={bf16} noise={noise} step={it}", flush=True)
        mask_ref = torch.zeros(n, dtype=torch.uint8, device=DEV)
        gs.gs_visibility(ref_groups[0].param, cam, mask=mask_ref)
        gs.adamw_gs_step(ref_groups, n, ref_t, gs.StepConfig(schedule=gs.GS_SCHED_MASKED, **dict(kw, unit=128)),
                         visible=mask_ref)
        mask = torch.full((n,), 9, dtype=torch.uint8, device=DEV)
        gs.adamw_gs_step_view(st.groups, n, st.t, gs.StepConfig(**kw), st.groups[0].param, cam, visible_out=mask)
        gs.adamw_gs_step_view(a_groups, n, a_t, gs.StepConfig(**kw), a_groups[0].param, cam)
        torch.cuda.synchronize()
        assert torch.equal(mask, mask_ref)
        for t in (st.t, a_t):
            assert torch.equal(t, ref_t)
        for x, y, r in zip(st.groups, a_groups, ref_groups):
            for field in ("param", "exp_avg", "exp_avg_sq"):
                assert torch.equal(_bits(getattr(x, field)), _bits(getattr(r, field)))
                assert torch.equal(_bits(getattr(y, field)), _bits(getattr(r, field)))
    assert int((ref_t > 0).sum()) > 0 or n == 1
