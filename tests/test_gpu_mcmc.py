"""The MCMC-shaped workload at full size, in the benchmark's launch
configuration: 6M primitives with means from a 64-cluster mixture put in
Morton order, opacity and scale regularisation 0.01, one fused view step
(windows of 32, Re-State on) followed by the relocation reset of the 1 %
lowest opacity logits.  Checked: the mask against the oracle's FP32
predicate over all 6M; the step counts over all 6M; the selected list
against a stable sort of the post-step logits; and sampled visible,
invisible, Re-State-sampled and relocated rows one by one against the
oracle's step followed by the reset."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

gs = pytest.importorskip("paper_2601_16736_amd")
from _gpu_util import DEV, compare, oracle_config, oracle_groups, rsr_sampled_mask  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)


def _take(groups, t, rows_t, spec):
    out = {}
    for (name, *_), g in zip(spec, groups):
        out[name] = {"param": g.param[rows_t].cpu().numpy(), "grad": g.grad[rows_t].cpu().numpy(),
                     "m": g.exp_avg[rows_t].cpu().numpy().astype(np.float64),
                     "v": g.exp_avg_sq[rows_t].cpu().numpy().astype(np.float64)}
    out["_t"] = t[rows_t].cpu().numpy()
    return out


def test_mcmc_shape_full_size_view_step_and_relocation():
    import bench
    n, k_reloc = 6_000_000, 60_000
    spec = synth.GROUPS_59
    means = synth.scene_clustered(n, seed=0, groups=[("means", 3, 0.0, 0)]).params["means"]
    gen = torch.Generator(device=DEV)
    gen.manual_seed(31)
    params = [torch.from_numpy(means).to(DEV)] + [torch.randn((n, d), generator=gen, device=DEV)
                                                  for _, d, _, _ in spec[1:]]
    perm = torch.empty(n, dtype=torch.int32, device=DEV)
    ws = torch.empty(gs.gs_spatial_order_workspace_size(n), dtype=torch.uint8, device=DEV)
    gs.gs_spatial_order(params[0], perm, ws)
    params = gs.apply_spatial_order(params, perm)
    del ws, perm
    groups = []
    for (name, d, lr, dar), p in zip(spec, params):
        g = torch.randn((n, d), generator=gen, device=DEV) * 1e-3
        m = torch.randn((n, d), generator=gen, device=DEV) * 1e-4
        v = torch.rand((n, d), generator=gen, device=DEV) * 1e-6 + 1e-9
        groups.append(gs.Group(p, g, m, v, lr, dar_kind=dar, dar_lambda=0.01 if dar else 0.0, dar_clip=10.0))
    t = torch.randint(0, 40, (n,), generator=gen, device=DEV, dtype=torch.int32)
    cam = synth.camera_rig()[91]
    gcam = gs.Camera(cam.view, cam.fx, cam.fy, cam.cx, cam.cy, cam.width, cam.height, cam.z_near, cam.z_far)
    ocam = oracle.Camera(cam.view, cam.fx, cam.fy, cam.cx, cam.cy, cam.width, cam.height, cam.z_near, cam.z_far)
    cfg = gs.StepConfig(reg_norm=bench.REG_NORM, seed=0, iteration=200, rsr_enable=True, rsr_ratio=bench.RSR_P,
                        rsr_alpha1=bench.RSR_A1, rsr_alpha2=bench.RSR_A2, unit=bench.VIEW_UNIT)

    means_h = groups[0].param.cpu().numpy()
    ref_mask = oracle.visibility(means_h, ocam)
    frac = ref_mask.mean()
    assert 0.05 < frac < 0.6, frac
    sampled = rsr_sampled_mask(n, cfg.seed, cfg.iteration, cfg.rsr_ratio)
    r = synth.rng(32)
    rows = np.unique(np.concatenate([r.choice(np.flatnonzero(ref_mask), 2000, replace=False),
                                     r.choice(np.flatnonzero(ref_mask == 0), 2000, replace=False),
                                     r.choice(np.flatnonzero(sampled), 1000, replace=False)])).astype(np.int64)
    rows_t = torch.from_numpy(rows).to(DEV)
    before = _take(groups, t, rows_t, spec)
    t_before = t.clone()

    mask = torch.zeros(n, dtype=torch.uint8, device=DEV)
    print(f"mcmc full size: n={n} visible {frac:.3f}", flush=True)
    gs.adamw_gs_step_view(groups, n, t, cfg, groups[0].param, gcam, visible_out=mask)
    opacity_after = groups[3].param[:, 0].clone()
    sel = torch.empty(k_reloc, dtype=torch.int32, device=DEV)
    rws = torch.empty(gs.gs_relocate_workspace_size(n), dtype=torch.uint8, device=DEV)
    gs.gs_relocate_reset(groups[3].param, k_reloc, groups, gs.GS_MOMENT_F32, t, True, rws, selected=sel)
    torch.cuda.synchronize()

    np.testing.assert_array_equal(mask.cpu().numpy(), ref_mask)
    key = opacity_after.cpu().numpy()
    ref_sel = np.sort(np.argsort(key, kind="stable")[:k_reloc])
    np.testing.assert_array_equal(sel.cpu().numpy().astype(np.int64), ref_sel)
    relocated = np.zeros(n, bool)
    relocated[ref_sel] = True
    dt = (t - t_before).cpu().numpy()
    expect_t = np.where(relocated, -t_before.cpu().numpy(), ref_mask.astype(np.int32))
    np.testing.assert_array_equal(dt, expect_t)

    # the oracle's step on the sampled rows, then the reset of the relocated ones
    og = oracle_groups(before, spec, groups)
    t_ref = before["_t"].copy()
    oracle.adamw_gs_step(og, len(rows), ref_mask[rows].copy(), t_ref, oracle_config(cfg, cfg.reg_norm), ids=rows)
    hit = relocated[rows]
    for O in og:
        O.m[hit] = 0.0
        O.v[hit] = 0.0
    t_ref[hit] = 0
    after = _take(groups, t, rows_t, spec)
    touched = ref_mask[rows].astype(bool) | sampled[rows] | hit
    compare(after, before, og, spec, t_ref, touched, False, "6M MCMC-shaped")
    assert hit.any() or not relocated.any()
