"""Batched plan: one persistent launch over many scenes must give, bit for bit,
what per-scene adamw_gs_step calls with seed + s give, on every graph
replay (eager work and synchronisations in between), for mixed schedules,
sizes, visibility ratios, RSR iterations and both moment precisions; and one
scene is checked against the oracle directly."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

gs = pytest.importorskip("paper_2601_16736_amd")
from _gpu_util import DEV, compare, make_state, oracle_config, oracle_groups, rsr_sampled_mask  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)


def _clone_state(st):
    groups = [gs.Group(g.param.clone(), g.grad.clone(), g.exp_avg.clone(), g.exp_avg_sq.clone(), g.lr,
                       dar_kind=g.dar_kind, dar_lambda=g.dar_lambda, dar_clip=g.dar_clip, reg_mode=g.reg_mode)
              for g in st.groups]
    return groups, st.t.clone()


SCENES = [  # (n, visible ratio, schedule, layout)
    (30_001, 0.02, gs.GS_SCHED_COMPACTED, synth.GROUPS_59),
    (257, 0.6, gs.GS_SCHED_MASKED, synth.GROUPS_59),
    (75_000, 0.3, gs.GS_SCHED_COMPACTED, synth.GROUPS_60_SPLIT),
    (4096, 1.0, gs.GS_SCHED_DENSE, synth.GROUPS_59),
    (1, 1.0, gs.GS_SCHED_MASKED, synth.GROUPS_59),
    (12_345, 0.45, gs.GS_SCHED_AUTO, synth.GROUPS_60_SPLIT),
]


def _noise_kw(on):
    # position noise on the mean group; both layouts start means, scales, quats, opacity
    return dict(noise_enable=on, noise_groups=(0, 1, 2, 3), noise_lr=0.05 / synth.GROUPS_59[0][2], noise_k=100.0,
                noise_t=0.5)     # opacities of these states spread around 0.5


@pytest.mark.parametrize("bf16,noise,resident", [(False, False, False), (True, False, False), (True, True, False),
                                                  (True, False, True), (False, True, True)])
def test_batched_equals_per_scene_calls(bf16, noise, resident):
    """noise=True switches position noise on every other replay, so one plan
    runs both of its kernel variants."""
    rng = np.random.default_rng(3)
    plans, refs = [], []
    for s, (n, p, sched, spec) in enumerate(SCENES):
        st = make_state(gs, n, spec, 100 + s, bf16=bf16)
        for g in st.groups:
            g.grad.copy_(torch.from_numpy((1e-3 * rng.standard_normal(tuple(g.grad.shape))).astype(np.float32)))
        mask = torch.zeros(n, dtype=torch.uint8, device=DEV)
        idx = torch.zeros(n, dtype=torch.int32, device=DEV)
        cnt = torch.zeros(1, dtype=torch.int32, device=DEV)
        plans.append(dict(st=st, mask=mask, idx=idx, cnt=cnt, n=n, p=p, sched=sched, spec=spec))
        rg, rt = _clone_state(st)
        refs.append(dict(groups=rg, t=rt))
    scenes = [gs.Scene(groups=d["st"].groups, n=d["n"], step_count=d["st"].t, visible=d["mask"],
                       vis_idx=d["idx"], vis_count=d["cnt"], schedule=d["sched"], visible_hint=d["p"])
              for d in plans]
    batch = gs.Batch(scenes, moment_dtype=int(bf16))
    batch.set_resident(resident)
    for s, d in enumerate(plans):
        assert batch.schedule(s) in (gs.GS_SCHED_COMPACTED, gs.GS_SCHED_MASKED, gs.GS_SCHED_DENSE)
    for it in range(5):                       # five replays of the plan's graph
        for s, d in enumerate(plans):         # eager work between replays: new masks + compaction
            m = synth.bernoulli_mask(d["n"], d["p"], s, it)
            d["mask"].copy_(torch.from_numpy(m))
            gs.gs_compact(d["mask"], d["idx"], d["cnt"])
        nz = _noise_kw(noise and it % 2 == 0)
        nz.update(aiu_enable=(it % 3 == 2), aiu_ratio=0.3, aiu_scale=0.5)     # AIU on replays 2 (and 5)
        cfg = gs.StepConfig(iteration=it, seed=77, rsr_enable=(it % 2 == 1), rsr_ratio=0.25,
                            moment_dtype=int(bf16), stochastic_round=True, **nz)
        batch.step(cfg)
        torch.cuda.synchronize()
        for s, (d, r) in enumerate(zip(plans, refs)):
            sched = batch.schedule(s)
            c1 = gs.StepConfig(iteration=it, seed=77 + s, rsr_enable=(it % 2 == 1), rsr_ratio=0.25,
                               moment_dtype=int(bf16), stochastic_round=True, schedule=sched, **nz)
            gs.adamw_gs_step(r["groups"], d["n"], r["t"], c1, visible=d["mask"], vis_idx=d["idx"],
                             vis_count=d["cnt"])
        torch.cuda.synchronize()
        for s, (d, r) in enumerate(zip(plans, refs)):
            assert torch.equal(d["st"].t, r["t"]), f"replay {it} scene {s}: step counts"
            for a, b in zip(d["st"].groups, r["groups"]):
                assert torch.equal(a.param, b.param), f"replay {it} scene {s}: theta"
                assert torch.equal(a.exp_avg.view(torch.int16) if bf16 else a.exp_avg,
                                   b.exp_avg.view(torch.int16) if bf16 else b.exp_avg), f"replay {it} scene {s}: m"
                assert torch.equal(a.exp_avg_sq.view(torch.int16) if bf16 else a.exp_avg_sq,
                                   b.exp_avg_sq.view(torch.int16) if bf16 else b.exp_avg_sq)
    batch.close()


def test_batched_scene_against_oracle():
    """Scene 1 of a 3-scene plan (seed offset 1) against the oracle."""
    spec = synth.GROUPS_59
    sts, masks = [], []
    for s, n in enumerate((5000, 20_000, 999)):
        st = make_state(gs, n, spec, 200 + s)
        m = synth.bernoulli_mask(n, 0.3, 9, s)
        gr = synth.grads(n, spec, m, 9, s)
        for (name, *_), g in zip(spec, st.groups):
            g.grad.copy_(torch.from_numpy(gr[name]))
        sts.append(st)
        masks.append(m)
    d_masks = [torch.from_numpy(m).to(DEV) for m in masks]
    scenes = [gs.Scene(groups=st.groups, n=st.t.shape[0], step_count=st.t, visible=dm,
                       schedule=gs.GS_SCHED_MASKED) for st, dm in zip(sts, d_masks)]
    batch = gs.Batch(scenes)
    before = sts[1].host()
    cfg = gs.StepConfig(iteration=100, seed=5, rsr_enable=True, rsr_ratio=0.05)
    batch.step(cfg)
    torch.cuda.synchronize()
    og = oracle_groups(before, spec, sts[1].groups)
    t_ref = before["_t"].copy()
    ocfg = oracle_config(cfg)
    ocfg.seed = 6                               # scene 1 draws with seed + 1
    oracle.adamw_gs_step(og, 20_000, masks[1], t_ref, ocfg)
    touched = masks[1].astype(bool) | rsr_sampled_mask(20_000, 6, 100, 0.05)
    compare(sts[1].host(), before, og, spec, t_ref, touched, False, "batched scene 1")
    batch.close()


def test_batch_rejects_bad_plans():
    st = make_state(gs, 10, synth.GROUPS_59, 1)
    sc = gs.Scene(groups=st.groups, n=10, step_count=st.t, schedule=gs.GS_SCHED_COMPACTED)   # no index list
    with pytest.raises(gs.GsError):
        gs.Batch([sc])
    with pytest.raises(gs.GsError):
        gs.Batch([gs.Scene(groups=st.groups, n=10, step_count=st.t)] * 65)
    b = gs.Batch([gs.Scene(groups=st.groups, n=10, step_count=st.t, schedule=gs.GS_SCHED_DENSE)])
    with pytest.raises(gs.GsError):
        b.step(gs.StepConfig(moment_dtype=gs.GS_MOMENT_BF16))
    b.close()


def test_batched_full_size_16_scenes():
    """The benchmark's many-scene workload at full size: 16 scenes with sizes
    log-uniform in [2e5, 4e6] (16.3M primitives in all) and Bernoulli
    visibility U[0.02, 0.60], schedules from the tuner, BF16 moments with
    stochastic rounding, RSR on.  One plan step equals the 16 per-scene calls
    bit for bit over every primitive, and sampled visible, invisible and
    RSR-sampled rows of three scenes match the oracle one by one."""
    spec = synth.GROUPS_59
    dims = [d for _, d, _, _ in spec]
    sizes, ratios = synth.batch_scene_sizes(16, seed=0)
    gen = torch.Generator(device=DEV)
    gen.manual_seed(21)
    bf = torch.bfloat16

    def rand_state(n):
        groups = []
        for name, d, lr, dar in spec:
            p = torch.randn((n, d), generator=gen, device=DEV)
            g = torch.randn((n, d), generator=gen, device=DEV) * 1e-3
            m = (torch.randn((n, d), generator=gen, device=DEV) * 1e-4).to(bf)
            v = (torch.rand((n, d), generator=gen, device=DEV) * 1e-6 + 1e-9).to(bf)
            groups.append(gs.Group(p, g, m, v, lr, dar_kind=dar, dar_lambda=1e-3 if dar == 1 else (1e-5 if dar else 0.0),
                                   dar_clip=10.0))
        t = torch.randint(0, 40, (n,), generator=gen, device=DEV, dtype=torch.int32)
        return groups, t

    scenes, refs, masks, scheds = [], [], [], []
    for s, (n, p) in enumerate(zip(sizes.tolist(), ratios.tolist())):
        sched, _ = gs.gs_tune(n, dims, float(p), gs.GS_MOMENT_BF16)
        groups, t = rand_state(n)
        mask = (torch.rand(n, generator=gen, device=DEV) < p).to(torch.uint8)
        idx = torch.zeros(n, dtype=torch.int32, device=DEV)
        cnt = torch.zeros(1, dtype=torch.int32, device=DEV)
        if sched == gs.GS_SCHED_COMPACTED:
            gs.gs_compact(mask, idx, cnt)
        ref_groups = [gs.Group(g.param.clone(), g.grad, g.exp_avg.clone(), g.exp_avg_sq.clone(), g.lr,
                               dar_kind=g.dar_kind, dar_lambda=g.dar_lambda, dar_clip=g.dar_clip) for g in groups]
        scenes.append(gs.Scene(groups=groups, n=n, step_count=t, visible=mask, vis_idx=idx, vis_count=cnt,
                               schedule=sched, visible_hint=float(p)))
        refs.append((ref_groups, t.clone()))
        masks.append(mask)
        scheds.append(sched)
    print(f"batched full size: {int(sizes.sum())} primitives, schedules {scheds}", flush=True)
    cfg = gs.StepConfig(iteration=300, seed=0, rsr_enable=True, rsr_ratio=0.05, moment_dtype=gs.GS_MOMENT_BF16,
                        stochastic_round=True)

    # sampled rows of three scenes, taken before the step
    check = [int(np.argmin(sizes)), int(np.argmax(sizes)), 7]
    r = synth.rng(22)
    picked, before = {}, {}
    for s in check:
        n = int(sizes[s])
        m = masks[s].cpu().numpy()
        smp = rsr_sampled_mask(n, cfg.seed + s, cfg.iteration, cfg.rsr_ratio)
        rows = np.unique(np.concatenate([
            r.choice(np.flatnonzero(m), min(1500, int(m.sum())), replace=False),
            r.choice(np.flatnonzero(m == 0), 1500, replace=False),
            r.choice(np.flatnonzero(smp), 800, replace=False)])).astype(np.int64)
        picked[s] = (rows, m[rows].copy(), smp[rows])
        before[s] = _take(scenes[s].groups, scenes[s].step_count, rows, spec)

    batch = gs.Batch(scenes, moment_dtype=gs.GS_MOMENT_BF16)
    batch.step(cfg)
    for s, (sc, (rg, rt)) in enumerate(zip(scenes, refs)):
        gs.adamw_gs_step(rg, sc.n, rt, gs.StepConfig(**dict(vars(cfg), seed=cfg.seed + s, schedule=sc.schedule)),
                         visible=sc.visible, vis_idx=sc.vis_idx, vis_count=sc.vis_count)
    torch.cuda.synchronize()
    for s, (sc, (rg, rt)) in enumerate(zip(scenes, refs)):
        assert torch.equal(sc.step_count, rt), f"scene {s}: t"
        for a, b in zip(sc.groups, rg):
            assert torch.equal(a.param, b.param), f"scene {s}: theta"
            assert torch.equal(a.exp_avg.view(torch.int16), b.exp_avg.view(torch.int16)), f"scene {s}: m"
            assert torch.equal(a.exp_avg_sq.view(torch.int16), b.exp_avg_sq.view(torch.int16)), f"scene {s}: v"
    for s in check:
        rows, m_rows, smp_rows = picked[s]
        b = before[s]
        og = oracle_groups(b, spec, scenes[s].groups)
        t_ref = b["_t"].copy()
        ocfg = oracle_config(cfg)
        ocfg.seed = cfg.seed + s
        oracle.adamw_gs_step(og, len(rows), m_rows, t_ref, ocfg, ids=rows)
        after = _take(scenes[s].groups, scenes[s].step_count, rows, spec)
        compare(after, b, og, spec, t_ref, m_rows.astype(bool) | smp_rows, True, f"full-size scene {s}")
    batch.close()


def _take(groups, t, rows, spec):
    rows_t = torch.from_numpy(rows).to(DEV)
    out = {}
    for (name, *_), g in zip(spec, groups):
        out[name] = {"param": g.param[rows_t].cpu().numpy(), "grad": g.grad[rows_t].cpu().numpy(),
                     "m": g.exp_avg[rows_t].float().cpu().numpy().astype(np.float64),
                     "v": g.exp_avg_sq[rows_t].float().cpu().numpy().astype(np.float64)}
    out["_t"] = t[rows_t].cpu().numpy()
    return out
