"""The largest scene the ABI accepts: n = 2^31 - 1 primitives.  Row
indices near 2^31 exercise every index computation at its limit.

A 1-wide group through the masked and the compacted schedules (with
Re-State): both give the same bits; step counts are exact over all n; the
last rows and a random sample match the oracle.  Then the fused view step
on a 3-wide mean group: the mask of sampled rows (the last ones included)
equals the oracle's FP32 predicate, and those rows match the oracle's step.
About 110 GB of device memory at the peak."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

gs = pytest.importorskip("paper_2601_16736_amd")
from _gpu_util import DEV, compare, oracle_config, oracle_groups  # noqa: E402

N_MAX = (1 << 31) - 1


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    free, _ = torch.cuda.mem_get_info()
    if free < 140 << 30:
        pytest.skip("needs about 140 GB of free device memory")
    oracle.build(force=False)
    yield
    # the tests after this module run in the same process
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _sample_rows(n, seed):
    """The last 300 rows and 3000 random ones."""
    r = synth.rng(seed)
    return np.unique(np.concatenate([np.arange(n - 300, n, dtype=np.int64), r.integers(0, n, 3000, dtype=np.int64)]))


def _take(groups, t, rows_t, spec):
    out = {}
    for (name, *_), g in zip(spec, groups):
        out[name] = {"param": g.param[rows_t].cpu().numpy(), "grad": g.grad[rows_t].cpu().numpy(),
                     "m": g.exp_avg[rows_t].cpu().numpy().astype(np.float64),
                     "v": g.exp_avg_sq[rows_t].cpu().numpy().astype(np.float64)}
    out["_t"] = t[rows_t].cpu().numpy()
    return out


def test_max_size_masked_and_compacted_schedules():
    n = N_MAX
    spec = [("opacity", 1, 5e-2, 1)]
    gen = torch.Generator(device=DEV)
    gen.manual_seed(81)
    p = torch.randn((n, 1), generator=gen, device=DEV)
    g = torch.randn((n, 1), generator=gen, device=DEV) * 1e-3
    m = torch.randn((n, 1), generator=gen, device=DEV) * 1e-4
    v = torch.rand((n, 1), generator=gen, device=DEV) * 1e-6 + 1e-9
    t = torch.randint(0, 30, (n,), generator=gen, device=DEV, dtype=torch.int32)
    mask = (torch.rand(n, generator=gen, device=DEV) < 0.3).to(torch.uint8)
    mask[-5:] = torch.tensor([1, 0, 1, 1, 0], dtype=torch.uint8, device=DEV)
    cfg = gs.StepConfig(iteration=100, seed=2, rsr_enable=True, rsr_ratio=0.05, schedule=gs.GS_SCHED_MASKED,
                        unit=32)
    rows = _sample_rows(n, 82)
    rows_t = torch.from_numpy(rows).to(DEV)
    A = [gs.Group(p, g, m, v, 5e-2, dar_kind=1, dar_lambda=1e-3, dar_clip=10.0)]
    before = _take(A, t, rows_t, spec)
    t0 = t.clone()
    # the compacted run starts from copies of the same state
    B = [gs.Group(p.clone(), g, m.clone(), v.clone(), 5e-2, dar_kind=1, dar_lambda=1e-3, dar_clip=10.0)]
    tb = t.clone()
    print(f"max size: n={n} masked step", flush=True)
    gs.adamw_gs_step(A, n, t, cfg, visible=mask)
    torch.cuda.synchronize()
    assert torch.equal(t - t0, mask.to(torch.int32))
    del t0
    torch.cuda.empty_cache()

    m_rows = mask[rows_t].cpu().numpy()
    og = oracle_groups(before, spec, A)
    t_ref = before["_t"].copy()
    oracle.adamw_gs_step(og, len(rows), m_rows.copy(), t_ref, oracle_config(cfg), ids=rows)
    touched = m_rows.astype(bool) | oracle.rsr_sample_mask(cfg.seed, cfg.iteration, n, cfg.rsr_ratio,
                                                           ids=rows).astype(bool)
    compare(_take(A, t, rows_t, spec), before, og, spec, t_ref, touched, False, "max-size masked")

    idx = torch.empty(n, dtype=torch.int32, device=DEV)
    cnt = torch.zeros(1, dtype=torch.int32, device=DEV)
    gs.gs_compact(mask, idx, cnt)
    cfg.schedule, cfg.unit = gs.GS_SCHED_COMPACTED, 64
    print(f"max size: n={n} compacted step", flush=True)
    gs.adamw_gs_step(B, n, tb, cfg, visible=mask, vis_idx=idx, vis_count=cnt)
    torch.cuda.synchronize()
    assert int(cnt.item()) == int(mask.sum(dtype=torch.int64).item())
    assert torch.equal(tb, t)
    assert torch.equal(B[0].param, A[0].param)
    assert torch.equal(B[0].exp_avg, A[0].exp_avg)
    assert torch.equal(B[0].exp_avg_sq, A[0].exp_avg_sq)


def test_max_size_fused_view_step():
    n = N_MAX
    spec = [("means", 3, 1.6e-4, 0)]
    gen = torch.Generator(device=DEV)
    gen.manual_seed(83)
    p = (torch.rand((n, 3), generator=gen, device=DEV) * 20.0 - 10.0)
    g = torch.randn((n, 3), generator=gen, device=DEV) * 1e-3
    m = torch.zeros((n, 3), device=DEV)
    v = torch.zeros((n, 3), device=DEV)
    t = torch.zeros(n, dtype=torch.int32, device=DEV)
    c = synth.camera_rig()[17]
    cam = gs.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far)
    ocam = oracle.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far)
    rows = _sample_rows(n, 84)
    rows_t = torch.from_numpy(rows).to(DEV)
    G = [gs.Group(p, g, m, v, 1.6e-4)]
    before = _take(G, t, rows_t, spec)
    ref_mask = oracle.visibility(before["means"]["param"], ocam)
    assert 0 < ref_mask.sum() < len(rows)
    cfg = gs.StepConfig(iteration=7, seed=4, rsr_enable=True, rsr_ratio=0.05, unit=32)
    print(f"max size: n={n} fused view step", flush=True)
    gs.adamw_gs_step_view(G, n, t, cfg, p, cam)
    torch.cuda.synchronize()
    after = _take(G, t, rows_t, spec)
    np.testing.assert_array_equal(after["_t"], ref_mask.astype(np.int32))
    og = oracle_groups(before, spec, G)
    t_ref = before["_t"].copy()
    oracle.adamw_gs_step(og, len(rows), ref_mask.copy(), t_ref, oracle_config(cfg), ids=rows)
    touched = ref_mask.astype(bool) | oracle.rsr_sample_mask(cfg.seed, cfg.iteration, n, cfg.rsr_ratio,
                                                             ids=rows).astype(bool)
    compare(after, before, og, spec, t_ref, touched, False, "max-size view")


def test_max_size_append():
    """gs_append up to n + k = 2^31 - 1 rows.  One wave per unit would need
    more work-items than a dispatch holds, so the grid is capped and its
    waves stride over the remaining units.  Every new row is a clone of its
    source with zero state; the old rows are untouched."""
    n = 100
    k = N_MAX - n
    gen = torch.Generator(device=DEV)
    gen.manual_seed(91)
    p = torch.zeros((n + k, 1), device=DEV)
    p[:n, 0] = torch.arange(1, n + 1, dtype=torch.float32, device=DEV)     # source s holds s + 1
    m = torch.full((n + k, 1), 7.0, device=DEV)
    v = torch.full((n + k, 1), 7.0, device=DEV)
    t = torch.full((n + k,), 5, dtype=torch.int32, device=DEV)
    src = torch.randint(0, n, (k,), generator=gen, device=DEV, dtype=torch.int32)
    print(f"append n={n} k={k}", flush=True)
    gs.gs_append([gs.Group(p, None, m, v, 1e-3)], gs.GS_MOMENT_F32, n, src, t)
    torch.cuda.synchronize()
    assert torch.equal(p[n:, 0], src.to(torch.float32) + 1)
    assert int((m[n:] != 0).sum()) == 0 and int((v[n:] != 0).sum()) == 0 and int((t[n:] != 0).sum()) == 0
    assert torch.equal(p[:n, 0], torch.arange(1, n + 1, dtype=torch.float32, device=DEV))
    assert int((m[:n] != 7).sum()) == 0 and int((v[:n] != 7).sum()) == 0 and int((t[:n] != 5).sum()) == 0
    del p, m, v, t, src
