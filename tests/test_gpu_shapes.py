"""Group shapes and layouts the 3DGS workloads do not exercise, against the
oracle through the C ABI: dims from 1 to 4096 (rows shorter than a wave and
rows spanning many wave-widths of chunks), and groups that are views into
one packed buffer at offsets that force 8- or 4-byte accesses.  Same bars
as the step parity tests."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

gs = pytest.importorskip("paper_2601_16736_amd")
from _gpu_util import DEV, compare, oracle_config, oracle_groups  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)


class _St:
    def __init__(self, groups, spec, t, bf16):
        self.groups, self.spec, self.t, self.bf16 = groups, spec, t, bf16

    def host(self):
        from _gpu_util import GpuState
        return GpuState(self.groups, self.spec, self.t, self.bf16).host()


def _packed_state(n, dims, seed, bf16, offsets=None):
    """Every array of every group is a view into one flat buffer per kind
    (param, grad, m, v); `offsets` (elements) shifts each group's start."""
    r = synth.rng(seed, 200)
    offsets = offsets or [0] * len(dims)
    total = sum(n * d + o for d, o in zip(dims, offsets))
    mdt = torch.bfloat16 if bf16 else torch.float32
    bufs = {k: torch.zeros(total + 8, dtype=torch.float32 if k in ("p", "g") else mdt, device=DEV)
            for k in ("p", "g", "m", "v")}
    groups, spec, at = [], [], 0
    for k, (d, o) in enumerate(zip(dims, offsets)):
        at += o
        views = {key: buf[at:at + n * d].view(n, d) for key, buf in bufs.items()}
        views["p"].copy_(torch.from_numpy(r.standard_normal((n, d), dtype=np.float32)))
        views["g"].copy_(torch.from_numpy((1e-3 * r.standard_normal((n, d))).astype(np.float32)))
        views["m"].copy_(torch.from_numpy((1e-4 * r.standard_normal((n, d))).astype(np.float32)).to(mdt))
        views["v"].copy_(torch.from_numpy((1e-6 * r.random((n, d)) + 1e-9).astype(np.float32)).to(mdt))
        dar = (1, 2, 0)[k % 3]
        lam = (1e-3, 1e-5, 0.0)[k % 3]
        lr = (5e-2, 5e-3, 1e-3)[k % 3]
        groups.append(gs.Group(views["p"], views["g"], views["m"], views["v"], lr, dar_kind=dar, dar_lambda=lam,
                               dar_clip=10.0))
        spec.append((f"g{k}", d, lr, dar))
        at += n * d
    t = torch.from_numpy(r.integers(0, 30, n).astype(np.int32)).to(DEV)
    return _St(groups, spec, t, bf16)


def _run(n, dims, sched, unit, bf16, seed, offsets=None, rsr=True):
    st = _packed_state(n, dims, seed, bf16, offsets)
    mask = synth.bernoulli_mask(n, 0.4, seed, 1)
    for g in st.groups:
        g.grad[torch.from_numpy(mask == 0).to(DEV)] = float("nan")    # invisible gradients are never read
    d_mask = torch.from_numpy(mask).to(DEV)
    idx = torch.zeros(max(n, 1), dtype=torch.int32, device=DEV)
    cnt = torch.zeros(1, dtype=torch.int32, device=DEV)
    gs.gs_compact(d_mask, idx, cnt)
    cfg = gs.StepConfig(iteration=9, seed=seed, moment_dtype=int(bf16), stochastic_round=bf16, rsr_enable=rsr,
                        rsr_ratio=0.3, schedule=sched, unit=unit)
    torch.cuda.synchronize()
    before = st.host()
    print(f"shapes n={n} dims={dims} sched={sched}/{unit} bf16={bf16} offsets={offsets}", flush=True)
    gs.adamw_gs_step(st.groups, n, st.t, cfg, visible=d_mask, vis_idx=idx, vis_count=cnt)
    torch.cuda.synchronize()
    og = oracle_groups(before, st.spec, st.groups)
    t_ref = before["_t"].copy()
    oracle.adamw_gs_step(og, n, mask, t_ref, oracle_config(cfg))
    touched = mask.astype(bool)
    if rsr:
        touched |= oracle.rsr_sample_mask(cfg.seed, cfg.iteration, n, cfg.rsr_ratio)
    compare(st.host(), before, og, st.spec, t_ref, touched, bf16, label=f"dims={dims}")


@pytest.mark.parametrize("dims", [(1,), (2, 6, 10), (5, 7, 129), (64, 256), (1024,), (4096,)])
@pytest.mark.parametrize("sched,unit", [(gs.GS_SCHED_COMPACTED, 64), (gs.GS_SCHED_MASKED, 256)])
@pytest.mark.parametrize("bf16", [False, True])
def test_step_dims(dims, sched, unit, bf16):
    n = 1500 if max(dims) < 1024 else 300
    _run(n, dims, sched, unit, bf16, seed=sum(dims))


@pytest.mark.parametrize("offsets", [[1, 1, 1], [2, 0, 2], [0, 3, 1]])
@pytest.mark.parametrize("bf16", [False, True])
def test_step_packed_views_at_odd_offsets(offsets, bf16):
    """Views at odd element offsets into shared buffers: 16-byte accesses are
    impossible, so the kernels fall back to 8- or 4-byte ones."""
    _run(2001, (4, 48, 8), gs.GS_SCHED_COMPACTED, 128, bf16, seed=7 + sum(offsets), offsets=offsets)
