"""GSOPT_TRACE: with the variable set, each step entry point logs one line
per launch on stderr (what it launches); unset or "0", it writes nothing."""
import os

import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

gs = pytest.importorskip("paper_2601_16736_amd")
from _gpu_util import DEV, make_state  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_trace_lines(capfd, monkeypatch):
    n = 3000
    st = make_state(gs, n, synth.GROUPS_59, 70)
    mask = torch.from_numpy(synth.bernoulli_mask(n, 0.3, 70, 0)).to(DEV)
    c = synth.camera_rig()[3]
    cam = gs.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far)

    def calls():
        gs.adamw_gs_step(st.groups, n, st.t, gs.StepConfig(iteration=2, schedule=gs.GS_SCHED_MASKED, unit=64),
                         visible=mask)
        gs.adamw_gs_step_view(st.groups, n, st.t, gs.StepConfig(iteration=3, moment_dtype=0, rsr_enable=True,
                                                                rsr_ratio=0.1), st.groups[0].param, [cam, cam])
        b = gs.Batch([gs.Scene(groups=st.groups, n=n, step_count=st.t, visible=mask,
                               schedule=gs.GS_SCHED_MASKED)])
        b.step(gs.StepConfig(iteration=4))
        b.close()
        torch.cuda.synchronize()

    monkeypatch.delenv("GSOPT_TRACE", raising=False)
    capfd.readouterr()
    calls()
    assert "gsopt:" not in capfd.readouterr().err
    monkeypatch.setenv("GSOPT_TRACE", "0")
    calls()
    assert "gsopt:" not in capfd.readouterr().err
    monkeypatch.setenv("GSOPT_TRACE", "1")
    calls()
    err = capfd.readouterr().err
    lines = [l for l in err.splitlines() if l.startswith("gsopt:")]
    assert len(lines) == 3, err
    assert lines[0].startswith("gsopt: adamw_gs_step n=3000 groups=5 schedule=masked unit=64 moments=f32 iteration=2")
    # a Re-State call: the fused step's default window is then 64
    assert lines[1].startswith("gsopt: adamw_gs_step_view n=3000 groups=5 schedule=view unit=64") and \
        "rsr=1" in lines[1] and lines[1].endswith("views=2")
    assert lines[2].startswith("gsopt: adamw_gs_step_batched n=3000 groups=5 schedule=plan") and "scenes=1" in lines[2]
