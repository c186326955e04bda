"""bench.py's host-side logic, without a GPU: the one-GPU contract, the
byte accounting constants, the counter-traffic lookup (valid only for the
source it was taken on) and the CPU oracle baseline leg."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
import synth  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_byte_constants():
    # theta r+w, g r, m r+w, v r+w per element; t r+w per primitive
    assert bench.BYTES_PER_VISIBLE["f32"] == 59 * (4 + 4 + 4 + 4 + 4 + 4 + 4) + 8 == 1660
    assert bench.BYTES_PER_VISIBLE["bf16"] == 59 * (4 + 4 + 4 + 2 + 2 + 2 + 2) + 8 == 1188
    assert bench.BYTES_PER_PRIMITIVE == {"two_launch": 1, "view": 12}


def test_traffic_lookup_only_for_the_measured_source_and_layout(tmp_path, monkeypatch):
    f = tmp_path / "traffic.json"
    f.write_text(json.dumps({"source_hash": bench.kernel_source_hash("view"), "order": "morton", "moments": "f32",
                             "bytes_per_launch": 1.5e9}))
    monkeypatch.setitem(bench.TRAFFIC_FILES, "view", str(f))
    assert bench.measured_traffic("morton", "f32", "view") == 1.5e9
    assert bench.measured_traffic("index", "f32", "view") is None
    assert bench.measured_traffic("morton", "bf16", "view") is None
    monkeypatch.setattr(bench, "kernel_source_hash", lambda path="view": "0" * 16)
    assert bench.measured_traffic("morton", "f32", "view") is None
    monkeypatch.setitem(bench.TRAFFIC_FILES, "view", str(tmp_path / "missing.json"))
    assert bench.measured_traffic("morton", "f32", "view") is None


def test_committed_traffic_summaries_name_the_sources_they_cover():
    for path in ("view", "two_launch"):
        d = json.load(open(bench.TRAFFIC_FILES[path]))
        assert d["hash_covers"] == list(bench.KERNEL_SOURCES[path]) + ["build.py"]
        assert d["source_hash"] == bench.kernel_source_hash(path), "counters taken on other sources or flags"
        assert d["bytes_per_launch"] == pytest.approx(d["fetched"] + d["written"])


def test_committed_traffic_is_close_to_the_algorithmic_bytes():
    """The committed counter figure is per launch of the headline instance
    (the plain steps).  It must lie between the algorithmic bytes and 10 %
    above them: a figure taken from another instance of the kernel, e.g. a
    Re-State launch, which also moves its sampled invisible rows, lands
    outside."""
    import re
    md = open(os.path.join(os.path.dirname(bench.TRAFFIC_FILES["view"]), "step_view_kernel_3M_traffic.md")).read()
    nv = float(re.search(r"visible (\d+) x 1660 B", md).group(1))
    for path in ("view", "two_launch"):
        d = json.load(open(bench.TRAFFIC_FILES[path]))
        alg = nv * bench.BYTES_PER_VISIBLE["f32"] + bench.N_PRIMS * bench.BYTES_PER_PRIMITIVE[path]
        assert 1.0 <= d["bytes_per_launch"] / alg <= 1.10, (path, d["bytes_per_launch"] / alg)


def test_gpu_clocks_never_raises():
    c = bench.gpu_clocks()
    assert c is None or all(isinstance(k, str) and isinstance(v, str) for k, v in c.items())


def test_cpu_baseline_leg_on_a_tiny_sample():
    pytest.importorskip("oracle")
    scene = synth.scene_uniform(5000, seed=0)
    cams = synth.camera_rig()
    order = synth.camera_order(len(cams), 50, seed=0)
    out = bench.cpu_baseline(scene, cams, order, budget_s=0.3, sample_n=2000, cores=3)
    assert out["kind"] == "oracle" and out["cores"] == 3 and out["unit"] == "attr-updates/s"
    assert out["value"] > 0 and np.isfinite(out["value"]) and out["value_1_thread"] > 0
    assert "2000" in out["sample"]
    assert 1 <= bench.host_cores() <= 16


def test_cpu_baseline_shards_reproduce_the_unsharded_oracle_step():
    """The baseline's threads each step a contiguous shard with its rows'
    scene indices; the result is the unsharded oracle's, bit for bit
    (Re-State draws included)."""
    import oracle
    n = 3000
    scene = synth.scene_uniform(n, seed=4)
    r = np.random.default_rng(0)

    def groups():
        out = []
        for name, dim, lr, dar in synth.GROUPS_59:
            p = scene.params[name].astype(np.float64)
            out.append(oracle.Group(p, 1e-3 * np.ones_like(p), np.full_like(p, 0.1), np.full_like(p, 0.2), lr,
                                    dar_kind=dar, dar_lambda=1e-3, dar_clip=10.0))
        return out

    mask = (r.random(n) < 0.4).astype(np.uint8)
    cfg = oracle.Config(iteration=7, rsr_enable=True, rsr_ratio=0.3)
    whole, t_whole = groups(), np.zeros(n, np.int32)
    oracle.adamw_gs_step(whole, n, mask, t_whole, cfg)
    parts, t_parts = groups(), np.zeros(n, np.int32)
    for a, b in ((0, 1100), (1100, 1101), (1101, n)):
        sub = [oracle.Group(G.param[a:b], G.grad[a:b], G.m[a:b], G.v[a:b], G.lr, dar_kind=G.dar_kind,
                            dar_lambda=G.dar_lambda, dar_clip=G.dar_clip) for G in parts]
        oracle.adamw_gs_step(sub, b - a, mask[a:b], t_parts[a:b], cfg, ids=np.arange(a, b, dtype=np.int64))
    assert np.array_equal(t_whole, t_parts)
    for A, B in zip(whole, parts):
        assert np.array_equal(A.param, B.param) and np.array_equal(A.m, B.m) and np.array_equal(A.v, B.v)


# --------------------------------------------------------------------------
# The whole default run on the CPU, with a stand-in for the HIP library: it
# exercises bench.py's own loops, camera orders and bookkeeping under the
# driver's flags (--steps 20 --warmup 5), which a leg with a step count of
# its own once indexed past the end of.
# --------------------------------------------------------------------------
class _FakeGS:
    """Records the calls the bench makes and writes plausible outputs: a
    visibility mask that depends on the camera, its count and index list;
    the steps leave every state unchanged."""

    GS_MOMENT_F32, GS_MOMENT_BF16 = 0, 1
    GS_SCHED_AUTO, GS_SCHED_COMPACTED, GS_SCHED_MASKED, GS_SCHED_DENSE = 0, 1, 2, 3

    def __init__(self, torch):
        import types
        self.torch = torch
        self.calls = {}

        class Group(types.SimpleNamespace):
            def __init__(self, param, grad, exp_avg, exp_avg_sq, lr, dar_kind=0, dar_lambda=0.0, dar_clip=0.0):
                super().__init__(param=param, grad=grad, exp_avg=exp_avg, exp_avg_sq=exp_avg_sq, lr=lr,
                                 dar_kind=dar_kind, dar_lambda=dar_lambda, dar_clip=dar_clip)

        class Camera(types.SimpleNamespace):
            def __init__(self, view, fx, fy, cx, cy, width, height, z_near=0.2, z_far=float("inf")):
                super().__init__(key=int(abs(float(np.asarray(view).sum())) * 1000) % 1000)

        class Scene(types.SimpleNamespace):
            pass

        fake = self

        class Batch:
            def __init__(self, scenes, moment_dtype=0):
                self.scenes = scenes

            def set_resident(self, r):
                pass

            def step(self, cfg, stream=None):
                fake._count("batched")

            def close(self):
                pass

        self.Group, self.Camera, self.Scene, self.Batch = Group, Camera, Scene, Batch
        self.StepConfig = lambda **kw: types.SimpleNamespace(**kw)

    def _count(self, name):
        self.calls[name] = self.calls.get(name, 0) + 1

    def _mask(self, n, cams):
        cams = cams if isinstance(cams, (list, tuple)) else [cams]
        m = self.torch.zeros(n, dtype=self.torch.bool)
        for c in cams:
            m |= (self.torch.arange(n) * 7 + c.key) % 10 < 3
        return m

    def gs_visibility(self, means, cam, mask=None, vis_idx=None, vis_count=None, stream=None):
        self._count("visibility")
        m = self._mask(means.shape[0], cam)
        if mask is not None:
            mask.copy_(m.to(mask.dtype))
        if vis_idx is not None:
            k = int(m.sum())
            vis_idx[:k] = self.torch.nonzero(m).squeeze(1).to(vis_idx.dtype)
            vis_count.fill_(k)

    def gs_visibility_multi(self, means, cams, mask=None, view_bits=None, vis_idx=None, vis_count=None,
                            stream=None):
        self._count("visibility_multi")
        self.gs_visibility(means, list(cams), mask=mask, vis_idx=vis_idx, vis_count=vis_count)

    def gs_compact(self, mask, vis_idx, vis_count, stream=None):
        k = int(mask.sum())
        vis_idx[:k] = self.torch.nonzero(mask).squeeze(1).to(vis_idx.dtype)
        vis_count.fill_(k)

    def adamw_gs_step(self, groups, n, t, cfg, visible=None, vis_idx=None, vis_count=None, stream=None):
        self._count("step")
        assert all(G.param.shape[0] == n for G in groups)

    def adamw_gs_step_view(self, groups, n, t, cfg, means, cams, visible_out=None, stream=None):
        self._count("step_view")
        if visible_out is not None:
            visible_out.copy_(self._mask(n, cams).to(visible_out.dtype))

    def prepare_step_view(self, groups, n, t, cfg, means, cams, visible_out=None, stream=None):
        groups = list(groups)
        return lambda: self.adamw_gs_step_view(groups, n, t, cfg, means, cams, visible_out, stream)

    def gs_spatial_order_workspace_size(self, n):
        return 16

    def gs_spatial_order(self, means, perm, ws, stream=None):
        perm.copy_(self.torch.arange(means.shape[0], dtype=perm.dtype))

    def apply_spatial_order(self, tensors, perm, stream=None):
        return [x[perm.long()].clone() for x in tensors]

    def gs_prune_workspace_size(self, n):
        return 16

    def gs_prune(self, keep, src, dst, mom, t, t_dst, kept, ws, stream=None):
        kept.fill_(int(keep.sum()))

    def gs_append(self, groups, mom, n, src_idx, t, stream=None):
        self._count("append")

    def gs_relocate_workspace_size(self, n):
        return 16

    def gs_relocate_reset(self, key, k, groups, mom, t, reset_t, ws, stream=None):
        self._count("relocate")

    def gs_tune(self, n, dims, p, mom=0):
        return (self.GS_SCHED_COMPACTED if p < 0.1 else self.GS_SCHED_MASKED), 64

    def gs_tune_mask(self, n, dims, mask, mom=0):
        self._count("tune_mask")
        return self.GS_SCHED_MASKED, 32

    def gs_tune_clear(self):
        pass


class _FakeEvents:
    def __init__(self, count):
        self.count = count

    def record(self, which, slot, stream):
        assert 0 <= slot < self.count

    def ms(self, slot):
        assert 0 <= slot < self.count
        return 0.25

    def close(self):
        pass


def test_default_run_under_the_driver_flags_prints_its_line(monkeypatch, capsys):
    import types

    import torch
    pytest.importorskip("oracle")
    fake = _FakeGS(torch)
    monkeypatch.setitem(sys.modules, "paper_2601_16736_amd", fake)
    monkeypatch.setattr(bench, "DEVICE", "cpu")
    monkeypatch.setattr(bench, "N_PRIMS", 3000)
    monkeypatch.setattr(bench, "MCMC_N", 4000)
    monkeypatch.setattr(bench, "BATCH_SIZE_RANGE", (200.0, 800.0))
    monkeypatch.setattr(bench, "CHECK_UNFUSED", False)
    monkeypatch.setattr(bench, "TimingEvents", _FakeEvents)
    monkeypatch.setattr(bench, "stream_ceilings",
                        lambda torch: {"rmw_4r3w_GBps": 5000.0, "rmw_4r3w_best_GBps": 6000.0, "table": {}})
    # the probes' kernels need a GPU: their results are stood in for
    monkeypatch.setattr(bench, "rows_ceiling", lambda *a, **k: {"GBps": 5500.0, "best_GBps": 5600.0})
    monkeypatch.setattr(bench, "batched_rows_ceiling", lambda *a, **k: {"kernel_ms_per_step": {"win32_i4": 2.0}})
    stream = types.SimpleNamespace(cuda_stream=0)
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a: None)
    monkeypatch.setattr(torch.cuda, "empty_cache", lambda *a: None)
    monkeypatch.setattr(torch.cuda, "set_device", lambda *a: None)
    monkeypatch.setattr(torch.cuda, "current_stream", lambda *a: stream)
    assert bench.main(["--steps", "20", "--warmup", "5", "--cpu-budget", "0.2"]) == 0
    line = [ln for ln in capsys.readouterr().out.splitlines() if ln.startswith("{")]
    assert len(line) == 1
    out = json.loads(line[0])
    assert out["steps"] == 20 and out["warmup"] == 5 and out["n_gpus"] == 1
    assert out["value"] > 0 and out["roofline"]["frac"] > 0
    assert out["cpu_baseline"]["kind"] == "oracle" and out["cpu_baseline"]["cores"] >= 1
    assert out["config"]["same_state_as_two_launch"] is True
    errors = []

    def walk(x, path=""):
        if isinstance(x, dict):
            if "error" in x:
                errors.append((path, x["error"]))
            for k, v in x.items():
                walk(v, f"{path}/{k}")
        elif isinstance(x, list):
            for i, v in enumerate(x):
                walk(v, f"{path}[{i}]")

    walk(out["variants"])
    assert errors == []
    names = set()
    for v in out["variants"]:
        names.update(v.keys())
    assert {"next_rows", "unfused_comparator", "tuner_3m", "config1_100k", "batched", "mcmc_6m"} <= names
    assert {"rows_f32", "rows_bf16"} <= set(out["stream_ceiling"])
    assert "two_launch_step_frac_of_best" in out["stream_ceiling"]["rows_f32"]
    assert fake.calls["step_view"] > 200 and fake.calls["relocate"] > 0 and fake.calls["batched"] > 0


def test_a_failing_variant_does_not_suppress_the_line(monkeypatch, capsys):
    import types

    import torch
    fake = _FakeGS(torch)
    monkeypatch.setitem(sys.modules, "paper_2601_16736_amd", fake)
    monkeypatch.setattr(bench, "DEVICE", "cpu")
    monkeypatch.setattr(bench, "N_PRIMS", 2000)
    monkeypatch.setattr(bench, "TimingEvents", _FakeEvents)

    def boom(*a, **k):
        raise IndexError("planted")

    for leg in ("run_next_rows", "run_unfused", "run_tuner", "run_config1", "run_batched", "run_mcmc_both",
                "stream_ceilings"):
        monkeypatch.setattr(bench, leg, boom)
    stream = types.SimpleNamespace(cuda_stream=0)
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a: None)
    monkeypatch.setattr(torch.cuda, "empty_cache", lambda *a: None)
    monkeypatch.setattr(torch.cuda, "set_device", lambda *a: None)
    monkeypatch.setattr(torch.cuda, "current_stream", lambda *a: stream)
    assert bench.main(["--steps", "20", "--warmup", "5", "--no-cpu-baseline"]) == 0
    line = [ln for ln in capsys.readouterr().out.splitlines() if ln.startswith("{")]
    out = json.loads(line[0])
    assert out["value"] > 0 and "roofline" in out
    assert "planted" in out["stream_ceiling"]["error"]
    assert any("planted" in json.dumps(v) for v in out["variants"])


@pytest.mark.parametrize("flag", ["--next-only", "--unfused-only", "--tuner-only"])
def test_single_leg_flags_print_their_leg(flag, monkeypatch, capsys):
    import types

    import torch
    fake = _FakeGS(torch)
    monkeypatch.setitem(sys.modules, "paper_2601_16736_amd", fake)
    monkeypatch.setattr(bench, "DEVICE", "cpu")
    monkeypatch.setattr(bench, "N_PRIMS", 3000)
    monkeypatch.setattr(bench, "CHECK_UNFUSED", False)
    monkeypatch.setattr(bench, "TimingEvents", _FakeEvents)
    stream = types.SimpleNamespace(cuda_stream=0)
    monkeypatch.setattr(torch.cuda, "synchronize", lambda *a: None)
    monkeypatch.setattr(torch.cuda, "current_stream", lambda *a: stream)
    assert bench.main([flag]) == 0
    line = [ln for ln in capsys.readouterr().out.splitlines() if ln.startswith("{")]
    assert len(line) == 1 and "error" not in json.loads(line[0])
