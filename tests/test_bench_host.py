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
        assert d["hash_covers"] == list(bench.KERNEL_SOURCES[path])
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
    out = bench.cpu_baseline(scene, cams, order, budget_s=0.3, sample_n=2000)
    assert out["kind"] == "oracle" and out["cores"] == 1 and out["unit"] == "attr-updates/s"
    assert out["value"] > 0 and np.isfinite(out["value"])
    assert "2000" in out["sample"]
