"""The benchmark's streaming-ceiling kernels (bench_probe/libgsprobe.so):
exported symbols and argument rejection on the host; on a GPU, that each
kernel does the work it is timed for (every element read and written as
stated), in every launch shape the benchmark sweeps."""
import ctypes
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench_probe  # noqa: E402


def _lib():
    if not os.path.exists(bench_probe.LIB):
        pytest.skip("libgsprobe.so not built")
    return bench_probe.load()


def test_probe_rejects_bad_arguments_before_any_launch():
    lib = _lib()
    assert lib.gsprobe_rmw_4r3w(None, None, None, None, 16, None) == -1
    assert lib.gsprobe_copy(None, 16, 16, None) == -1            # null destination
    assert lib.gsprobe_copy(32, 17, 16, None) == -1              # misaligned source
    assert lib.gsprobe_copy(32, 48, 0, None) == -1               # empty
    assert lib.gsprobe_read(None, 16, 64, None) == -1
    assert lib.gsprobe_rmw_4r3w_cfg(32, 48, 64, 80, 16, 12, 4, 1, 1, 0, None) == -1   # width
    assert lib.gsprobe_rmw_4r3w_cfg(32, 48, 64, 80, 16, 16, 3, 1, 1, 0, None) == -1   # items
    assert lib.gsprobe_copy_cfg(32, 48, 16, 8, 4, 1, 1, -1, None) == -1               # blocks
    assert lib.gsprobe_read_cfg(32, 0, 64, 16, 4, 1, 0, None) == -1                   # empty


@pytest.mark.gpu
def test_probe_kernels_do_their_work():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib = _lib()
    dev = torch.device("cuda:0")
    n16 = 5 * 1024 + 37                       # several blocks and a ragged tail
    r = np.random.default_rng(5)
    host = [r.standard_normal(4 * n16).astype(np.float32) for _ in range(4)]
    p, g, m, v = [torch.from_numpy(h).to(dev) for h in host]
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.gsprobe_rmw_4r3w(p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), n16, sp) == 0
    dst = torch.zeros_like(g)
    assert lib.gsprobe_copy(dst.data_ptr(), g.data_ptr(), n16, sp) == 0
    sink = torch.zeros(4, device=dev)
    assert lib.gsprobe_read(g.data_ptr(), n16, sink.data_ptr(), sp) == 0
    torch.cuda.synchronize()
    P, G, M, V = host
    mm = np.float32(0.875) * M + np.float32(0.125) * G
    vv = np.float32(0.5) * V + np.float32(0.5) * G * G
    np.testing.assert_allclose(m.cpu().numpy(), mm, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(v.cpu().numpy(), vv, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(p.cpu().numpy(), P - np.float32(0.0625) * mm, rtol=1e-6, atol=1e-7)
    np.testing.assert_array_equal(dst.cpu().numpy(), G)
    assert sink.cpu().numpy()[0] == 0.0


@pytest.mark.gpu
def test_every_swept_launch_shape_does_its_work():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import bench
    lib = _lib()
    dev = torch.device("cuda:0")
    n16 = 3 * 2048 + 21                       # several tiles of every shape and a ragged tail
    r = np.random.default_rng(6)
    host = [r.standard_normal(4 * n16).astype(np.float32) for _ in range(4)]
    P, G, M, V = host
    mm = np.float32(0.875) * M + np.float32(0.125) * G
    vv = np.float32(0.5) * V + np.float32(0.5) * G * G
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    sink = torch.zeros(4, device=dev)
    for (w, it, ntl, nts, b) in bench.PROBE_SHAPES:
        p, g, m, v = [torch.from_numpy(h).to(dev) for h in host]
        assert lib.gsprobe_rmw_4r3w_cfg(p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), n16, w, it, ntl,
                                        nts, min(b, 5), sp) == 0
        dst = torch.zeros_like(g)
        assert lib.gsprobe_copy_cfg(dst.data_ptr(), g.data_ptr(), n16, w, it, ntl, nts, min(b, 5), sp) == 0
        assert lib.gsprobe_read_cfg(g.data_ptr(), n16, sink.data_ptr(), w, it, ntl, min(b, 5), sp) == 0
        torch.cuda.synchronize()
        shape = (w, it, ntl, nts, b)
        np.testing.assert_allclose(m.cpu().numpy(), mm, rtol=1e-6, atol=1e-7, err_msg=str(shape))
        np.testing.assert_allclose(v.cpu().numpy(), vv, rtol=1e-6, atol=1e-7, err_msg=str(shape))
        np.testing.assert_allclose(p.cpu().numpy(), P - np.float32(0.0625) * mm, rtol=1e-6, atol=1e-7,
                                   err_msg=str(shape))
        np.testing.assert_array_equal(dst.cpu().numpy(), G, err_msg=str(shape))
    assert sink.cpu().numpy()[0] == 0.0
