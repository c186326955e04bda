"""The benchmark's streaming-ceiling kernels (libgsprobe): exported symbols and
argument rejection on the host; on a GPU, that each kernel does the work it
is timed for (every element read and written as stated)."""
import ctypes
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2601_16736_amd", "libgsprobe.so")


def _lib():
    if not os.path.exists(LIB):
        pytest.skip("libgsprobe.so not built")
    lib = ctypes.CDLL(LIB)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    lib.gsprobe_rmw_4r3w.argtypes = [vp, vp, vp, vp, i64, vp]
    lib.gsprobe_copy.argtypes = [vp, vp, i64, vp]
    lib.gsprobe_read.argtypes = [vp, i64, vp, vp]
    return lib


def test_probe_rejects_bad_arguments_before_any_launch():
    lib = _lib()
    assert lib.gsprobe_rmw_4r3w(None, None, None, None, 16, None) == -1
    assert lib.gsprobe_copy(None, 16, 16, None) == -1            # null destination
    assert lib.gsprobe_copy(32, 17, 16, None) == -1              # misaligned source
    assert lib.gsprobe_copy(32, 48, 0, None) == -1               # empty
    assert lib.gsprobe_read(None, 16, 64, None) == -1


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
