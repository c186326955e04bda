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


def _rows_args(arrs):
    ng = len(arrs)
    ptrs = [(ctypes.c_void_p * ng)(*[a[k] for a in arrs]) for k in range(4)]
    return ptrs


def test_rows_probe_rejects_bad_arguments_before_any_launch():
    lib = _lib()
    dims = (ctypes.c_int32 * 2)(3, 48)
    good = [(16, 32, 48, 64), (80, 96, 112, 128)]
    ptrs = _rows_args(good)
    assert lib.gsprobe_rows_4r3w_cfg(None, 16, *ptrs, dims, 2, 100, 32, 4, 0, None) == -1      # mask
    assert lib.gsprobe_rows_4r3w_cfg(16, 16, *ptrs, dims, 0, 100, 32, 4, 0, None) == -1        # no group
    assert lib.gsprobe_rows_4r3w_cfg(16, 16, *ptrs, dims, 9, 100, 32, 4, 0, None) == -1        # too many
    assert lib.gsprobe_rows_4r3w_cfg(16, 16, *ptrs, dims, 2, 0, 32, 4, 0, None) == -1          # empty
    assert lib.gsprobe_rows_4r3w_cfg(16, 16, *ptrs, dims, 2, 100, 48, 4, 0, None) == -1        # window
    assert lib.gsprobe_rows_4r3w_cfg(16, 16, *ptrs, dims, 2, 100, 32, 3, 0, None) == -1        # items
    bad_dims = (ctypes.c_int32 * 2)(3, 65)
    assert lib.gsprobe_rows_4r3w_cfg(16, 16, *ptrs, bad_dims, 2, 100, 32, 4, 0, None) == -1    # width
    mis = _rows_args([(16, 32, 48, 64), (80, 100, 112, 128)])                               # 4-wide, misaligned
    assert lib.gsprobe_rows_4r3w_cfg(16, 16, *mis, dims, 2, 100, 32, 4, 0, None) == -1
    assert lib.gsprobe_rows_4r3w_cfg(16, 16, *ptrs, dims, 2, 100, 32, 4, 2, None) == -1     # moment type
    mis8 = _rows_args([(16, 32, 48, 64), (80, 96, 116, 128)])                               # BF16 moments at 4 B
    assert lib.gsprobe_rows_4r3w_cfg(16, 16, *mis8, dims, 2, 100, 32, 4, 1, None) == -1


@pytest.mark.gpu
@pytest.mark.parametrize("bf16", [0, 1])
def test_rows_probe_touches_exactly_the_masked_rows_in_every_shape(bf16):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import bench
    lib = _lib()
    dev = torch.device("cuda:0")
    n = 4 * 256 + 77                          # several windows of every size and a ragged tail
    dims = [3, 3, 4, 1, 48]
    r = np.random.default_rng(8)
    mask_h = (r.random(n) < 0.35).astype(np.uint8)
    mask_h[:64] = 1                           # a full window
    mask_h[64:128] = 0                        # an empty one
    keep = mask_h.astype(bool)
    sp = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for (win, items) in bench.ROWS_PROBE_SHAPES:
        host = []
        for d in dims:
            p, g = (r.standard_normal((n, d)).astype(np.float32) for _ in range(2))
            if bf16:
                m, v = (r.integers(0, 1 << 16, (n, d)).astype(np.uint16) for _ in range(2))
            else:
                m, v = (r.standard_normal((n, d)).astype(np.float32) for _ in range(2))
            host.append((p, g, m, v))
        dev_arrs = [[torch.from_numpy(h.view(np.int16) if h.dtype == np.uint16 else h).to(dev) for h in grp]
                    for grp in host]
        t = torch.zeros(n, dtype=torch.int32, device=dev)
        mask = torch.from_numpy(mask_h).to(dev)
        ptrs = [(ctypes.c_void_p * len(dims))(*[grp[k].data_ptr() for grp in dev_arrs]) for k in range(4)]
        cd = (ctypes.c_int32 * len(dims))(*dims)
        assert lib.gsprobe_rows_4r3w_cfg(mask.data_ptr(), t.data_ptr(), *ptrs, cd, len(dims), n, win, items, bf16,
                                         sp) == 0
        torch.cuda.synchronize()
        np.testing.assert_array_equal(t.cpu().numpy(), keep.astype(np.int32))
        for (P, G, M, V), grp in zip(host, dev_arrs):
            pp = P - np.float32(0.0625) * G
            np.testing.assert_allclose(grp[0].cpu().numpy(), np.where(keep[:, None], pp, P), rtol=1e-6, atol=1e-7,
                                       err_msg=f"window {win}, items {items}")
            np.testing.assert_array_equal(grp[1].cpu().numpy(), G)
            if bf16:
                for want, got in ((M, grp[2]), (V, grp[3])):
                    np.testing.assert_array_equal(got.cpu().numpy().view(np.uint16),
                                                  np.where(keep[:, None], want ^ np.uint16(1), want))
            else:
                mm = np.float32(0.875) * M + np.float32(0.125) * G
                vv = np.float32(0.5) * V + np.float32(0.5) * G * G
                for want, got in ((np.where(keep[:, None], mm, M), grp[2]), (np.where(keep[:, None], vv, V), grp[3])):
                    np.testing.assert_allclose(got.cpu().numpy(), want, rtol=1e-6, atol=1e-7,
                                               err_msg=f"window {win}, items {items}")
