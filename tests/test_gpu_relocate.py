"""Relocation state reset: the selected index list must equal the oracle's
(k smallest keys, ties to the lower index) exactly; the selected rows' m, v
(and t) are zero; every other row is bit-identical."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

gs = pytest.importorskip("paper_2601_16736_amd")
from _gpu_util import DEV, make_state  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)


def _run(key: np.ndarray, k: int, bf16: bool = False, reset_t: bool = True, spec=synth.GROUPS_59, seed=0,
         want_list: bool = True):
    n = key.shape[0]
    st = make_state(gs, n, spec, seed, bf16=bf16)
    before = st.host()
    d_key = torch.from_numpy(key).to(DEV)
    sel = torch.full((max(k, 1),), -7, dtype=torch.int32, device=DEV)
    ws = torch.empty(gs.gs_relocate_workspace_size(n), dtype=torch.uint8, device=DEV)
    gs.gs_relocate_reset(d_key, k, st.groups, int(bf16), st.t, reset_t, ws, selected=sel if want_list else None)
    torch.cuda.synchronize()
    after = st.host()
    ref = oracle.select_smallest(key, k)
    if want_list:
        np.testing.assert_array_equal(sel.cpu().numpy()[:k].astype(np.int64), ref)
    picked = np.zeros(n, bool)
    picked[ref] = True
    for name, *_ in spec:
        A, B = after[name], before[name]
        assert (A["m"][picked] == 0).all() and (A["v"][picked] == 0).all()
        np.testing.assert_array_equal(A["m"][~picked], B["m"][~picked])
        np.testing.assert_array_equal(A["v"][~picked], B["v"][~picked])
        np.testing.assert_array_equal(A["param"], B["param"])
    if reset_t:
        assert (after["_t"][picked] == 0).all()
    else:
        np.testing.assert_array_equal(after["_t"][picked], before["_t"][picked])
    np.testing.assert_array_equal(after["_t"][~picked], before["_t"][~picked])


@pytest.mark.parametrize("n", [1, 4095, 4096, 4097, 50_001])
def test_select_with_many_ties(n):
    key = synth.rng(n, 60).integers(-20, 20, n).astype(np.float32) * np.float32(0.25)
    for k in sorted({0, 1, min(n, 50), n // 2, n}):
        _run(key, k, seed=n + k)


def test_select_continuous_keys_and_signed_zero():
    n = 20_000
    key = synth.rng(61).standard_normal(n).astype(np.float32)
    key[::7] = np.float32(-0.0)
    key[3::7] = np.float32(0.0)
    for k in (1, 2857, 2858, 6000, 19_999):
        _run(key, k)


def test_reset_without_index_list():
    """selected = NULL: the rows are still reset, from the same selection."""
    key = synth.rng(65).integers(-8, 8, 30_001).astype(np.float32)
    for k in (0, 1, 777, 30_001):
        _run(key, k, want_list=False, seed=k)


def test_bf16_moments_and_keep_t():
    key = synth.rng(62).standard_normal(9000).astype(np.float32)
    _run(key, 90, bf16=True, reset_t=False, spec=synth.GROUPS_60_SPLIT)


def test_mcmc_shape_6m_one_percent():
    """6M primitives (the 3DGS-MCMC cap), 1 % lowest opacity logits."""
    n, k = 6_000_000, 60_000
    key = synth.rng(63).standard_normal(n).astype(np.float32)
    d_key = torch.from_numpy(key).to(DEV)
    spec = [("opacity", 1, 5e-2, 1), ("sh", 48, 2.5e-3, 0)]
    st = make_state(gs, n, spec, 5)
    sel = torch.empty(k, dtype=torch.int32, device=DEV)
    ws = torch.empty(gs.gs_relocate_workspace_size(n), dtype=torch.uint8, device=DEV)
    gs.gs_relocate_reset(d_key, k, st.groups, 0, st.t, True, ws, selected=sel)
    torch.cuda.synchronize()
    ref = np.sort(np.argsort(key, kind="stable")[:k])
    np.testing.assert_array_equal(sel.cpu().numpy().astype(np.int64), ref)
    rows = torch.from_numpy(ref).to(DEV)
    assert torch.count_nonzero(st.groups[1].exp_avg[rows]).item() == 0
    assert torch.count_nonzero(st.t[rows]).item() == 0


def test_select_past_the_inline_scan_limit():
    """More than 2048 blocks of 4096 keys: the per-block counts go through
    the separate scan kernel instead of being summed by each block."""
    n = 2048 * 4096 + 4097
    key = (synth.rng(64).integers(-300, 300, n).astype(np.float32) * np.float32(0.5))
    d_key = torch.from_numpy(key).to(DEV)
    st = make_state(gs, n, [("opacity", 1, 5e-2, 1)], 6)
    ws = torch.empty(gs.gs_relocate_workspace_size(n), dtype=torch.uint8, device=DEV)
    for k in (1, 100_003, n - 5):
        sel = torch.empty(k, dtype=torch.int32, device=DEV)
        print(f"relocate n={n} k={k}", flush=True)
        gs.gs_relocate_reset(d_key, k, st.groups, 0, st.t, True, ws, selected=sel)
        torch.cuda.synchronize()
        ref = np.sort(np.argsort(key, kind="stable")[:k])
        np.testing.assert_array_equal(sel.cpu().numpy().astype(np.int64), ref)


@pytest.mark.parametrize("layout", ["offset", "strided"])
def test_select_unaligned_and_strided_keys(layout):
    """Keys one float past a 16-byte boundary, or every third float of a
    packed [n][3] tensor: the counting passes read them with per-key loads
    instead of 16-byte ones, over whole blocks and a ragged last block."""
    n = 3 * 4096 + 777
    key = synth.rng(66).integers(-50, 50, n).astype(np.float32) * np.float32(0.125)
    if layout == "offset":
        base = torch.zeros(n + 1, dtype=torch.float32, device=DEV)
        base[1:] = torch.from_numpy(key).to(DEV)
        d_key = base[1:]
        assert d_key.data_ptr() % 16 == 4
    else:
        base = torch.zeros((n, 3), dtype=torch.float32, device=DEV)
        base[:, 1] = torch.from_numpy(key).to(DEV)
        d_key = base[:, 1]
        assert d_key.stride() == (3,)
    st = make_state(gs, n, [("opacity", 1, 5e-2, 1), ("scale", 3, 5e-3, 2)], 7)
    ws = torch.empty(gs.gs_relocate_workspace_size(n), dtype=torch.uint8, device=DEV)
    for k in (1, 4096, 9000):
        sel = torch.full((k,), -7, dtype=torch.int32, device=DEV)
        print(f"relocate {layout} n={n} k={k}", flush=True)
        gs.gs_relocate_reset(d_key, k, st.groups, 0, st.t, True, ws, selected=sel)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(sel.cpu().numpy().astype(np.int64), oracle.select_smallest(key, k))


def test_select_keys_sharing_the_16_bit_prefix():
    """Every key has the same upper 16 bits (1.0 plus up to 65535 ulps), so all
    of them reach the last pass's 16-bit table, a wave's lanes in up to 64
    different bins; shuffled, with repeats (ties) and a ragged last block."""
    n = 3 * 4096 + 5
    r = synth.rng(67)
    low = r.integers(0, 1 << 16, n).astype(np.uint32)
    low[::5] = low[0]                                   # a large run of equal keys
    key = (np.uint32(0x3F800000) | low).view(np.float32)
    assert len({int(x) >> 16 for x in key.view(np.uint32)}) == 1
    for k in (1, 777, n // 5, n // 2, n - 1):
        _run(key, k, seed=k, spec=[("opacity", 1, 5e-2, 1)])
