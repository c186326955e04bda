"""The no-allocation relocation entry point (gs_relocate_reset_noalloc,
through the C ABI) against the workspace entry point (gs_relocate_reset) on
the same inputs: the selected index lists and the whole end state (theta, m,
v, t of every group) must be bit-identical, over calls in a row on one
stream whose sizes shrink, so that a later call runs on the fixed device
workspace the earlier one left behind."""
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


def _keys(n: int, seed: int) -> np.ndarray:
    """Opacity-logit-like keys with many ties (a quarter-step grid) and signed zeros."""
    key = synth.rng(n, seed).integers(-40, 40, n).astype(np.float32) * np.float32(0.25)
    key[::11] = np.float32(-0.0)
    return key


def _same(a: dict, b: dict, label: str) -> None:
    np.testing.assert_array_equal(a["_t"], b["_t"], err_msg=f"{label}: step counts")
    for name in a:
        if name == "_t":
            continue
        for k in ("param", "m", "v"):
            np.testing.assert_array_equal(a[name][k], b[name][k], err_msg=f"{label}: {name}.{k}")


# (n, k, bf16 moments, reset_t): several 4096-key blocks with ragged tails,
# every call smaller than the one before it; the first is above the size
# where the per-block counts take a separate scan kernel (2048 blocks)
SMALL_SPEC = [("opacity", 1, 5e-2, 1), ("means", 3, 1.6e-4, 0)]
CALLS = [(9_000_011, 90_000, False, True), (300_007, 3_001, False, True), (20_011, 777, True, False),
         (4_097, 4_097, False, True), (1, 1, True, True)]


def test_noalloc_matches_the_workspace_entry_point_over_shrinking_calls():
    stream = torch.cuda.current_stream()
    runs = []
    # every call of both entry points is enqueued back to back on one stream
    # before anything is read back
    for j, (n, k, bf16, reset_t) in enumerate(CALLS):
        # the largest call keeps its rows narrow (two groups, 4 floats) so the
        # host copies stay small
        spec = (SMALL_SPEC if n > 1_000_000 else synth.GROUPS_59 if j % 2 == 0 else synth.GROUPS_60_SPLIT)
        key = _keys(n, 70 + j)
        a = make_state(gs, n, spec, seed=j, bf16=bf16)
        b = make_state(gs, n, spec, seed=j, bf16=bf16)
        before = a.host()
        d_key = torch.from_numpy(key).to(DEV)
        sel_a = torch.full((max(k, 1),), -7, dtype=torch.int32, device=DEV)
        sel_b = torch.full((max(k, 1),), -9, dtype=torch.int32, device=DEV)
        ws = torch.empty(gs.gs_relocate_workspace_size(n), dtype=torch.uint8, device=DEV)
        torch.cuda.synchronize()
        runs.append((n, k, key, a, b, before, sel_a, sel_b, ws, d_key, reset_t))
    for n, k, key, a, b, before, sel_a, sel_b, ws, d_key, reset_t in runs:
        gs.gs_relocate_reset(d_key, k, a.groups, int(a.bf16), a.t, reset_t, ws, selected=sel_a, stream=stream)
        gs.gs_relocate_reset_noalloc(d_key, k, b.groups, int(b.bf16), b.t, reset_t, selected=sel_b, stream=stream)
    torch.cuda.synchronize()
    for n, k, key, a, b, before, sel_a, sel_b, ws, d_key, reset_t in runs:
        label = f"n={n} k={k}"
        sa, sb = sel_a.cpu().numpy()[:k], sel_b.cpu().numpy()[:k]
        np.testing.assert_array_equal(sb, sa, err_msg=f"{label}: selected lists differ")
        # and both are the k smallest keys with ties to the lower index
        np.testing.assert_array_equal(sb.astype(np.int64), oracle.select_smallest(key, k), err_msg=label)
        ha, hb = a.host(), b.host()
        _same(ha, hb, label)
        picked = np.zeros(n, bool)
        picked[sb] = True
        for name in ha:
            if name != "_t":
                assert (hb[name]["m"][picked] == 0).all() and (hb[name]["v"][picked] == 0).all()
                np.testing.assert_array_equal(hb[name]["m"][~picked], before[name]["m"][~picked])
        if reset_t:
            assert (hb["_t"][picked] == 0).all()
        np.testing.assert_array_equal(hb["_t"][~picked], before["_t"][~picked])


def test_noalloc_second_call_on_leftover_workspace_with_no_selection():
    """k = 0 after a call that selected rows: nothing may change."""
    n = 50_000
    key = _keys(n, 90)
    d_key = torch.from_numpy(key).to(DEV)
    st = make_state(gs, n, synth.GROUPS_59, seed=9)
    gs.gs_relocate_reset_noalloc(d_key, 4_000, st.groups, 0, st.t, True)
    torch.cuda.synchronize()
    before = st.host()
    sel = torch.full((4,), -3, dtype=torch.int32, device=DEV)
    gs.gs_relocate_reset_noalloc(d_key[:20_000], 0, [type(g)(g.param[:20_000], g.grad[:20_000],
                                                             g.exp_avg[:20_000], g.exp_avg_sq[:20_000], g.lr)
                                                     for g in st.groups], 0, st.t[:20_000], True, selected=sel)
    torch.cuda.synchronize()
    _same(st.host(), before, "k = 0")
    assert (sel.cpu().numpy() == -3).all()


def test_noalloc_refuses_sizes_above_its_maximum():
    class Big:
        shape = (gs.GS_RELOCATE_NOALLOC_MAX_N + 1,)

        @staticmethod
        def data_ptr():
            return 0x7F0000000000

    st = make_state(gs, 8, synth.GROUPS_59, seed=1)
    with pytest.raises(gs.GsError) as e:
        gs.gs_relocate_reset_noalloc(Big(), 1, st.groups, 0, st.t, True)
    assert e.value.status == gs.GS_EINVAL
