"""Stochastic rounding of BF16 moments on the GPU, statistically.

Every element of a group gets the same gradient from zero state, so all of
them round the same FP32 value x (m = (1 - beta1) g, v = (1 - beta2) g^2,
formed as the host below forms them).  Adding 16 uniform bits below the
kept bits and truncating rounds x up (away from zero) with probability
exactly (low 16 bits of x) / 2^16.  Checked within 5 binomial standard
deviations: that probability for m and v; that every stored value is one
of x's two bf16 neighbours; that the m and v decisions of an element (two
halves of one 32-bit word) are uncorrelated; and that two consecutive
elements (the two halves of one 64-bit draw) decide independently.  A
4-wide group (vector stores) and a 3-wide one (scalar stores, pairs that
straddle rows, negative values) are both covered."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

gs = pytest.importorskip("paper_2601_16736_amd")
from _gpu_util import DEV  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _within(count, n, p, label):
    sd = np.sqrt(n * p * (1 - p))
    assert abs(count - n * p) <= 5 * sd, f"{label}: {count} of {n}, expected {n * p:.0f} +- {5 * sd:.0f}"


def test_stochastic_rounding_is_unbiased_and_independent():
    n = 400_000
    g0 = np.float32(1.2345e-3)
    omb1, omb2 = np.float32(1 - 0.9), np.float32(1 - 0.999)
    groups = []
    for dim, sign in ((4, None), (3, np.array([1, -1, 1], np.float32))):
        grad = np.full((n, dim), g0, np.float32)
        if sign is not None:
            grad *= sign
        groups.append(gs.Group(torch.zeros((n, dim), device=DEV), torch.from_numpy(grad).to(DEV),
                               torch.zeros((n, dim), dtype=torch.bfloat16, device=DEV),
                               torch.zeros((n, dim), dtype=torch.bfloat16, device=DEV), 1e-3))
    t = torch.zeros(n, dtype=torch.int32, device=DEV)
    mask = torch.ones(n, dtype=torch.uint8, device=DEV)
    cfg = gs.StepConfig(iteration=5, seed=123, schedule=gs.GS_SCHED_MASKED, unit=32, moment_dtype=gs.GS_MOMENT_BF16,
                        stochastic_round=True)
    gs.adamw_gs_step(groups, n, t, cfg, visible=mask)
    torch.cuda.synchronize()
    for k, G in enumerate(groups):
        grad = G.grad.cpu().numpy()
        ups = {}
        for key, stored, x in (("m", G.exp_avg, omb1 * grad), ("v", G.exp_avg_sq, omb2 * (grad * grad))):
            bits = stored.view(torch.int16).cpu().numpy().view(np.uint16).astype(np.uint32)
            xb = x.view(np.uint32)
            lo, hi = xb >> 16, (xb >> 16) + 1
            assert np.all((bits == lo) | (bits == hi)), f"group {k} {key}: a value outside x's bf16 neighbours"
            up = bits == hi
            p = (xb & 0xFFFF).astype(np.float64) / 65536.0
            assert np.all(p == p.flat[0]) or key == "m"          # one x per group (m: +-x)
            _within(int(up.sum()), up.size, float(p.flat[0]), f"group {k} {key} rounded up")
            ups[key] = (up, float(p.flat[0]))
        (um, pm), (uv, pv) = ups["m"], ups["v"]
        _within(int((um & uv).sum()), um.size, pm * pv, f"group {k}: m and v of one element both up")
        flat = um.reshape(-1)
        pairs = flat[: flat.size // 2 * 2].reshape(-1, 2)        # elements 2j, 2j+1 share a 64-bit draw
        _within(int((pairs[:, 0] & pairs[:, 1]).sum()), pairs.shape[0], pm * pm,
                f"group {k}: both elements of a draw pair up")
