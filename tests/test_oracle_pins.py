"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test checks the oracle against something the paper or the mathematics
fixes: published test vectors, closed forms, a library implementation of
textbook Adam, hand computations written as numbers, invariants the paper
states, and brute force on tiny inputs.  None needs a GPU.
"""
import math
import os

import numpy as np
import pytest
import torch

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def _one_group(n, dim, lr, dar_kind=0, lam=0.0, clip=0.0, theta=None, reg_mode=0):
    theta = np.zeros((n, dim)) if theta is None else np.array(theta, dtype=np.float64).reshape(n, dim)
    return oracle.Group(param=theta.copy(), grad=np.zeros((n, dim)), m=np.zeros((n, dim)),
                        v=np.zeros((n, dim)), lr=lr, dar_kind=dar_kind, dar_lambda=lam,
                        dar_clip=clip, reg_mode=reg_mode)


# ---------------------------------------------------------------- hashing
def test_splitmix64_reference_vector():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_seed0.txt")) if l[0] != "#"]
    for k, hexv in rows:
        assert oracle.splitmix_output(0, int(k)) == int(hexv, 16)


def test_nested_stream_definition():
    # draw(seed, tag, it, e) is the (e+1)-th output of the stream whose state
    # is the (it+1)-th output of the stream whose state is the (tag+1)-th
    # output of the stream seeded with `seed`.
    seed, tag, it, e = 12345, 1, 77, 999
    s1 = oracle.splitmix_output(seed, tag + 1)
    s2 = oracle.splitmix_output(s1, it + 1)
    assert oracle.stream_state(seed, tag, it) == s2
    assert oracle.draw(seed, tag, it, e) == oracle.splitmix_output(s2, e + 1)


def test_rsr_threshold_edges():
    assert oracle.rsr_threshold(0.0) == 0
    assert oracle.rsr_threshold(1.0) == 2**32
    assert oracle.rsr_threshold(0.5) == 2**31
    assert oracle.rsr_threshold(0.05) == math.floor(0.05 * 2**32)


# ---------------------------------------------------------------- N_I'
def test_reg_norm_examples():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "reg_norm.txt")) if l[0] != "#"]
    for n_i, expect in rows:
        assert oracle.reg_norm(float(n_i)) == pytest.approx(float(expect), rel=0, abs=1e-12)


# ---------------------------------------------------------------- Adam reductions
def _torch_adam_on_sequence(theta0, grads, lr, betas, eps):
    p = torch.tensor(theta0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([p], lr=lr, betas=betas, eps=eps, foreach=False)
    for g in grads:
        p.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
    st = opt.state[p]
    return p.detach().numpy(), st["exp_avg"].numpy(), st["exp_avg_sq"].numpy()


@pytest.mark.parametrize("dim", [1, 3, 48])
def test_sparse_adam_is_textbook_adam_on_visible_subsequence(dim):
    """Sparse Adam (sparse-beta equation): each primitive's trajectory is
    Kingma-Ba Adam run on the subsequence of its visible-step gradients."""
    n, steps, lr, b1, b2, eps = 7, 25, 1e-2, 0.9, 0.999, 1e-8
    g_rng = np.random.default_rng(3)
    theta0 = g_rng.standard_normal((n, dim))
    grp = _one_group(n, dim, lr, theta=theta0)
    t = np.zeros(n, np.int32)
    masks = (g_rng.random((steps, n)) < 0.4).astype(np.uint8)
    masks[:, 0] = 1                      # one always-visible primitive (dense Adam)
    allg = g_rng.standard_normal((steps, n, dim)) * 1e-2
    seen = [[] for _ in range(n)]
    for s in range(steps):
        grp.grad[:] = np.where(masks[s][:, None] == 1, allg[s], np.nan)   # invisible grads never read
        oracle.adamw_gs_step([grp], n, masks[s], t, oracle.Config(beta1=b1, beta2=b2, eps=eps, iteration=s))
        for i in range(n):
            if masks[s, i]:
                seen[i].append(allg[s, i])
    for i in range(n):
        assert t[i] == len(seen[i])
        if not seen[i]:
            np.testing.assert_array_equal(grp.param[i], theta0[i])
            continue
        p, m, v = _torch_adam_on_sequence(theta0[i], seen[i], lr, (b1, b2), eps)
        np.testing.assert_allclose(grp.param[i], p, rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(grp.m[i], m, rtol=1e-12, atol=1e-18)
        np.testing.assert_allclose(grp.v[i], v, rtol=1e-12, atol=1e-20)


def test_dense_when_no_mask():
    n, dim = 5, 4
    rng = np.random.default_rng(0)
    theta0 = rng.standard_normal((n, dim))
    grp = _one_group(n, dim, 1e-3, theta=theta0)
    t = np.zeros(n, np.int32)
    gs = [rng.standard_normal((n, dim)) for _ in range(6)]
    for s, g in enumerate(gs):
        grp.grad[:] = g
        oracle.adamw_gs_step([grp], n, None, t, oracle.Config(eps=1e-8, iteration=s))
    p, _, _ = _torch_adam_on_sequence(theta0, gs, 1e-3, (0.9, 0.999), 1e-8)
    np.testing.assert_allclose(grp.param, p, rtol=1e-12, atol=1e-14)
    assert (t == 6).all()


def test_constant_gradient_closed_form():
    """From zero state with constant g: m_hat = g and v_hat = g^2 exactly, so
    every step moves theta by lr * g / (|g| + eps)."""
    n, dim, lr, eps, k = 4, 3, 0.01, 1e-8, 40
    g = np.array([[0.3, -2.0, 1e-3]] * n)
    grp = _one_group(n, dim, lr)
    t = np.zeros(n, np.int32)
    grp.grad[:] = g
    for s in range(k):
        oracle.adamw_gs_step([grp], n, np.ones(n, np.uint8), t, oracle.Config(eps=eps, iteration=s))
    np.testing.assert_allclose(grp.param, -k * lr * g / (np.abs(g) + eps), rtol=1e-12)


def test_alternating_gradient_closed_form():
    """g_k = (-1)^k g: m_k = (1-b1) g sum_j (-b1)^j (1 - ...) and v_hat = g^2."""
    b1, b2, g0, k = 0.9, 0.999, 0.5, 9
    grp = _one_group(1, 1, 1e-3)
    t = np.zeros(1, np.int32)
    for s in range(k):
        grp.grad[:] = g0 * (-1) ** s
        oracle.adamw_gs_step([grp], 1, np.ones(1, np.uint8), t, oracle.Config(iteration=s))
    # m_k = sum_{j=0}^{k-1} b1^j (1-b1) g_{k-1-j}
    expect_m = sum((b1 ** j) * (1 - b1) * g0 * (-1) ** (k - 1 - j) for j in range(k))
    assert grp.m[0, 0] == pytest.approx(expect_m, rel=1e-13)
    assert grp.v[0, 0] / (1 - b2 ** k) == pytest.approx(g0 * g0, rel=1e-12)


def test_first_step_hand_computation_with_dar():
    """Hand computation (opacity group, tau = 0, g = 0.002, first step):
    m = 2e-4, v = 4e-9, b1 = 0.1, b2 = 1e-3 -> m_hat = 0.002, sqrt(v_hat) = 0.002;
    sigma(0)(1-sigma(0)) = 0.25; DAR term = 1e-3 * 0.25 / 1e5 / 0.002 = 1.25e-6;
    tau = -0.05 * (1 + 1.25e-6) = -0.0500000625; eps = 1e-15 scales both terms
    by 0.002 / (0.002 + 1e-15) = 1 - 5e-13, i.e. +2.5e-14: -0.050000062499975."""
    grp = _one_group(1, 1, 0.05, dar_kind=oracle.DAR_OPACITY_SIGMOID, lam=1e-3, clip=10.0)
    grp.grad[:] = 0.002
    t = np.zeros(1, np.int32)
    oracle.adamw_gs_step([grp], 1, np.ones(1, np.uint8), t, oracle.Config(reg_norm=1e5, eps=1e-15))
    assert grp.m[0, 0] == pytest.approx(2e-4, rel=1e-13)
    assert grp.v[0, 0] == pytest.approx(4e-9, rel=1e-13)
    assert grp.param[0, 0] == pytest.approx(-0.050000062499975, rel=0, abs=2e-16)


def test_logscale_dar_uses_pre_update_theta_hand_computation():
    """Log-scale group, kappa = 1, g = 0.1, lambda = 4e4 (large, so the DAR
    term matters), N_I' = 1e5, first step: sqrt(v_hat) = 0.1, Adam part = 1,
    DAR = 0.4 * e / 0.1 = 10.87312731383618 (below C = 100), taken at the
    pre-update kappa = 1: kappa = 1 - 0.01 * (1 + 10.87312731383618)."""
    grp = _one_group(1, 1, 0.01, dar_kind=oracle.DAR_LOGSCALE_EXP, lam=4e4, clip=100.0, theta=[1.0])
    grp.grad[:] = 0.1
    t = np.zeros(1, np.int32)
    oracle.adamw_gs_step([grp], 1, np.ones(1, np.uint8), t, oracle.Config(reg_norm=1e5, eps=1e-15))
    # 4e4 * 2.718281828459045 / 1e5 / 0.1 = 10.87312731383618
    assert grp.param[0, 0] == pytest.approx(1.0 - 0.01 * (1.0 + 10.87312731383618), rel=0, abs=1e-13)


def test_dar_clamps_at_c_when_gradient_is_zero():
    """Visible primitive with g = 0 and zero state: d = eps, Adam part = 0, the
    DAR term lambda R'/N_I'/eps exceeds C, so theta <- theta - lr * C exactly."""
    for kind, theta in ((oracle.DAR_OPACITY_SIGMOID, 0.3), (oracle.DAR_LOGSCALE_EXP, -2.0)):
        grp = _one_group(1, 1, 0.05, dar_kind=kind, lam=1e-3, clip=10.0, theta=[theta])
        t = np.zeros(1, np.int32)
        oracle.adamw_gs_step([grp], 1, np.ones(1, np.uint8), t, oracle.Config(reg_norm=1e5, eps=1e-15))
        assert grp.param[0, 0] == theta - 0.05 * 10.0


def test_dar_off_equals_sparse_adam_and_dar_never_increases():
    rng = np.random.default_rng(5)
    n, steps = 64, 12
    th0 = rng.standard_normal((n, 1))
    a = _one_group(n, 1, 0.05, dar_kind=oracle.DAR_OPACITY_SIGMOID, lam=0.0, clip=10.0, theta=th0)
    b = _one_group(n, 1, 0.05, dar_kind=oracle.DAR_NONE, theta=th0)
    c = _one_group(n, 1, 0.05, dar_kind=oracle.DAR_OPACITY_SIGMOID, lam=1e-1, clip=10.0, theta=th0)
    ta, tb, tc = (np.zeros(n, np.int32) for _ in range(3))
    for s in range(steps):
        mask = (rng.random(n) < 0.5).astype(np.uint8)
        g = rng.standard_normal((n, 1)) * 1e-3
        for grp, t in ((a, ta), (b, tb), (c, tc)):
            grp.grad[:] = g
            oracle.adamw_gs_step([grp], n, mask, t, oracle.Config(iteration=s))
        np.testing.assert_array_equal(a.param, b.param)
    # Adam parts are identical (moments see only g), so DAR only pushes down.
    assert (c.param <= a.param).all()


def test_constant_penalty_variants_hand_values():
    """AdamW-style decoupling (Sec. "AdamW Style Decoupling"): with g = 0 the
    update is lr * lambda R' (unclipped) or lr * min(lambda R', C)."""
    # sigma(0)(1 - sigma(0)) = 0.25; lr = 0.1; C = 0.4
    for mode, lam, expect in ((oracle.REG_CONSTANT, 2.0, -0.05),
                              (oracle.REG_CONSTANT_CLIPPED, 2.0, -0.04),
                              (oracle.REG_CONSTANT_CLIPPED, 0.1, -0.0025)):
        grp = _one_group(1, 1, 0.1, dar_kind=oracle.DAR_OPACITY_SIGMOID, lam=lam, clip=0.4,
                         theta=[0.0], reg_mode=mode)
        grp.param[:] = 0.0
        t = np.zeros(1, np.int32)
        oracle.adamw_gs_step([grp], 1, np.ones(1, np.uint8), t, oracle.Config())
        assert grp.param[0, 0] == pytest.approx(expect, abs=1e-15)


# ---------------------------------------------------------------- RSR
def test_rsr_sampling_fraction_and_untouched_rows():
    n, p = 200_000, 0.05
    sampled = np.array([oracle.rsr_sampled(7, 300, i, p) for i in range(0, n, 20)])
    k, m = sampled.sum(), sampled.size
    assert abs(k - p * m) < 5 * math.sqrt(m * p * (1 - p))
    # state-level check: only sampled rows change, and only m, v by alpha
    n = 4000
    rng = np.random.default_rng(1)
    grp = _one_group(n, 3, 0.1, theta=rng.standard_normal((n, 3)))
    grp.m[:] = rng.standard_normal((n, 3))
    grp.v[:] = rng.random((n, 3))
    th0, m0, v0 = grp.param.copy(), grp.m.copy(), grp.v.copy()
    t = rng.integers(0, 50, n).astype(np.int32)
    t0 = t.copy()
    cfg = oracle.Config(seed=7, iteration=300, rsr_enable=True, rsr_alpha1=0.2, rsr_alpha2=0.04, rsr_ratio=p)
    oracle.adamw_gs_step([grp], n, np.zeros(n, np.uint8), t, cfg)
    s = np.array([oracle.rsr_sampled(7, 300, i, p) for i in range(n)])
    np.testing.assert_array_equal(t, t0)
    np.testing.assert_array_equal(grp.param, th0)
    np.testing.assert_array_equal(grp.m[~s], m0[~s])
    np.testing.assert_array_equal(grp.v[~s], v0[~s])
    np.testing.assert_array_equal(grp.m[s], 0.2 * m0[s])
    np.testing.assert_array_equal(grp.v[s], 0.04 * v0[s])


def test_rsr_ratio_preserving_rescale():
    """alpha2 = alpha1^2 keeps m_hat / sqrt(v_hat) unchanged right after the
    rescale (Sec. "Hyperparameter Selection", scaling in RSR)."""
    grp = _one_group(1, 2, 0.1)
    grp.m[:] = [[3e-4, -1e-3]]
    grp.v[:] = [[2e-7, 5e-6]]
    r0 = grp.m / np.sqrt(grp.v)
    t = np.array([5], np.int32)
    oracle.adamw_gs_step([grp], 1, np.zeros(1, np.uint8), t,
                         oracle.Config(rsr_enable=True, rsr_alpha1=0.3, rsr_alpha2=0.09, rsr_ratio=1.0))
    np.testing.assert_allclose(grp.m / np.sqrt(grp.v), r0, rtol=1e-14)


def test_rsr_zero_alpha_then_step_closed_form():
    """alpha = 0 zeroes the state (a fresh primitive) but keeps t, so the next
    visible step is u = ((1-b1) g / (1-b1^t)) / (sqrt((1-b2) g^2 / (1-b2^t)) + eps)."""
    b1, b2, eps, lr, g = 0.9, 0.999, 1e-15, 0.1, 0.004
    grp = _one_group(1, 1, lr)
    grp.m[:] = 5.0
    grp.v[:] = 7.0
    t = np.array([9], np.int32)
    grp.grad[:] = g
    oracle.adamw_gs_step([grp], 1, np.ones(1, np.uint8), t,
                         oracle.Config(rsr_enable=True, rsr_alpha1=0.0, rsr_alpha2=0.0, rsr_ratio=1.0, eps=eps))
    T = 10
    u = ((1 - b1) * g / (1 - b1 ** T)) / (math.sqrt((1 - b2) * g * g / (1 - b2 ** T)) + eps)
    assert grp.param[0, 0] == pytest.approx(-lr * u, rel=1e-13)
    assert t[0] == 10


def test_step_counts_equal_visible_counts():
    rng = np.random.default_rng(9)
    n, steps = 300, 30
    grp = _one_group(n, 4, 1e-3)
    t = np.zeros(n, np.int32)
    total = np.zeros(n, np.int32)
    for s in range(steps):
        mask = (rng.random(n) < 0.3).astype(np.uint8)
        total += mask
        grp.grad[:] = rng.standard_normal((n, 4))
        oracle.adamw_gs_step([grp], n, mask, t, oracle.Config(iteration=s, rsr_enable=(s % 7 == 0),
                                                               rsr_ratio=0.5))
    np.testing.assert_array_equal(t, total)


# ---------------------------------------------------------------- visibility
def _axis_camera(z_far=float("inf")):
    view = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 15.0]], np.float32)
    f = 500.0 / math.tan(math.radians(30.0))
    return oracle.Camera(view, f, f, 500.0, 500.0, 1000, 1000, 0.2, z_far)


def test_visibility_special_points():
    cam = _axis_camera()
    pts = np.array([[0, 0, 0],          # on the axis, in front: visible
                    [0, 0, -15.1],      # behind the camera: invisible
                    [0, 0, -14.85],     # in front of the near plane (z = 0.15): invisible
                    [100, 0, 0],        # far outside the frustum
                    [np.nan, 0, 0]], np.float32)
    np.testing.assert_array_equal(oracle.visibility(pts, cam), [1, 0, 0, 0, 0])
    # radius pushes a point just outside the left edge back in, r_min culls small ones
    x = -(15.0 * math.tan(math.radians(30.0))) - 0.05
    p = np.array([[x, 0, 0]], np.float32)
    assert oracle.visibility(p, cam)[0] == 0
    assert oracle.visibility(p, cam, np.array([0.1], np.float32))[0] == 1
    cam.r_min = 10.0
    assert oracle.visibility(p, cam, np.array([0.1], np.float32))[0] == 0


def test_visibility_exact_edges_and_anisotropic_focal():
    """Hand-placed points: with t = (0, 0, 15), fx = 500, cx = 500, W = 1000,
    the mean (10, 0, -5) sits at depth 10 and projects to u = 500*10/10 + 500 =
    1000 = W exactly (inside: the edge counts), (-10, 0, -5) to u = 0 exactly;
    nudged outward they leave the image.  With fy = 1000 != fx, (0, 6, -5)
    projects to v = 1000*6/10 + 500 = 1100 > H (outside) although fx would
    put it at 800 (inside); (6, 0, -5) lands at u = 800 (inside)."""
    view = np.array([[1, 0, 0, 0], [0, 1, 0, 0], [0, 0, 1, 15.0]], np.float32)
    cam = oracle.Camera(view, 500.0, 1000.0, 500.0, 500.0, 1000, 1000, 0.2, float("inf"))
    pts = np.array([[10, 0, -5], [-10, 0, -5], [10.001, 0, -5], [-10.001, 0, -5],
                    [0, 6, -5], [6, 0, -5], [0, -6, -5], [0, 5, -5]], np.float32)
    np.testing.assert_array_equal(oracle.visibility(pts, cam), [1, 1, 0, 0, 0, 1, 0, 1])


def test_visibility_axis_camera_closed_form_fraction():
    """Axis camera at distance 15, 60 deg square FOV, means ~ U[-10,10]^3, no
    far plane: P(visible) = (1/20)[(zc^3 - 125)/900 + (25 - zc)], zc = 10 sqrt 3."""
    zc = 10 * math.sqrt(3)
    expect = ((zc ** 3 - 125) / 900 + (25 - zc)) / 20
    assert expect == pytest.approx(0.6657, abs=1e-4)
    n = 400_000
    mu = synth.rng(11).uniform(-10, 10, (n, 3)).astype(np.float32)
    frac = oracle.visibility(mu, _axis_camera()).mean()
    assert abs(frac - expect) < 5 * math.sqrt(expect * (1 - expect) / n)


def test_visibility_mirror_symmetry_and_f64_agreement():
    cam = _axis_camera(z_far=20.0)
    mu = synth.rng(12).uniform(-10, 10, (50_000, 3)).astype(np.float32)
    mirror = mu * np.array([-1, -1, 1], np.float32)
    # cx = cy = W/2, so a point and its mirror image through the axis project
    # symmetrically about the principal point
    np.testing.assert_array_equal(oracle.visibility(mu, cam), oracle.visibility(mirror, cam))
    m32, m64 = oracle.visibility(mu, cam), oracle.visibility_f64(mu, cam)
    assert (m32 != m64).sum() <= 2      # flips only at the boundary


def test_visibility_two_opposite_views_union_closed_form():
    """The axis camera and its mirror (at z = +15 looking down -z), no far
    plane, means ~ U[-10,10]^3: a point is in the union iff
    |x|, |y| <= (15 + |z|) / sqrt 3, so with a = 10 sqrt 3 - 15,
    P = (1/10)[((10 sqrt 3)^3 - 15^3)/900 + (10 - a)] = 0.9703."""
    a = 10 * math.sqrt(3) - 15
    expect = (((10 * math.sqrt(3)) ** 3 - 15 ** 3) / 900 + (10 - a)) / 10
    assert expect == pytest.approx(0.9703, abs=1e-4)
    front = _axis_camera()
    f = 500.0 / math.tan(math.radians(30.0))
    back = oracle.Camera(np.array([[1, 0, 0, 0], [0, -1, 0, 0], [0, 0, -1, 15.0]], np.float32), f, f, 500.0, 500.0,
                         1000, 1000, 0.2, float("inf"))
    n = 400_000
    mu = synth.rng(15).uniform(-10, 10, (n, 3)).astype(np.float32)
    mask, bits = oracle.visibility_multi(mu, [front, back])
    assert abs(mask.mean() - expect) < 5 * math.sqrt(expect * (1 - expect) / n)
    # each bit is that view's own mask, in list order
    np.testing.assert_array_equal(bits & 1, oracle.visibility(mu, front))
    np.testing.assert_array_equal((bits >> 1) & 1, oracle.visibility(mu, back))
    np.testing.assert_array_equal(mask, (bits != 0).astype(np.uint8))


def test_visibility_multi_bit_order_and_rig():
    """Bits follow the camera list (a reversed list reverses them); the rig's
    200 views all see the origin, and a far point is seen by none."""
    cams = [oracle.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far)
            for c in synth.camera_rig()]
    mu = synth.rng(16).uniform(-10, 10, (3000, 3)).astype(np.float32)
    sub = cams[:32:3]
    _, b = oracle.visibility_multi(mu, sub)
    _, r = oracle.visibility_multi(mu, sub[::-1])
    k = len(sub)
    rev = np.zeros_like(b)
    for v in range(k):
        rev |= ((b >> v) & 1) << (k - 1 - v)
    np.testing.assert_array_equal(r, rev)
    pts = np.array([[0, 0, 0], [1e6, 0, 0]], np.float32)
    for start in range(0, 200, 32):
        m, bb = oracle.visibility_multi(pts, cams[start:start + 32])
        width = len(cams[start:start + 32])
        assert bb[0] == (1 << width) - 1 and bb[1] == 0
        assert m.tolist() == [1, 0]


def test_compaction_is_sorted_nonzero():
    mask = (synth.rng(13).random(10_001) < 0.27).astype(np.uint8)
    np.testing.assert_array_equal(oracle.compact(mask), np.flatnonzero(mask))


def test_rig_visible_fraction_in_band():
    """The synthetic rig (radius 15, 60 deg, z_far = 17.5) lands inside the
    5-40 % visible band of the 3M-primitive workload."""
    cams = synth.camera_rig()
    mu = synth.rng(14).uniform(-10, 10, (100_000, 3)).astype(np.float32)
    for c in cams[::40]:
        cam = oracle.Camera(c.view, c.fx, c.fy, c.cx, c.cy, c.width, c.height, c.z_near, c.z_far)
        assert 0.05 < oracle.visibility(mu, cam).mean() < 0.40


# ---------------------------------------------------------------- relocation
def test_select_smallest_matches_stable_argsort():
    rng = np.random.default_rng(2)
    key = rng.integers(0, 20, 5000).astype(np.float32)        # many ties
    for k in (0, 1, 50, 777, 5000):
        expect = np.sort(np.argsort(key, kind="stable")[:k])
        np.testing.assert_array_equal(oracle.select_smallest(key, k), expect)


def test_reset_state_zeroes_selected_rows():
    grp = _one_group(10, 2, 0.1)
    grp.m[:] = 1.0
    grp.v[:] = 2.0
    t = np.arange(10, dtype=np.int32)
    oracle.reset_state([grp], np.array([2, 5], np.int64), t, True)
    assert (grp.m[[2, 5]] == 0).all() and (grp.v[[2, 5]] == 0).all()
    assert (grp.m[[0, 1, 3, 4, 6, 7, 8, 9]] == 1).all()
    assert t[2] == 0 and t[5] == 0 and t[3] == 3


# ---------------------------------------------------------------- bf16 storage
def test_bf16_rne_matches_torch():
    x = np.concatenate([synth.rng(15).standard_normal(20000).astype(np.float32) * 1e-3,
                        np.array([0.0, -0.0, 1.0, 65504.0, 3.0e38], np.float32)])
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().astype(np.uint16)
    got = np.array([oracle.bf16_rne(float(v)) for v in x], np.uint16)
    np.testing.assert_array_equal(got, ref)


def test_bf16_sr_counts_exact():
    """Over all 2^16 random words, SR rounds up exactly (low 16 bits) times:
    the rounding is unbiased by construction."""
    for xv in (1.2345678e-3, -7.77e-6, 3.0):
        x = np.float32(xv)
        bits = int(x.view(np.uint32))
        low = bits & 0xFFFF
        ups = 0
        for r in range(0, 65536, 1):
            out = oracle.bf16_sr(float(x), r)
            assert out in ((bits >> 16), (bits >> 16) + 1)
            ups += out == (bits >> 16) + 1
        assert ups == low


# ---------------------------------------------------------------- position noise
def test_noise_gamma_is_standard_normal():
    """Box-Muller on the counter draws: each component N(0, 1), uncorrelated
    (KS test against the normal CDF, moments within 5 standard errors)."""
    from scipy import stats
    n = 60_000
    g = np.array([oracle.noise_gamma(3, 17, i) for i in range(n)])
    assert np.abs(g.mean(axis=0)).max() < 5 / math.sqrt(n)
    assert np.abs(g.var(axis=0) - 1).max() < 5 * math.sqrt(2 / n)
    c = np.corrcoef(g.T)
    assert np.abs(c[np.triu_indices(3, 1)]).max() < 5 / math.sqrt(n)
    for k in range(3):
        assert stats.kstest(g[:, k], "norm").pvalue > 1e-3


def test_noise_displacement_against_scipy_rotation():
    """eta_Ro * eta_mu * sigma(-k (sigma(tau) - t)) * R diag(e^{2 kappa}) R^T gamma,
    with R from scipy's quaternion rotation (scalar-last there)."""
    from scipy.spatial.transform import Rotation
    rng = np.random.default_rng(21)
    cfg = oracle.Config(noise_lr=5e5, noise_k=100.0, noise_t=0.005)
    for _ in range(50):
        q = rng.standard_normal(4) * 3.0               # not normalised on purpose
        kappa = rng.normal(-3.0, 1.0, 3)
        tau = rng.normal(-4.0, 2.0)
        gamma = rng.standard_normal(3)
        R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        sigma = R @ np.diag(np.exp(2 * kappa)) @ R.T
        o = 1 / (1 + np.exp(-tau))
        gate = 1 / (1 + np.exp(100.0 * (o - 0.005)))
        expect = 5e5 * 1.6e-4 * gate * (sigma @ gamma)
        np.testing.assert_allclose(oracle.noise_displacement(q, kappa, tau, 1.6e-4, cfg, gamma), expect,
                                   rtol=1e-10, atol=1e-300)


def test_noise_displacement_hand_cases():
    cfg = oracle.Config(noise_lr=2.0, noise_k=10.0, noise_t=0.5)
    tau = 0.0                                            # o = 0.5 = t: gate = 1/2
    g = np.array([1.0, -2.0, 0.5])
    kap = np.array([0.0, math.log(2.0), math.log(3.0)])  # S^2 = diag(1, 4, 9)
    # identity rotation: lr * eta_Ro * 1/2 * (1, -8, 4.5)
    np.testing.assert_allclose(oracle.noise_displacement([1, 0, 0, 0], kap, tau, 0.1, cfg, g),
                               0.1 * 2.0 * 0.5 * np.array([1.0, -8.0, 4.5]), rtol=1e-14)
    # 90 degrees about z: x and y scales swap -> S^2 seen as diag(4, 1, 9)
    h = math.sqrt(0.5)
    np.testing.assert_allclose(oracle.noise_displacement([h, 0, 0, h], kap, tau, 0.1, cfg, g),
                               0.1 * 2.0 * 0.5 * np.array([4.0, -2.0, 4.5]), rtol=1e-13, atol=1e-15)
    # a scaled quaternion is the same rotation
    np.testing.assert_allclose(oracle.noise_displacement([7 * h, 0, 0, 7 * h], kap, tau, 0.1, cfg, g),
                               oracle.noise_displacement([h, 0, 0, h], kap, tau, 0.1, cfg, g), rtol=1e-14)


def test_noise_in_step_moves_visible_means_only():
    n, spec = 500, synth.GROUPS_59
    rng = np.random.default_rng(22)
    base = []
    for name, dim, lr, dar in spec:
        base.append(_one_group(n, dim, lr, dar_kind=dar, lam=1e-3, clip=10.0, theta=rng.standard_normal((n, dim))))
        base[-1].grad[:] = 1e-3 * rng.standard_normal((n, dim))
    def copy(gs_):
        return [oracle.Group(g.param.copy(), g.grad.copy(), g.m.copy(), g.v.copy(), g.lr, g.dar_kind, g.dar_lambda,
                             g.dar_clip) for g in gs_]
    a, b = copy(base), copy(base)
    mask = (rng.random(n) < 0.5).astype(np.uint8)
    ta, tb = np.zeros(n, np.int32), np.zeros(n, np.int32)
    cfg_on = oracle.Config(seed=4, iteration=9, noise_enable=True, noise_groups=(0, 1, 2, 3), noise_lr=50.0)
    oracle.adamw_gs_step(a, n, mask, ta, cfg_on)
    oracle.adamw_gs_step(b, n, mask, tb, oracle.Config(seed=4, iteration=9))
    for k in range(1, 5):                                # other groups: identical
        np.testing.assert_array_equal(a[k].param, b[k].param)
    inv = mask == 0
    np.testing.assert_array_equal(a[0].param[inv], base[0].param[inv])
    for i in np.flatnonzero(mask)[:40]:
        d = oracle.noise_displacement(base[2].param[i], base[1].param[i], base[3].param[i, 0], spec[0][2], cfg_on,
                                      oracle.noise_gamma(4, 9, int(i)))
        np.testing.assert_allclose(a[0].param[i], b[0].param[i] - d, rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------- AIU
def _aiu_state(n, spec, seed, lam=0.0, t_max=30):
    """Groups with moments and step counts in use (t = 0 on some rows)."""
    rng = np.random.default_rng(seed)
    gr = []
    for name, dim, lr, dar in spec:
        g = _one_group(n, dim, lr, dar_kind=dar if lam else 0, lam=lam, clip=10.0, theta=rng.standard_normal((n, dim)))
        g.m[:] = 1e-3 * rng.standard_normal((n, dim))
        g.v[:] = 1e-6 * rng.random((n, dim)) + 1e-8
        g.grad[:] = 1e-3 * rng.standard_normal((n, dim))
        gr.append(g)
    t = rng.integers(0, t_max, n).astype(np.int32)
    return gr, t


def _copy_groups(gs_):
    return [oracle.Group(g.param.copy(), g.grad.copy(), g.m.copy(), g.v.copy(), g.lr, g.dar_kind, g.dar_lambda,
                         g.dar_clip, g.reg_mode) for g in gs_]


def test_aiu_repeats_the_last_visible_update():
    """A primitive visible at one step and AIU-sampled (Pro = 1, eta = 1) at
    the next, invisible one, moves again by exactly the update it just made:
    AIU takes the Adam direction of the unchanged moments with the same step
    count.  eta_AIU scales it; moments and t do not change."""
    n, spec = 300, synth.GROUPS_59
    g, t = _aiu_state(n, spec, 31)
    t[:] = np.maximum(t, 1)
    ones = np.ones(n, np.uint8)
    zeros = np.zeros(n, np.uint8)
    for scale in (1.0, 0.25):
        a, ta = _copy_groups(g), t.copy()
        oracle.adamw_gs_step(a, n, ones, ta, oracle.Config(seed=1, iteration=5))
        delta = [x.param - y.param for x, y in zip(a, g)]
        mid = _copy_groups(a)
        tb = ta.copy()
        oracle.adamw_gs_step(a, n, zeros, tb, oracle.Config(seed=1, iteration=6, aiu_enable=True, aiu_ratio=1.0,
                                                            aiu_scale=scale))
        np.testing.assert_array_equal(tb, ta)
        for x, y, d in zip(a, mid, delta):
            np.testing.assert_array_equal(x.m, y.m)
            np.testing.assert_array_equal(x.v, y.v)
            np.testing.assert_allclose(x.param - y.param, scale * d, rtol=1e-9, atol=1e-15)


def test_aiu_carries_no_regulariser_term():
    """With DAR on, the visible update holds the DAR term but the AIU update
    is the Adam direction alone (the step without DAR)."""
    n, spec = 200, synth.GROUPS_59
    g, t = _aiu_state(n, spec, 32, lam=50.0)
    t[:] = np.maximum(t, 1)
    plain = _copy_groups(g)
    for x in plain:
        x.dar_kind, x.dar_lambda = 0, 0.0
    ones = np.ones(n, np.uint8)
    a, ta = _copy_groups(g), t.copy()
    b, tb = _copy_groups(plain), t.copy()
    oracle.adamw_gs_step(a, n, ones, ta, oracle.Config(seed=2, iteration=1))
    oracle.adamw_gs_step(b, n, ones, tb, oracle.Config(seed=2, iteration=1))
    d_plain = [y.param - x.param for x, y in zip(plain, b)]
    assert any(np.abs((y.param - x.param) - d).max() > 1e-6 for x, y, d in zip(g, a, d_plain))   # DAR acted
    mid = _copy_groups(a)
    oracle.adamw_gs_step(a, n, np.zeros(n, np.uint8), ta,
                         oracle.Config(seed=2, iteration=2, aiu_enable=True, aiu_ratio=1.0, aiu_scale=1.0))
    for x, y, d in zip(a, mid, d_plain):
        np.testing.assert_allclose(x.param - y.param, d, rtol=1e-9, atol=1e-15)


def test_aiu_samples_invisible_rows_with_moments_only():
    """Only invisible, sampled rows with t > 0 move; the sampled fraction is
    Pro_AIU within binomial bounds; visible rows are those of the step
    without AIU, bit for bit."""
    n, spec, p = 20_000, [("a", 2, 0.1, 0), ("b", 1, 0.2, 0)], 0.3
    g, t = _aiu_state(n, spec, 33)
    mask = (np.random.default_rng(34).random(n) < 0.4).astype(np.uint8)
    a, ta = _copy_groups(g), t.copy()
    b, tb = _copy_groups(g), t.copy()
    cfg = oracle.Config(seed=9, iteration=3, aiu_enable=True, aiu_ratio=p, aiu_scale=0.5)
    oracle.adamw_gs_step(a, n, mask, ta, cfg)
    oracle.adamw_gs_step(b, n, mask, tb, oracle.Config(seed=9, iteration=3))
    np.testing.assert_array_equal(ta, tb)
    vis = mask == 1
    moved = np.any(a[0].param != b[0].param, axis=1)
    assert not moved[vis].any()
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x.param[vis], y.param[vis])
        np.testing.assert_array_equal(x.m, y.m)
        np.testing.assert_array_equal(x.v, y.v)
    sampled = oracle.aiu_sample_mask(9, 3, n, p)
    np.testing.assert_array_equal(moved, ~vis & sampled & (t > 0))
    k, m = int(sampled.sum()), n
    assert abs(k - p * m) < 5 * math.sqrt(m * p * (1 - p))
    # an independent stream: the Re-State sample of the same iteration differs
    assert (sampled != oracle.rsr_sample_mask(9, 3, n, p)).sum() > 0.2 * n


def test_aiu_reads_the_rescaled_moments():
    """AIU and Re-State in one iteration: the extra update uses the moments
    after the rescale, so with alpha1 = 0.5, alpha2 = 0.04 (not alpha1^2) the
    direction grows by alpha1 / sqrt(alpha2) = 2.5."""
    n, spec = 100, [("a", 3, 0.1, 0)]
    g, t = _aiu_state(n, spec, 35)
    t[:] = np.maximum(t, 1)
    zeros = np.zeros(n, np.uint8)
    a, b = _copy_groups(g), _copy_groups(g)
    oracle.adamw_gs_step(a, n, zeros, t.copy(), oracle.Config(seed=3, iteration=4, aiu_enable=True, aiu_ratio=1.0,
                                                               aiu_scale=1.0))
    oracle.adamw_gs_step(b, n, zeros, t.copy(), oracle.Config(seed=3, iteration=4, aiu_enable=True, aiu_ratio=1.0,
                                                               aiu_scale=1.0, rsr_enable=True, rsr_ratio=1.0,
                                                               rsr_alpha1=0.5, rsr_alpha2=0.04))
    np.testing.assert_allclose(b[0].param - g[0].param, 2.5 * (a[0].param - g[0].param), rtol=1e-9, atol=1e-15)
    np.testing.assert_allclose(b[0].m, 0.5 * g[0].m, rtol=1e-15)


# ---------------------------------------------------------------- primitive-set mutation
def test_prune_is_boolean_row_selection():
    """Pruning keeps the rows with keep != 0 in order: numpy's boolean
    indexing of every array, including the step counts."""
    rng = np.random.default_rng(40)
    n, spec = 1000, synth.GROUPS_59
    g, t = _aiu_state(n, spec, 41)
    for p in (0.0, 0.3, 1.0):
        keep = (rng.random(n) < p).astype(np.uint8)
        d, td = oracle.prune(g, keep, t)
        np.testing.assert_array_equal(td, t[keep == 1])
        for x, y in zip(d, g):
            np.testing.assert_array_equal(x.param, y.param[keep == 1])
            np.testing.assert_array_equal(x.m, y.m[keep == 1])
            np.testing.assert_array_equal(x.v, y.v[keep == 1])


def test_prune_commutes_with_the_step():
    """The optimizer state travels with its primitive: pruning then stepping
    the kept rows gives what stepping then pruning gives (no Re-State, whose
    draws are keyed by the scene index)."""
    rng = np.random.default_rng(42)
    n, spec = 500, synth.GROUPS_59
    g, t = _aiu_state(n, spec, 43, lam=1e-3)
    keep = (rng.random(n) < 0.6).astype(np.uint8)
    vis = (rng.random(n) < 0.5).astype(np.uint8)
    a, ta = _copy_groups(g), t.copy()
    oracle.adamw_gs_step(a, n, vis, ta, oracle.Config(iteration=3))
    a, ta = oracle.prune(a, keep, ta)
    b, tb = oracle.prune(_copy_groups(g), keep, t.copy())
    for x, y in zip(b, g):                     # gradients belong to the iteration: the caller's
        x.grad = np.ascontiguousarray(y.grad[keep == 1])
    kv = np.ascontiguousarray(vis[keep == 1])
    oracle.adamw_gs_step(b, b[0].param.shape[0], kv, tb, oracle.Config(iteration=3))
    np.testing.assert_array_equal(ta, tb)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x.param, y.param)
        np.testing.assert_array_equal(x.m, y.m)


def test_append_gives_clones_with_a_fresh_state():
    """New rows copy their source's attributes with m = v = 0 and t = 0 (RSR
    with alpha = 0, plus a new step count); their first visible step is then
    Adam's first step, theta - lr g / (|g| + eps) (Kingma & Ba); old rows
    do not change."""
    n, k, spec = 400, 150, synth.GROUPS_59
    g, t = _aiu_state(n + k, spec, 44)
    rng = np.random.default_rng(45)
    src = rng.integers(0, n, k).astype(np.int64)
    before = _copy_groups(g)
    t0 = t.copy()
    oracle.append(g, n, src, t)
    np.testing.assert_array_equal(t[:n], t0[:n])
    assert (t[n:] == 0).all()
    for x, y in zip(g, before):
        np.testing.assert_array_equal(x.param[:n], y.param[:n])
        np.testing.assert_array_equal(x.m[:n], y.m[:n])
        np.testing.assert_array_equal(x.param[n:], y.param[src])
        assert (x.m[n:] == 0).all() and (x.v[n:] == 0).all()
    vis = np.zeros(n + k, np.uint8)
    vis[n:] = 1
    new = _copy_groups(g)
    oracle.adamw_gs_step(g, n + k, vis, t, oracle.Config(iteration=1, eps=1e-15))
    for x, y in zip(g, new):
        gr = y.grad[n:]
        np.testing.assert_allclose(x.param[n:], y.param[n:] - y.lr * gr / (np.abs(gr) + 1e-15), rtol=1e-12,
                                   atol=1e-15)
    assert (t[n:] == 1).all()


def test_row_subset_step_equals_the_full_step():
    """The oracle's step on a subset of a scene's rows (each row keyed by its
    scene index, as the sampled-row GPU checks use it) must reproduce the
    pinned full-scene step on those rows exactly: Re-State, AIU and the
    position-noise draws all follow the scene index, not the row's place in
    the subset."""
    n, spec = 600, synth.GROUPS_59
    rng = np.random.default_rng(23)
    base = []
    for name, dim, lr, dar in spec:
        g = _one_group(n, dim, lr, dar_kind=dar, lam=1e-3, clip=10.0, theta=rng.standard_normal((n, dim)))
        g.grad[:] = 1e-3 * rng.standard_normal((n, dim))
        g.m[:] = 1e-4 * rng.standard_normal((n, dim))
        g.v[:] = 1e-6 * rng.random((n, dim)) + 1e-9
        base.append(g)
    t0 = rng.integers(0, 6, n).astype(np.int32)
    mask = (rng.random(n) < 0.4).astype(np.uint8)
    cfg = oracle.Config(seed=3, iteration=7, rsr_enable=True, rsr_ratio=0.3, aiu_enable=True, aiu_ratio=0.3,
                        aiu_scale=0.5, noise_enable=True, noise_groups=(0, 1, 2, 3), noise_lr=20.0)
    full = [oracle.Group(g.param.copy(), g.grad.copy(), g.m.copy(), g.v.copy(), g.lr, g.dar_kind, g.dar_lambda,
                         g.dar_clip) for g in base]
    t_full = t0.copy()
    oracle.adamw_gs_step(full, n, mask, t_full, cfg)
    rows = np.sort(rng.choice(n, 151, replace=False)).astype(np.int64)
    sub = [oracle.Group(g.param[rows].copy(), g.grad[rows].copy(), g.m[rows].copy(), g.v[rows].copy(), g.lr,
                        g.dar_kind, g.dar_lambda, g.dar_clip) for g in base]
    t_sub = t0[rows].copy()
    oracle.adamw_gs_step(sub, len(rows), mask[rows].copy(), t_sub, cfg, ids=rows)
    np.testing.assert_array_equal(t_sub, t_full[rows])
    for S, F in zip(sub, full):
        np.testing.assert_array_equal(S.param, F.param[rows])
        np.testing.assert_array_equal(S.m, F.m[rows])
        np.testing.assert_array_equal(S.v, F.v[rows])
    # the case is not vacuous: visible, Re-State-only and AIU-only rows are all in the subset
    inv = mask[rows] == 0
    moved_inv = np.any(sub[4].param[inv] != base[4].param[rows][inv], axis=1)
    rescaled_inv = np.any(sub[4].m[inv] != base[4].m[rows][inv], axis=1)
    assert moved_inv.any() and rescaled_inv.any() and (mask[rows] == 1).any()
