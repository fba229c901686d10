"""Pins of the densification reference against facts fixed independently of it."""
import math

import numpy as np
import pytest
import torch

from oracle import densify, focus, spec32

CFG = dict(grad_threshold=5e-5, min_alpha=0.02, max_radius=64.0, split_scale=2.0, split_factor=1.6)


def _one(mu, l, q, alpha):
    p = np.zeros((11, 1), np.float32)
    p[0:3, 0], p[3:6, 0], p[6:10, 0], p[10, 0] = mu, l, q, alpha
    return p


def _slice(z, sigma_z=1.0, W=64, H=48, dx=1.0, dy=1.0):
    return dict(z=z, sigma_z=sigma_z, x0=0.0, y0=0.0, dx=dx, dy=dy, width=W, height=H)


def test_mean_gradient_norm_equals_lateral_parameter_gradient():
    # The projected mean depends on mu_x, mu_y with unit slope and nothing else
    # in the image depends on them, so |dL/dmu_2d| is the norm of the full
    # parameter gradient's first two rows (an independent autograd route).
    rng = np.random.default_rng(3)
    p = np.zeros((11, 5), np.float32)
    p[0] = rng.uniform(16, 48, 5)
    p[1] = rng.uniform(12, 36, 5)
    p[2] = rng.uniform(-1.5, 1.5, 5)
    p[3:6] = np.log(rng.uniform(1.0, 4.0, (3, 5)))
    p[6:10] = rng.normal(size=(4, 5))
    p[10] = rng.uniform(0.2, 1.0, 5)
    dx = 0.75
    sl = _slice(0.3, 1.5, dx=dx, dy=dx)
    w = rng.normal(size=(48, 64))
    gn, cnt, _ = densify.stats(p, [sl], [w])
    g = focus.grad(p, [sl], [w])
    assert (cnt == 1).all()
    np.testing.assert_allclose(gn, dx * np.hypot(g[0], g[1]), rtol=1e-10, atol=1e-14)


def test_count_is_the_axial_cut_closed_form():
    # Isotropic s: a slice at depth z holds the Gaussian iff
    # (mu_z - z)^2 / (sigma_z^2 + s^2) <= 2 ln 255 (and it is in view).
    s, sz, muz = 1.5, 2.0, 10.0
    p = _one((32, 24, muz), [math.log(s)] * 3, (1, 0, 0, 0), 0.8)
    zs = np.linspace(0.0, 20.0, 41)
    slices = [_slice(float(z), sz) for z in zs]
    _, cnt, _ = densify.stats(p, slices, [np.ones((48, 64))] * len(zs))
    expect = sum((muz - z) ** 2 / (sz * sz + s * s) <= 2 * math.log(255) for z in zs)
    assert int(cnt[0]) == expect and 0 < expect < len(zs)


def test_radius_of_axis_aligned_gaussian():
    # Diagonal covariance: the in-plane marginal is diag(sx^2, sy^2) on every slice.
    sx, sy, sz = 2.0, 5.0, 1.0
    p = _one((32, 24, 0.0), [math.log(sx), math.log(sy), math.log(sz)], (1, 0, 0, 0), 0.8)
    _, _, rad = densify.stats(p, [_slice(0.2, dx=0.5, dy=2.0)], [np.ones((48, 64))])
    assert rad[0] == pytest.approx(spec32.BBOX_DEFAULT * max(sx / 0.5, sy / 2.0), rel=1e-6)  # float32 log-scales


def test_decisions_on_hand_made_cases():
    n = 7
    p = np.zeros((11, n), np.float32)
    p[6] = 1.0
    p[10] = 0.5
    p[3:6] = math.log(1.0)
    p[10, 0] = 0.01                       # 0: faint -> drop
    p[0, 1] = np.nan                      # 1: non-finite -> drop
    p[3:6, 4] = math.log(3.0)             # 4: large and hot -> split
    gn = np.array([1, 1, 0, 1e-3, 1e-3, 1e-3, 1e-3], np.float32)
    cnt = np.array([1, 1, 1, 10, 10, 0, 10], np.int32)
    rad = np.array([1, 1, 1, 1, 1, 1, 100], np.float32)   # 6: too wide -> drop
    act = densify.decide(p, gn, cnt, rad, CFG)
    D, K, Cl, S = densify.DROP, densify.KEEP, densify.CLONE, densify.SPLIT
    assert act.tolist() == [D, D, K, Cl, S, K, D]


def test_output_order_and_moments():
    n = 4
    rng = np.random.default_rng(0)
    p = np.zeros((11, n), np.float32)
    p[0:3] = rng.normal(size=(3, n))
    p[6] = 1.0
    p[10] = 0.5
    p[3:6, 2] = math.log(4.0)             # split
    m = rng.normal(size=(11, n))
    v = rng.uniform(size=(11, n))
    gn = np.array([0, 1, 1, 0], np.float32)
    cnt = np.array([1, 1, 1, 1], np.int32)
    rad = np.ones(n, np.float32)
    noise = rng.normal(size=(6, n)).astype(np.float32)
    po, mo, vo, act = densify.densify_prune(p, m, v, gn, cnt, rad, noise, CFG)
    assert act.tolist() == [densify.KEEP, densify.CLONE, densify.SPLIT, densify.KEEP]
    assert po.shape == (11, 6)
    np.testing.assert_array_equal(po[:, 0], p[:, 0])
    np.testing.assert_array_equal(po[:, 1], p[:, 1])
    np.testing.assert_array_equal(po[:, 2], p[:, 1])
    np.testing.assert_array_equal(po[:, 5], p[:, 3])
    np.testing.assert_array_equal(mo[:, [0, 1, 5]], m[:, [0, 1, 3]])
    assert not mo[:, 2:5].any() and not vo[:, 2:5].any()
    for c in (3, 4):
        np.testing.assert_allclose(po[3:6, c], np.log(4.0) - np.log(1.6), rtol=1e-7)
        np.testing.assert_array_equal(po[6:11, c], p[6:11, 2])


def test_split_children_sample_the_parent_covariance():
    # With standard normal noise, child offsets mu + R diag(s) n are distributed
    # N(0, Sigma) with Sigma the parent's covariance; a transposed rotation or a
    # scale applied on the wrong side gives another matrix.
    n = 6000
    q = np.array([0.8, 0.3, -0.4, 0.33])
    l = np.log([3.0, 1.0, 0.5])
    p = np.repeat(_one((0, 0, 0), l, q, 0.5), n, axis=1)
    rng = np.random.default_rng(11)
    noise = rng.normal(size=(6, n)).astype(np.float32)
    z = np.zeros((11, n))
    cfg = dict(CFG, split_scale=1.0)
    po, _, _, act = densify.densify_prune(p, z, z, np.ones(n, np.float32), np.ones(n, np.int32),
                                          np.ones(n, np.float32), noise, cfg)
    assert (act == densify.SPLIT).all()
    off = po[0:3]
    cov = off @ off.T / off.shape[1]
    _, Sigma, _ = focus.activate(torch.from_numpy(p[:, :1].astype(np.float64)))
    Sigma = Sigma[0].numpy()
    assert np.abs(cov - Sigma).max() <= 0.05 * np.abs(Sigma).max()
    # the transposed-rotation alternative is far away for this quaternion
    qn = q / np.linalg.norm(q)
    R = focus.quat_to_matrix(torch.from_numpy(qn)).numpy()
    S2 = np.diag(np.exp(2 * l))
    assert np.abs(R.T @ S2 @ R - Sigma).max() > 0.3 * np.abs(Sigma).max()
