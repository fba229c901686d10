"""Pins of the L1 + D-SSIM reference against closed forms and invariants."""
import numpy as np
import pytest
import torch

from oracle import ssim

F64 = torch.float64


def _t(a):
    return torch.as_tensor(np.asarray(a, np.float64))


def test_identical_images_give_one_everywhere():
    rng = np.random.default_rng(0)
    x = rng.uniform(0, 2, size=(2, 23, 37))
    s = ssim.ssim_map(_t(x), _t(x)).numpy()
    np.testing.assert_allclose(s, 1.0, rtol=0, atol=1e-13)


def test_constant_images_closed_form_in_the_interior():
    # constant a and b: local means a, b and zero variances wherever the window
    # lies inside the slice, so S = (2ab + C1) / (a^2 + b^2 + C1).
    a, b = 0.7, 0.2
    x = np.full((1, 30, 30), a)
    y = np.full((1, 30, 30), b)
    s = ssim.ssim_map(_t(x), _t(y)).numpy()[0]
    expect = (2 * a * b + 1e-4) / (a * a + b * b + 1e-4)
    np.testing.assert_allclose(s[5:-5, 5:-5], expect, rtol=1e-11)  # E[x^2] - mu^2 rounding
    # next to the border the zeros outside lower both means: not the closed form
    assert abs(s[0, 0] - expect) > 1e-3


def test_impulse_reaches_exactly_five_pixels():
    # an impulse against a zero target changes S only where the 11 x 11 window
    # covers it: offsets up to 5 give S < 1, offset 6 gives exactly 1.
    x = np.zeros((1, 41, 41))
    x[0, 20, 20] = 1.0
    s = ssim.ssim_map(_t(x), _t(np.zeros_like(x))).numpy()[0]
    for d in range(6):
        assert s[20, 20 + d] < 1.0 and s[20 + d, 20] < 1.0 and s[20 + d, 20 + d] < 1.0
    assert s[20, 26] == 1.0 and s[26, 20] == 1.0 and s[20, 14] == 1.0
    # and the response is symmetric under the dihedral group of the window
    np.testing.assert_array_equal(s, s[::-1, :])
    np.testing.assert_array_equal(s, s.T)


def test_impulse_closed_form_with_unit_gaussian_weights():
    # at offset (i, j): mu_x = h w, E[x^2] = h^2 w with w the window weight, and
    # every y statistic is zero, so S = C1 C2 / ((h^2 w^2 + C1)(h^2 w (1 - w) + C2)).
    # The weights are the normalised samples of exp(-k^2 / 4.5) (sigma 1.5).
    h = 0.8
    x = np.zeros((1, 31, 31))
    x[0, 15, 15] = h
    s = ssim.ssim_map(_t(x), _t(np.zeros_like(x))).numpy()[0]
    k = np.arange(-5, 6)
    g = np.exp(-k * k / 4.5)
    g /= g.sum()
    for i, j in [(0, 0), (1, 0), (2, 3), (5, 5), (4, 1)]:
        w = g[i + 5] * g[j + 5]
        expect = 1e-4 * 9e-4 / ((h * h * w * w + 1e-4) * (h * h * w * (1 - w) + 9e-4))
        assert s[15 + i, 15 + j] == pytest.approx(expect, rel=1e-12)


def test_symmetric_and_bounded():
    rng = np.random.default_rng(1)
    x = rng.uniform(0, 1, size=(1, 20, 24))
    y = rng.uniform(0, 1, size=(1, 20, 24))
    sxy = ssim.ssim_map(_t(x), _t(y)).numpy()
    syx = ssim.ssim_map(_t(y), _t(x)).numpy()
    np.testing.assert_allclose(sxy, syx, rtol=1e-14)
    assert np.abs(sxy).max() <= 1.0


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    x = rng.uniform(0, 1, size=(2, 14, 17))
    y = rng.uniform(0, 1, size=(2, 14, 17))
    L, l1, d, g = ssim.loss(x, y, lam=0.2)
    assert L == pytest.approx(l1 + 0.2 * d, rel=1e-14)
    h = 1e-6
    for idx in [(0, 0, 0), (1, 7, 8), (0, 13, 16), (1, 3, 0), (0, 6, 12)]:
        xp = x.copy()
        xm = x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd = (ssim.loss(xp, y)[0] - ssim.loss(xm, y)[0]) / (2 * h)
        assert g[idx] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_l1_part_and_tie():
    x = np.array([[[0.5, 0.2], [0.1, 0.9]]])
    y = np.array([[[0.5, 0.3], [0.0, 0.9]]])
    _, l1, _, g = ssim.loss(x, y, lam=0.0)
    assert l1 == pytest.approx((0.1 + 0.1) / 4, rel=1e-14)
    np.testing.assert_allclose(g, np.array([[[0.0, -0.25], [0.25, 0.0]]]), rtol=1e-14)
