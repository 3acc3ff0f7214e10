"""Pins of the oracle's D-SSIM (eq. 3, lambda_SSIM = 0.2): the window, the
zero-padded filter against scipy, closed forms (identical images, constant
images including the border), symmetry, and finite differences of the
gradient.  All CPU."""
import math

import numpy as np
import pytest
import scipy.ndimage as nd

import oracle as O


def test_window_taps():
    w = O.ssim_window_1d()
    assert w.shape == (11,)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    np.testing.assert_allclose(w, w[::-1], rtol=0, atol=0)
    assert w[5] / w[4] == pytest.approx(math.exp(1.0 / 4.5), rel=1e-14)
    assert w[5] / w[0] == pytest.approx(math.exp(25.0 / 4.5), rel=1e-14)


def test_filter_matches_scipy_zero_padded_correlation():
    rng = np.random.default_rng(1)
    w = O.ssim_window_1d()
    for shape in [(1, 1), (5, 3), (17, 23), (2, 3, 12, 9)]:
        x = rng.random(shape)
        got = O.filter2d_same(x, w)
        k = np.outer(w, w)
        if x.ndim == 2:
            ref = nd.correlate(x, k, mode="constant", cval=0.0)
        else:
            ref = np.stack([np.stack([nd.correlate(x[i, j], k, mode="constant", cval=0.0)
                                      for j in range(shape[1])]) for i in range(shape[0])])
        np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-15)


def test_identical_images_give_one():
    x = np.random.default_rng(2).random((2, 3, 14, 19))
    np.testing.assert_allclose(O.ssim_map(x, x), 1.0, rtol=0, atol=1e-12)
    loss, grad, ssum = O.dssim_loss(x, x)
    assert loss == pytest.approx(0.0, abs=1e-12)
    assert ssum == pytest.approx(x.size, rel=1e-13)
    np.testing.assert_allclose(grad, 0.0, atol=1e-12)     # a maximum of SSIM


def test_constant_images_closed_form_with_border():
    # x = a, y = b everywhere: mu_x = a W(p), sigma_x^2 = a^2 W (1 - W),
    # sigma_xy = a b W (1 - W), with W(p) the window weight inside the image
    H, W_ = 9, 14
    a, b = 0.3, 0.7
    w = O.ssim_window_1d()
    r = 5

    def inside(n):
        return np.array([sum(w[t] for t in range(11) if 0 <= i + t - r < n) for i in range(n)])

    Wp = np.outer(inside(H), inside(W_))
    mx, my = a * Wp, b * Wp
    sxx, syy, sxy = a * a * Wp * (1 - Wp), b * b * Wp * (1 - Wp), a * b * Wp * (1 - Wp)
    C1, C2 = 1e-4, 9e-4
    ref = ((2 * mx * my + C1) * (2 * sxy + C2)) / ((mx ** 2 + my ** 2 + C1) * (sxx + syy + C2))
    got = O.ssim_map(np.full((H, W_), a), np.full((H, W_), b))
    np.testing.assert_allclose(got, ref, rtol=1e-12)
    # far enough from the border (a 21 x 21 image has an interior point): W = 1
    g = O.ssim_map(np.full((21, 21), a), np.full((21, 21), b))
    assert g[10, 10] == pytest.approx((2 * a * b + C1) / (a * a + b * b + C1), rel=1e-12)


def test_symmetric_in_its_arguments():
    rng = np.random.default_rng(3)
    x, y = rng.random((3, 10, 12)), rng.random((3, 10, 12))
    np.testing.assert_allclose(O.ssim_map(x, y), O.ssim_map(y, x), rtol=1e-14)


def test_dssim_gradient_matches_finite_differences():
    rng = np.random.default_rng(4)
    x, y = rng.random((1, 3, 9, 11)), rng.random((1, 3, 9, 11))
    _, g, _ = O.dssim_loss(x, y)
    h = 1e-6
    fd = np.zeros_like(x)
    for idx in np.ndindex(x.shape):
        xp, xm = x.copy(), x.copy()
        xp[idx] += h
        xm[idx] -= h
        fd[idx] = (O.dssim_loss(xp, y)[0] - O.dssim_loss(xm, y)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-10)


def test_total_loss_weights():
    rng = np.random.default_rng(5)
    x, y = rng.random((1, 3, 8, 8)), rng.random((1, 3, 8, 8))
    L, g = O.total_loss(x, y, 0.2)
    l1, g1, _ = O.l1_loss(x, y)
    ld, gd, _ = O.dssim_loss(x, y)
    assert L == pytest.approx(0.8 * l1 + 0.2 * ld, rel=1e-14)
    np.testing.assert_allclose(g, 0.8 * g1 + 0.2 * gd, rtol=1e-14)
