"""Pins of the oracle's finetune-stage absolute opacity activation (Section
4.1: sigmoid -> absolute value when the finetune starts): a closed form with
an opacity above 1, equivalence with the sigmoid parameterisation after the
switch, and finite differences of the backward.  All CPU."""
import math

import numpy as np
import pytest

import oracle as O
import synthetic as S
from tests.test_oracle_pins import _decisions, _same, _single, tiny_scene


def test_single_gaussian_above_one_closed_form():
    cam = S.config_cameras("c1")[0]
    s, x, rgb = 0.08, -2.5, np.array([0.2, 0.5, 0.9])
    p = _single([0.0, 0.0, 0.0], [math.log(s)] * 3, logit=x, rgb=rgb)
    with O.opacity_activation(1):
        out = O.render(p, 0, cam)
    sig2 = (cam.fx * s / 3.0) ** 2 + 0.3
    py, px = np.mgrid[0:cam.height, 0:cam.width].astype(np.float64)
    power = -0.5 * ((px - cam.cx) ** 2 + (py - cam.cy) ** 2) / sig2
    alpha = np.minimum(0.99, 2.5 * np.exp(power))            # o = |x| = 2.5: capped near the centre
    mem = (power >= -4.5) & (alpha >= 1 / 255)
    np.testing.assert_allclose(out["image"], rgb[:, None, None] * np.where(mem, alpha, 0.0)[None], atol=1e-13)
    assert (alpha[mem] == 0.99).sum() > 4 and (alpha[mem] < 0.99).sum() > 20
    # the activation is reset after the block
    out0 = O.render(p, 0, cam)
    assert np.abs(out0["image"] - out["image"]).max() > 0.1


def test_switch_keeps_every_opacity():
    p, cams = tiny_scene(n=64, degree=3, size=32, log_s_shift=0.9)
    m = np.random.default_rng(1).standard_normal(p.shape)
    P2, M2, V2 = O.opacity_to_absolute(p, m, np.abs(m))
    assert (M2[10] == 0).all() and (V2[10] == 0).all()
    np.testing.assert_array_equal(M2[:10], m[:10])
    a = O.render(p, 3, cams[0])["image"]
    with O.opacity_activation(1):
        b = O.render(P2, 3, cams[0])["image"]
    np.testing.assert_allclose(b, a, atol=1e-12)


@pytest.mark.parametrize("shift", [0.9, 1.3])
def test_absolute_backward_matches_finite_differences(shift):
    p, cams = tiny_scene(n=48, degree=1, size=32, log_s_shift=shift)
    rng = np.random.default_rng(12)
    p[10] = rng.uniform(-1.6, 1.6, p.shape[1])            # opacities |x| up to 1.6, both signs
    wimg = rng.standard_normal((len(cams), 3, 32, 32))
    with O.opacity_activation(1):
        def loss(pp):
            return sum((O.render(pp, 1, c)["image"] * wimg[v]).sum() for v, c in enumerate(cams))

        grads, _, _ = O.render_backward(p, 1, cams, wimg)
        base = _decisions(p, 1, cams)
        R, n = p.shape
        gmax = np.abs(grads).max()
        checked = skipped = 0
        for g in range(n):
            for row in (0, 3, 6, 10, 11):
                h = 1e-6 * max(abs(p[row, g]), 0.1)
                pp, pm = p.copy(), p.copy()
                pp[row, g] += h
                pm[row, g] -= h
                if not (_same(_decisions(pp, 1, cams), base) and _same(_decisions(pm, 1, cams), base)):
                    skipped += 1
                    continue
                fd = (loss(pp) - loss(pm)) / (2 * h)
                assert abs(fd - grads[row, g]) <= 1e-6 * gmax + 1e-5 * abs(grads[row, g]), (row, g, fd)
                checked += 1
        assert checked > 0.9 * (checked + skipped)
        assert np.abs(grads[10]).max() > 0
