"""Pins of the oracle's SH-band masking (Section 3.3, the finetune stage of
the +small variant): gated bands equal a scene with those coefficients set
to zero, open gates equal no masking, the straight-through gradient of a
mask logit equals a finite difference of the loss in the band's scale
factor times sigmoid'(logit), and the sparsity term's closed form.  All CPU."""
import numpy as np
import pytest

import oracle as O
from tests.test_oracle_pins import tiny_scene

THR = 0.01
BANDS = {1: range(1, 4), 2: range(4, 9), 3: range(9, 16)}


def _sh_rows(band):
    return [11 + 3 * k + ch for k in BANDS[band] for ch in range(3)]


def _loss_and_grads(p, cams, wimg, logits=None):
    if logits is None:
        img = [O.render(p, 3, c)["image"] for c in cams]
        g, _, _ = O.render_backward(p, 3, cams, wimg)
        return img, g, None
    with O.sh_mask(logits, THR) as m:
        img = [O.render(p, 3, c)["image"] for c in cams]
        g, _, _ = O.render_backward(p, 3, cams, wimg)
    return img, g, m.grad


def test_open_gates_equal_no_mask():
    p, cams = tiny_scene(n=64, degree=3, size=32, log_s_shift=0.9)
    rng = np.random.default_rng(3)
    wimg = rng.standard_normal((len(cams), 3, 32, 32))
    logits = rng.uniform(0.5, 4.0, (3, p.shape[1]))            # sigmoid > 0.62: every gate open
    a, ga, _ = _loss_and_grads(p, cams, wimg)
    b, gb, _ = _loss_and_grads(p, cams, wimg, logits)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    np.testing.assert_array_equal(ga, gb)


@pytest.mark.parametrize("closed", [(1, 2, 3), (2,), (1, 3)])
def test_closed_bands_equal_zero_coefficients(closed):
    p, cams = tiny_scene(n=64, degree=3, size=32, log_s_shift=0.9)
    rng = np.random.default_rng(4)
    wimg = rng.standard_normal((len(cams), 3, 32, 32))
    n = p.shape[1]
    logits = np.full((3, n), 3.0)
    for l in closed:
        logits[l - 1] = -8.0                                    # sigmoid = 3.4e-4 < 0.01: gate closed
    pz = p.copy()
    for l in closed:
        pz[_sh_rows(l)] = 0.0
    a, ga, _ = _loss_and_grads(pz, cams, wimg)
    b, gb, _ = _loss_and_grads(p, cams, wimg, logits)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    masked = sorted(r for l in closed for r in _sh_rows(l))
    rest = [r for r in range(p.shape[0]) if r not in masked]
    np.testing.assert_array_equal(gb[rest], ga[rest])
    assert (gb[masked] == 0).all()                              # a closed band's coefficients learn nothing
    assert np.abs(gb[rest]).max() > 0


def _scaled_loss(p, cams, wimg, g, band, s):
    q = p.copy()
    q[_sh_rows(band), g] *= s
    return sum((O.render(q, 3, c)["image"] * wimg[v]).sum() for v, c in enumerate(cams))


def test_straight_through_gradient_matches_band_scale_differences():
    p, cams = tiny_scene(n=48, degree=3, size=32, log_s_shift=1.0)
    rng = np.random.default_rng(5)
    wimg = rng.standard_normal((len(cams), 3, 32, 32))
    n = p.shape[1]
    p[11:] *= 3.0                                               # colours well away from the clamp at 0
    p[11:14] += 1.0
    logits = rng.uniform(0.5, 3.0, (3, n))
    logits[1, ::3] = -9.0                                       # band 2 closed on every third Gaussian
    _, _, gm = _loss_and_grads(p, cams, wimg, logits)
    sg = 1.0 / (1.0 + np.exp(-logits))
    gates = O.sh_band_gates(logits, THR)
    h = 1e-5
    # the masked scene written out: every closed band's coefficients zeroed
    q0 = p.copy()
    for b2 in (1, 2, 3):
        for g2 in range(n):
            if gates[b2 - 1, g2] == 0.0:
                q0[_sh_rows(b2), g2] = 0.0
    checked = 0
    for g in range(n):
        for band in (1, 2, 3):
            M = gates[band - 1, g]
            # dL/dM at the gate's value: the band's own coefficients scaled by
            # M +- h, rendered without masks
            q = q0.copy()
            q[_sh_rows(band), g] = p[_sh_rows(band), g]
            fd = (_scaled_loss(q, cams, wimg, g, band, M + h) - _scaled_loss(q, cams, wimg, g, band, M - h)) / (2 * h)
            want = fd * sg[band - 1, g] * (1.0 - sg[band - 1, g])
            got = gm[band - 1, g]
            assert abs(got - want) <= 1e-6 * max(1.0, abs(want)), (g, band, got, want)
            checked += abs(want) > 1e-8
        if checked >= 40:
            break
    assert checked >= 20


def test_sparsity_term_closed_form():
    x = np.zeros((3, 10))
    loss, grad = O.sh_mask_reg(x, 0.5)
    assert loss == pytest.approx(0.25)
    np.testing.assert_allclose(grad, 0.5 * 0.25 / 30)
    rng = np.random.default_rng(6)
    x = rng.standard_normal((3, 7))
    _, grad = O.sh_mask_reg(x, 2.0)
    h = 1e-6
    for i in range(3):
        for j in range(7):
            xp, xm = x.copy(), x.copy()
            xp[i, j] += h
            xm[i, j] -= h
            fd = (O.sh_mask_reg(xp, 2.0)[0] - O.sh_mask_reg(xm, 2.0)[0]) / (2 * h)
            assert grad[i, j] == pytest.approx(fd, rel=1e-6)
