"""The per-splat backward compositing variant (GSTA_OPT_BWD_VARIANT = 1:
lanes are splats, pixel state passed lane to lane; Section 3.2.4) against the
oracle and against the default per-pixel variant: gradients of every
parameter group, frozen rows untouched, per-view 2-D gradients, segment
lengths from 64 to unsegmented, several views per call, and the options'
checks.  The two variants add a splat's terms in different orders, so they
agree to rounding."""
import numpy as np
import pytest

import oracle as O
from tests.gpu_util import MARGIN_VALUE, GpuScene, compare_grads
from tests.test_gpu_parity import CASES, _forward_compare, _margins, scene

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2504_06716_amd import _lib
    return _lib


def _case(kind, frozen=None, bg=(0.0, 0.0, 0.0), seed=31):
    p, D, cams = scene(kind)
    g, img, outs, _ = _forward_compare(p, D, cams, bg=bg)
    V, H, W = len(cams), cams[0].height, cams[0].width
    dL = np.random.default_rng(seed).standard_normal((V, 3, H, W))
    for v, o in enumerate(outs):
        dL[v][:, (o["m_value"] < MARGIN_VALUE) | (o["m_grad"] < MARGIN_VALUE)] = 0.0
    dL = dL.astype(np.float32)
    g0, g20, _ = g.backward(dL, frozen=frozen, sentinel=7.0)
    g.ctx.set_option(_lib().OPT_BWD_VARIANT, 1)
    g1, g21, _ = g.backward(dL, frozen=frozen, sentinel=7.0)
    assert g.ctx.check()[0] == 0
    return p, D, cams, dL, (g0, g20), (g1, g21)


@pytest.mark.parametrize("kind", CASES + ["c2view"])
def test_per_splat_backward_matches_oracle_and_per_pixel(kind):
    print(f"per-splat backward {kind}", flush=True)
    p, D, cams, dL, (g0, g20), (g1, g21) = _case(kind)
    ref, ref2, _ = O.render_backward(p, D, cams, dL.astype(np.float64))
    recs, marg = _margins(p, D, cams)
    for r in recs:
        marg |= (r[:, 28] < 1e-4) | (r[:, 29] < 1e-4)
    compare_grads(g1, ref, exclude_cols=marg)
    np.testing.assert_allclose(g1, g0, rtol=1e-4, atol=1e-6 * np.abs(g0).max())
    np.testing.assert_allclose(g21, g20, rtol=1e-4, atol=1e-6 * np.abs(g20).max())


def test_per_splat_backward_frozen_and_background():
    p, D, cams = scene("ragged")
    frozen = (np.random.default_rng(4).random(p.shape[1]) < 0.6).astype(np.uint8)
    _, _, _, dL, (g0, _), (g1, _) = _case("ragged", frozen=frozen, bg=(0.3, 0.6, 0.1))
    act = frozen == 0
    assert (g1[:, ~act] == 7.0).all()          # frozen rows untouched
    np.testing.assert_allclose(g1[:, act], g0[:, act], rtol=1e-4, atol=1e-6 * np.abs(g0[:, act]).max())


@pytest.mark.parametrize("kind", ["ragged", "c2view"])
def test_per_splat_backward_for_every_segment_length(kind):
    """Segments of 64 splats map one splat per lane; longer segments (and
    the unsegmented walk) run 64-splat spans one after the other, the pixel
    state carried between them through LDS."""
    from paper_2504_06716_amd import _lib as L
    p, D, cams = scene(kind)
    H, W = cams[0].height, cams[0].width
    dL = np.random.default_rng(12).standard_normal((len(cams), 3, H, W)).astype(np.float32)
    g = GpuScene(p, D, cams)
    g.forward()
    ref, ref2, _ = g.backward(dL)
    g.ctx.set_option(L.OPT_BWD_VARIANT, 1)
    for seg in (64, 128, 256, 4096, 0):
        print(f"per-splat backward {kind} segment {seg}", flush=True)
        g.ctx.set_option(L.OPT_BWD_SEGMENT, seg)
        g.forward()
        grad, g2, _ = g.backward(dL)
        np.testing.assert_allclose(grad, ref, rtol=1e-4, atol=1e-6 * np.abs(ref).max())
        np.testing.assert_allclose(g2, ref2, rtol=1e-4, atol=1e-6 * np.abs(ref2).max())
    assert g.ctx.check()[0] == 0


def test_per_splat_backward_multiview_and_options():
    import synthetic as S
    from paper_2504_06716_amd import _lib as L
    p = S.make_scene(4000, 3, seed=9)
    p[3:6] += 0.5
    cams = [S.look_at(-30.0 + 20.0 * k, 10.0 * k, 40, 48) for k in range(4)]
    dL = np.random.default_rng(2).standard_normal((4, 3, 48, 40)).astype(np.float32)
    g = GpuScene(p, 3, cams)
    g.forward()
    ref, _, _ = g.backward(dL)
    g.ctx.set_option(L.OPT_BWD_VARIANT, 1)
    grad, _, _ = g.backward(dL)
    np.testing.assert_allclose(grad, ref, rtol=1e-4, atol=1e-6 * np.abs(ref).max())
    with pytest.raises(L.GstaError):
        g.ctx.set_option(L.OPT_BWD_VARIANT, 2)
