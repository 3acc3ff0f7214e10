"""Long walks: faint splats (opacity 0.004-0.011, so alpha reaches 1/255
only near a splat's centre) whose pixels never reach the transmittance
floor, so every quarter walks its tile's whole list (~12000 splats) and the
forward writes a checkpoint at every multiple of the segment length.  The
checkpoint pool holds a slot per 64-pixel group and 64 instances of capacity
(where that fits 8 GiB, as here), so such walks cannot run out of it: the
call succeeds (no capacity flag), the images, final transmittance and last
members equal, bit for bit, those of the walk with no segments (one backward
item per tile, no checkpoints), and the gradients agree with it to rounding.
(The pool once held one slot per 256 instances: this scene needs ~6800
slots, at most 4096 were there.)"""
import numpy as np
import pytest
import torch

import synthetic as S
from tests.gpu_util import GpuScene

pytestmark = pytest.mark.gpu


def _faint_scene(n, size, seed):
    rng = np.random.default_rng(seed)
    p = S.make_scene(n, 0, seed=seed)
    p[10] = rng.uniform(-5.5, -4.5, n)
    return p.astype(np.float32), 0, [S.look_at(20.0, 35.0, size, size)]


def _run(p, D, cams, fwd, seg):
    from paper_2504_06716_amd import _lib as L
    V, H, W = len(cams), cams[0].height, cams[0].width
    g = GpuScene(p, D, cams, bg=(0.2, 0.1, 0.05), capacity=1 << 18)
    g.ctx.set_waves(fwd=fwd)
    g.ctx.set_option(L.OPT_BWD_SEGMENT, seg)
    img = g.forward()
    tf = g.state(L.STATE_T_FINAL, torch.float32, (V, H, W))
    last = g.state(L.STATE_LAST, torch.int32, (V, H, W))
    dL = np.random.default_rng(5).standard_normal((V, 3, H, W)).astype(np.float32)
    grad, g2, _ = g.backward(dL, sentinel=7.0)
    st, inst = g.ctx.check()
    assert st == L.GSTA_OK, (st, inst)
    return dict(img=img, tf=tf, last=last, grad=grad, g2=g2)


@pytest.mark.parametrize("fwd", [0, 4])
def test_long_walks_fit_the_checkpoint_pool(fwd):
    print(f"long walks fwd={fwd}", flush=True)
    p, D, cams = _faint_scene(30000, 48, 7)
    seg = _run(p, D, cams, fwd, 64)
    whole = _run(p, D, cams, fwd, 0)
    for k in ("img", "tf", "last"):
        assert np.array_equal(seg[k], whole[k]), k
    for k in ("grad", "g2"):
        np.testing.assert_allclose(seg[k], whole[k], rtol=1e-4, atol=1e-6 * np.abs(whole[k]).max(), err_msg=k)
    # walks past thousands of list positions, nowhere near the floor
    assert seg["last"].max() > 6000
    assert seg["tf"].min() > 1e-3
