"""The L1 loss fused into the forward compositing (gsta_render_forward_l1)
against the separate pass (gsta_render_forward + gsta_l1_loss): the same
image and dL/dimage bit for bit, the same loss sums up to the order of their
double additions, and the same training run."""
import numpy as np
import pytest

import synthetic as S
from tests.gpu_util import GpuScene, dev

pytestmark = pytest.mark.gpu


def _case(kind):
    if kind == "tiny":
        p = S.make_scene(64, 3, seed=0)
        p[3:6] += 0.9
        return p, 3, [S.look_at(10.0 + 35.0 * k, 20.0 + 70.0 * k, 32, 32) for k in range(2)]
    if kind == "ragged":
        p = S.make_scene(3000, 3, seed=5)
        p[3:6] += 0.5
        return p, 3, [S.look_at(25.0, 130.0, 50, 37), S.look_at(-40.0, 10.0, 50, 37)]
    c = S.CONFIGS["c2"]
    return S.make_scene(c["n"], 3), 3, S.config_cameras("c2")[:1]


@pytest.mark.parametrize("kind", ["tiny", "ragged", "c2view"])
@pytest.mark.parametrize("fwd", [0, 1, 2, 4])
def test_fused_l1_equals_separate_loss(kind, fwd):
    import torch
    p, D, cams = _case(kind)
    print(f"fused l1 {kind} forward waves {fwd}", flush=True)
    V, H, W = len(cams), cams[0].height, cams[0].width
    tgt = dev(np.random.default_rng(7).random((V, 3, H, W)).astype(np.float32))
    out = []
    for fused in (False, True):
        g = GpuScene(p, D, cams, bg=(0.1, 0.2, 0.3))
        g.ctx.set_waves(fwd=fwd)
        img = torch.empty((V, 3, H, W), device="cuda")
        dL = torch.full_like(img, float("nan"))
        sums = torch.zeros(2, dtype=torch.float64, device="cuda")
        if fused:
            g.ctx.render_forward_l1(g.P, D, g.carr, g.bg, tgt, img, dL, sums, 0)
        else:
            g.ctx.render_forward(g.P, D, g.carr, g.bg, img, 0)
            g.ctx.l1_loss(img, tgt, dL, sums)
        grad, g2, _ = g.backward(dL.cpu().numpy())
        torch.cuda.synchronize()
        out.append((img.cpu().numpy(), dL.cpu().numpy(), sums.cpu().numpy(), grad, g2))
    (i0, d0, s0, gr0, g20), (i1, d1, s1, gr1, g21) = out
    assert np.array_equal(i0, i1)
    assert np.array_equal(d0, d1)
    np.testing.assert_allclose(s1, s0, rtol=1e-12)
    assert np.array_equal(gr0, gr1, equal_nan=True) and np.array_equal(g20, g21)


def test_fused_loss_training_equals_separate_loss():
    import torch
    from paper_2504_06716_amd.schedule import FreezeSchedule, LearningRates
    from paper_2504_06716_amd.train import Trainer, TrainConfig, render_targets
    import paper_2504_06716_amd as G
    p = S.make_scene(2000, 3, seed=4)
    p[3:6] += 0.4
    cams = [S.look_at(-20.0 + 10 * k, 40.0 * k, 48, 40) for k in range(4)]
    ctx = G.Context(2000, 4, 40, 48, 1 << 20)
    tgt = render_targets(ctx, S.perturb_scene(p, 3), 3, cams)
    res = []
    for fused in (False, True):
        sched = FreezeSchedule(total_iters=60, warmup=10, every=5, reset_every=30, wait=5, window_end=50,
                               eps_xyz0=1e-6, eps_rgb0=1e-7)
        cfg = TrainConfig(iters=60, freeze=True, schedule=sched, lrs=LearningRates(decay_iters=60),
                          fused_loss=fused)
        tr = Trainer(p, 3, cams, tgt, cfg, S.view_order(4, 60), ctx=ctx)
        tr.run(60)
        torch.cuda.synchronize()
        res.append((tr.P.cpu().numpy(), tr.frozen.cpu().numpy(), tr.sums.cpu().numpy()))
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1], res[1][1])
    np.testing.assert_allclose(res[1][2], res[0][2], rtol=1e-12)
