"""The fused D-SSIM term of eq. 3 (gsta_dssim_loss) against the FP64 oracle:
SSIM sums and the combined gradient (1 - lambda) dL_L1 + lambda dL_D-SSIM
element by element, on ragged, multi-view and c2-size images; closed cases;
argument checks; and a training step with lambda_SSIM = 0.2."""
import numpy as np
import pytest

import oracle as O
import synthetic as S
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("shape", [(1, 3, 7, 9), (2, 3, 37, 50), (1, 3, 16, 32), (1, 3, 480, 640)])
@pytest.mark.parametrize("lam", [0.2, 1.0])
def test_dssim_matches_oracle(shape, lam):
    import torch
    import paper_2504_06716_amd as G
    print(f"dssim shape {shape} lambda {lam}", flush=True)
    V, _, H, W = shape
    rng = np.random.default_rng(H * W + V)
    x = rng.random(shape).astype(np.float32)
    y = np.clip(x + rng.normal(0, 0.2, shape), 0, 1).astype(np.float32)
    dl_in = (rng.choice([-1.0, 0.0, 1.0], size=shape) / x.size).astype(np.float32)
    ctx = G.Context(16, V, H, W, 16)
    dL = dev(dl_in.copy())
    ssum = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.dssim_loss(dev(x), dev(y), lam, dL, ssum)
    torch.cuda.synchronize()
    _, g_ref, s_ref = O.dssim_loss(x.astype(np.float64), y.astype(np.float64))
    ref = (1.0 - lam) * dl_in.astype(np.float64) + lam * g_ref
    got = dL.cpu().numpy().astype(np.float64)
    assert ssum.item() == pytest.approx(s_ref, rel=1e-10)
    err = np.abs(got - ref)
    assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)
    assert (err <= 1e-5 * np.abs(ref) + 1e-6 * np.abs(ref).max()).all(), err.max()


def test_dssim_identical_images_and_zero_lambda():
    import torch
    import paper_2504_06716_amd as G
    rng = np.random.default_rng(1)
    x = rng.random((1, 3, 40, 48)).astype(np.float32)
    dl_in = rng.standard_normal(x.shape).astype(np.float32)
    ctx = G.Context(16, 1, 40, 48, 16)
    ssum = torch.zeros(1, dtype=torch.float64, device="cuda")
    dL = dev(dl_in.copy())
    ctx.dssim_loss(dev(x), dev(x), 0.2, dL, ssum)           # SSIM(x, x) = 1 is a maximum: no D-SSIM gradient
    torch.cuda.synchronize()
    assert ssum.item() == pytest.approx(x.size, rel=1e-12)
    np.testing.assert_allclose(dL.cpu().numpy(), 0.8 * dl_in, rtol=1e-6, atol=1e-7)
    y = rng.random(x.shape).astype(np.float32)
    dL = dev(dl_in.copy())
    ctx.dssim_loss(dev(x), dev(y), 0.0, dL, ssum)           # lambda = 0 leaves the L1 gradient as it is
    torch.cuda.synchronize()
    assert np.array_equal(dL.cpu().numpy(), dl_in)


def test_dssim_arguments_rejected():
    import torch
    import paper_2504_06716_amd as G
    ctx = G.Context(16, 1, 32, 32, 16)
    a = torch.zeros((1, 3, 32, 32), device="cuda")
    s = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(G.GstaError):
        ctx.dssim_loss(torch.zeros((2, 3, 32, 32), device="cuda"), torch.zeros((2, 3, 32, 32), device="cuda"), 0.2,
                       torch.zeros((2, 3, 32, 32), device="cuda"), s)           # more views than reserved
    with pytest.raises(G.GstaError):
        ctx.dssim_loss(torch.zeros((1, 3, 33, 32), device="cuda"), torch.zeros((1, 3, 33, 32), device="cuda"), 0.2,
                       torch.zeros((1, 3, 33, 32), device="cuda"), s)           # taller than reserved
    with pytest.raises(G.GstaError):
        ctx.dssim_loss(a, a, 1.5, a.clone(), s)


def test_training_step_with_ssim_matches_oracle_loss_gradient():
    """One trainer iteration with lambda_SSIM = 0.2: the image's gradient the
    backward receives is eq. 3's, (1 - lambda) dL1 + lambda dD-SSIM of the
    rendered image against its target, and the reported loss is eq. 3's."""
    import torch
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd.schedule import LearningRates
    from paper_2504_06716_amd.train import Trainer, TrainConfig, render_targets
    n = 2000
    p = S.make_scene(n, 3, seed=6)
    p[3:6] += 0.4
    cams = [S.look_at(-20.0 + 10 * k, 40.0 * k, 56, 40) for k in range(3)]
    ctx = G.Context(n, 3, 40, 56, 1 << 20)
    tgt = render_targets(ctx, S.perturb_scene(p, 3), 3, cams)
    cfg = TrainConfig(iters=5, freeze=False, lrs=LearningRates(decay_iters=5), lambda_ssim=0.2)
    tr = Trainer(p, 3, cams, tgt, cfg, S.view_order(3, 5), ctx=ctx)
    tr.step()
    torch.cuda.synchronize()
    view = int(tr.order[0])
    img = tr.image.cpu().numpy().astype(np.float64)
    t = tgt[view:view + 1].cpu().numpy().astype(np.float64)
    L_ref, g_ref = O.total_loss(img, t, 0.2)
    got = tr.dL.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(got - g_ref) <= 1e-5 * np.linalg.norm(g_ref)
    assert tr.loss() == pytest.approx(L_ref, rel=1e-6)
    tr.run(4)
    assert np.isfinite(tr.P.cpu().numpy()).all()
