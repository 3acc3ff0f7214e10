"""The finetune stage's absolute opacity activation on the GPU (Section 4.1)
against the oracle: records, images and gradients with opacity = |x|
(values above 1, both signs), the switch kernel, argument checks, and a
training run that switches when its freezing window closes."""
import numpy as np
import pytest

import oracle as O
import synthetic as S
from tests.gpu_util import IMAGE_ATOL, MARGIN_VALUE, GpuScene, compare_grads, dev

pytestmark = pytest.mark.gpu


def _scene(n, degree, size, shift, seed):
    p = S.make_scene(n, degree, seed=seed).astype(np.float64)
    p[3:6] += shift
    p[10] = np.random.default_rng(seed).uniform(-1.8, 1.8, n)      # opacity |x|, up to 1.8
    cams = [S.look_at(10.0 + 35.0 * k, 20.0 + 70.0 * k, size, size) for k in range(2)]
    return p.astype(np.float32), cams


@pytest.mark.parametrize("n,degree,size,shift", [(64, 3, 32, 0.9), (3000, 1, 56, 0.4)])
def test_absolute_opacity_forward_and_backward(n, degree, size, shift):
    print(f"abs opacity n={n} D={degree} size={size}", flush=True)
    p, cams = _scene(n, degree, size, shift, seed=n)
    g = GpuScene(p, degree, cams, opacity_act=1)
    img = g.forward()
    V = len(cams)
    rng = np.random.default_rng(3)
    dL = rng.standard_normal((V, 3, size, size))
    with O.opacity_activation(1):
        outs = [O.render(p, degree, c) for c in cams]
        for v, o in enumerate(outs):
            ok = o["m_value"] >= MARGIN_VALUE
            assert np.abs(img[v] - o["image"])[:, ok].max() <= IMAGE_ATOL
            assert (~ok).mean() < 0.01
            dL[v][:, (o["m_value"] < MARGIN_VALUE) | (o["m_grad"] < MARGIN_VALUE)] = 0.0
        ref, _, _ = O.render_backward(p, degree, cams, dL)
    grad, _, _ = g.backward(dL.astype(np.float32))
    recs = [O.project(p, degree, c) for c in cams]
    marg = np.zeros(n, bool)
    for r in recs:
        marg |= (r[:, 28] < 1e-4) | (r[:, 29] < 1e-4) | (r[:, 27] < 1e-3)
    compare_grads(grad, ref, exclude_cols=marg)
    assert np.abs(ref[10]).max() > 0


def test_switch_kernel_matches_oracle_and_is_checked():
    import torch
    import paper_2504_06716_amd as G
    n = 1001
    rng = np.random.default_rng(5)
    p = rng.standard_normal((14, n)).astype(np.float32)
    m = rng.standard_normal((14, n)).astype(np.float32)
    v = np.abs(m)
    ctx = G.Context(n, 1, 16, 16, 16)
    P, M, V = dev(p.copy()), dev(m.copy()), dev(v.copy())
    ctx.opacity_to_absolute(P, M, V, 0)
    torch.cuda.synchronize()
    rp, rm, rv = O.opacity_to_absolute(p, m, v)
    got = P.cpu().numpy()
    np.testing.assert_allclose(got[10], rp[10], rtol=2e-7, atol=1e-9)
    assert np.array_equal(np.delete(got, 10, 0), np.delete(p, 10, 0))
    assert (M.cpu().numpy()[10] == 0).all() and (V.cpu().numpy()[10] == 0).all()
    assert np.array_equal(np.delete(M.cpu().numpy(), 10, 0), np.delete(m, 10, 0))
    # densification and the opacity reset work on logits: they refuse the absolute activation
    from paper_2504_06716_amd import _lib
    from paper_2504_06716_amd.core import params_struct
    import ctypes
    L = _lib.load()
    sp = params_struct(P, 0, 1)
    sm, sv = params_struct(M, 0), params_struct(V, 0)
    st = torch.cuda.current_stream().cuda_stream
    assert L.gsta_opacity_reset(ctx.h, ctypes.byref(sp), ctypes.byref(sm), ctypes.byref(sv), None, 0.0,
                                st) == _lib.GSTA_ERR_INVALID
    assert L.gsta_opacity_to_absolute(ctx.h, ctypes.byref(sp), ctypes.byref(sm), ctypes.byref(sv),
                                      st) == _lib.GSTA_ERR_INVALID
    bad = params_struct(P, 0, 2)
    img = torch.empty((1, 3, 16, 16), device="cuda")
    cam = G.camera_array([S.look_at(0.0, 0.0, 16, 16)])
    assert L.gsta_render_forward(ctx.h, ctypes.byref(bad), cam, 1, (ctypes.c_float * 3)(0, 0, 0), img.data_ptr(),
                                 0, st) == _lib.GSTA_ERR_INVALID


@pytest.mark.parametrize("graph", [False, True])
def test_training_switches_to_absolute_at_the_finetune(graph):
    import torch
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd.schedule import FreezeSchedule, LearningRates
    from paper_2504_06716_amd.train import Trainer, TrainConfig, render_targets
    n = 2000
    p = S.make_scene(n, 1, seed=7)
    p[3:6] += 0.4
    cams = [S.look_at(-20.0 + 10 * k, 40.0 * k, 48, 40) for k in range(4)]
    ctx = G.Context(n, 4, 40, 48, 1 << 20)
    tgt = render_targets(ctx, S.perturb_scene(p, 1), 1, cams)
    fs = FreezeSchedule(total_iters=60, warmup=10, every=5, reset_every=30, wait=5, window_end=40,
                        eps_xyz0=1e-6, eps_rgb0=1e-7)
    cfg = TrainConfig(iters=60, freeze=True, schedule=fs, lrs=LearningRates(decay_iters=60), finetune_iters=20,
                      abs_opacity_finetune=True, graph=graph, device_sched=graph)
    tr = Trainer(p, 1, cams, tgt, cfg, S.view_order(4, 60), ctx=ctx)
    tr.run(40)
    assert tr.opacity_act == 0
    logits = tr.P[10].clone()
    img_before = tr.render_views([0])
    tr.step()                                         # iteration 40: the switch, then a finetune step
    assert tr.opacity_act == 1
    tr.run()
    torch.cuda.synchronize()
    assert tr.k == 60
    # at the switch every opacity was kept: re-render the pre-switch state in both activations
    P2 = tr.P.clone()
    P2[10] = torch.sigmoid(logits.double()).float()
    img_abs = torch.empty_like(img_before)
    ctx.render_forward(P2, 1, [cams[0]], (0, 0, 0), img_abs, 0, opacity_act=1)
    P3 = tr.P.clone()
    P3[10] = logits
    img_sig = torch.empty_like(img_before)
    ctx.render_forward(P3, 1, [cams[0]], (0, 0, 0), img_sig, 0)
    torch.cuda.synchronize()
    d = (img_abs - img_sig).abs()              # equal up to float rounding of the opacity (and rare flips of
    assert (d > 1e-5).float().mean().item() < 0.005     # a membership decision at its threshold)
    assert d.median().item() <= 1e-6
    # the finetune trained with |x|: the final state renders as the oracle does with |x|
    pf = tr.P.cpu().numpy().astype(np.float64)
    with O.opacity_activation(1):
        ref = O.render(pf, 1, cams[1])
    got = tr.render_views([1]).cpu().numpy()[0]
    ok = ref["m_value"] >= MARGIN_VALUE
    assert np.abs(got - ref["image"])[:, ok].max() <= IMAGE_ATOL
    assert np.isfinite(pf).all()
