"""SH-band masking of the finetune stage (Section 3.3) on the GPU against
the oracle: images and gradients with some bands gated off (coefficient and
mask-logit gradients, the latter the straight-through estimate), exact
equalities with unmasked and zeroed-coefficient renders, the sparsity term,
the masked Adam over the logits, and argument checks."""
import ctypes

import numpy as np
import pytest

import oracle as O
import synthetic as S
from tests.gpu_util import IMAGE_ATOL, MARGIN_VALUE, GpuScene, compare_grads, dev

pytestmark = pytest.mark.gpu

THR = 0.01
BANDS = {1: range(1, 4), 2: range(4, 9), 3: range(9, 16)}


def _sh_rows(band):
    return [11 + 3 * k + ch for k in BANDS[band] for ch in range(3)]


def _scene(n, size, shift, seed):
    p = S.make_scene(n, 3, seed=seed).astype(np.float64)
    p[3:6] += shift
    p[11:] *= 2.0                     # visible view dependence
    p[11:14] += 0.6
    cams = [S.look_at(10.0 + 35.0 * k, 20.0 + 70.0 * k, size, size) for k in range(2)]
    rng = np.random.default_rng(seed + 1)
    logits = rng.uniform(-6.0, 3.0, (3, n))
    # keep the logits away from the gate (sigmoid = 0.01 at logit -4.595)
    logits[np.abs(logits + 4.595) < 0.05] = 1.0
    return p.astype(np.float32), cams, logits.astype(np.float32)


@pytest.mark.parametrize("n,size,shift", [(64, 32, 0.9), (2000, 48, 0.5)])
def test_masked_forward_and_backward_match_oracle(n, size, shift):
    print(f"sh mask n={n} size={size}", flush=True)
    p, cams, logits = _scene(n, size, shift, seed=n)
    gates = O.sh_band_gates(logits, THR)
    assert 0.2 < gates.mean() < 0.9
    g = GpuScene(p, 3, cams, sh_mask=logits, sh_mask_threshold=THR)
    img = g.forward()
    V = len(cams)
    rng = np.random.default_rng(7)
    dL = rng.standard_normal((V, 3, size, size))
    with O.sh_mask(logits.astype(np.float64), THR) as om:
        outs = [O.render(p, 3, c) for c in cams]
        for v, o in enumerate(outs):
            ok = o["m_value"] >= MARGIN_VALUE
            assert np.abs(img[v] - o["image"])[:, ok].max() <= IMAGE_ATOL
            dL[v][:, (o["m_value"] < MARGIN_VALUE) | (o["m_grad"] < MARGIN_VALUE)] = 0.0
        ref, _, _ = O.render_backward(p, 3, cams, dL)
    grad, _, _ = g.backward(dL.astype(np.float32))
    marg = np.zeros(n, bool)
    for c in cams:
        r = O.project(p, 3, c)
        marg |= (r[:, 28] < 1e-4) | (r[:, 29] < 1e-4) | (r[:, 27] < 1e-3)
    compare_grads(grad, ref, exclude_cols=marg)
    # a closed band's coefficients get exactly zero
    for band in (1, 2, 3):
        closed = gates[band - 1] == 0
        assert (grad[_sh_rows(band)][:, closed] == 0).all()
    # the straight-through logit gradients
    mg, rm = g.mask_grad, om.grad
    keep = ~marg
    d = (mg - rm)[:, keep]
    assert np.linalg.norm(d) <= 2e-3 * np.linalg.norm(rm[:, keep])
    assert (np.abs(d) <= 2e-3 * np.abs(rm[:, keep]) + 2e-3 * np.abs(rm).max()).all()
    assert np.abs(rm).max() > 0


def test_open_and_closed_gates_are_exact():
    p, cams, logits = _scene(500, 40, 0.6, seed=3)
    plain = GpuScene(p, 3, cams)
    a = plain.forward()
    dL = np.random.default_rng(2).standard_normal(a.shape).astype(np.float32)
    ga, _, _ = plain.backward(dL)
    # every gate open: identical to no masking
    op = GpuScene(p, 3, cams, sh_mask=np.full((3, 500), 4.0, np.float32), sh_mask_threshold=THR)
    b = op.forward()
    gb, _, _ = op.backward(dL)
    assert np.array_equal(a, b) and np.array_equal(ga, gb)
    # bands 2 and 3 closed everywhere: identical to those coefficients set to zero
    lg = np.full((3, 500), 4.0, np.float32)
    lg[1:] = -9.0
    pz = p.copy()
    pz[_sh_rows(2) + _sh_rows(3)] = 0.0
    zs = GpuScene(pz, 3, cams)
    c = zs.forward()
    gc, _, _ = zs.backward(dL)
    ms = GpuScene(p, 3, cams, sh_mask=lg, sh_mask_threshold=THR)
    d = ms.forward()
    gd, _, _ = ms.backward(dL)
    assert np.array_equal(c, d)
    rest = [r for r in range(p.shape[0]) if r not in _sh_rows(2) + _sh_rows(3)]
    assert np.array_equal(gc[rest], gd[rest])
    assert (gd[_sh_rows(2) + _sh_rows(3)] == 0).all()


def test_sparsity_term_and_adam_rows():
    import torch
    import paper_2504_06716_amd as G
    n = 70001
    rng = np.random.default_rng(9)
    x = rng.uniform(-7.0, 4.0, (3, n)).astype(np.float32)
    ctx = G.Context(n, 1, 16, 16, 16)
    X = dev(x.copy())
    gr = rng.standard_normal((3, n)).astype(np.float32)
    GR = dev(gr.copy())
    frozen = (rng.random(n) < 0.3).astype(np.uint8)
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    ctx.sh_mask_reg(X, THR, 0.3, out, frozen=dev(frozen), grad=GR)
    torch.cuda.synchronize()
    loss, rg = O.sh_mask_reg(x.astype(np.float64), 0.3)
    o = out.cpu().numpy()
    assert o[0] == pytest.approx(loss, rel=1e-6)
    gates = O.sh_band_gates(x, THR)
    assert o[1:].tolist() == gates.sum(1).tolist()
    got = GR.cpu().numpy()
    want = gr.astype(np.float64) + np.where(frozen[None] == 0, rg, 0.0)
    np.testing.assert_allclose(got, want, rtol=1e-6, atol=1e-12)
    assert np.array_equal(got[:, frozen == 1], gr[:, frozen == 1])
    # masked Adam over the three logit rows
    m = rng.standard_normal((3, n)).astype(np.float32) * 0.01
    v = np.abs(rng.standard_normal((3, n)).astype(np.float32)) * 1e-4
    Pm, Gm, Mm, Vm = dev(x.copy()), dev(gr.copy()), dev(m.copy()), dev(v.copy())
    lrs = [0.05, 0.02, 0.01]
    ctx.adam_rows(Pm, Gm, Mm, Vm, lrs, 0.9, 0.999, 1e-15, 7, frozen=dev(frozen))
    torch.cuda.synchronize()
    rp, rm, rv = O.adam_masked(x.astype(np.float64), gr.astype(np.float64), m.astype(np.float64),
                               v.astype(np.float64), np.array(lrs), 0.9, 0.999, 1e-15, 7, frozen)
    np.testing.assert_allclose(Pm.cpu().numpy(), rp, rtol=2e-6, atol=2e-6)
    np.testing.assert_allclose(Mm.cpu().numpy(), rm, rtol=2e-6, atol=2e-7)   # float32 moments of O(1) gradients
    assert np.array_equal(Pm.cpu().numpy()[:, frozen == 1], x[:, frozen == 1])


def test_mask_arguments_are_checked():
    import torch
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd import _lib
    from paper_2504_06716_amd.core import params_struct
    p, cams, logits = _scene(100, 16, 0.5, seed=1)
    g = GpuScene(p, 3, cams, sh_mask=logits, sh_mask_threshold=THR)
    L = _lib.load()
    st = torch.cuda.current_stream().cuda_stream
    img = torch.empty((2, 3, 16, 16), device="cuda")
    bad = params_struct(g.P, 3, 0, g.M, 1.5)                      # threshold outside (0, 1)
    assert L.gsta_render_forward(g.ctx.h, ctypes.byref(bad), g.carr, 2, (ctypes.c_float * 3)(0, 0, 0),
                                 img.data_ptr(), 0, st) == _lib.GSTA_ERR_INVALID
    with pytest.raises(ValueError):
        params_struct(g.P, 3, 0, torch.zeros((3, 99), device="cuda"), THR)
    # a backward must use the forward's masks
    g.forward()
    dL = torch.zeros((2, 3, 16, 16), device="cuda")
    grad = torch.zeros_like(g.P)
    with pytest.raises(_lib.GstaError):
        g.ctx.render_backward(g.P, 3, g.carr, g.bg, 0, dL, None, grad)
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(_lib.GstaError):
        g.ctx.sh_mask_reg(g.M, 0.0, 0.1, out)


@pytest.mark.parametrize("lam,init", [(2000.0, -3.0), (0.0, 2.0)])
def test_training_learns_band_masks_in_the_finetune(lam, init):
    import torch
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd.schedule import FreezeSchedule, LearningRates
    from paper_2504_06716_amd.train import Trainer, TrainConfig, render_targets
    n = 2000
    p = S.make_scene(n, 3, seed=8)
    p[3:6] += 0.4
    cams = [S.look_at(-20.0 + 10 * k, 40.0 * k, 48, 40) for k in range(4)]
    ctx = G.Context(n, 4, 40, 48, 1 << 20)
    tgt = render_targets(ctx, S.perturb_scene(p, 3), 3, cams)
    fs = FreezeSchedule(total_iters=100, warmup=10, every=5, reset_every=30, wait=5, window_end=40,
                        eps_xyz0=1e-6, eps_rgb0=1e-7)
    # a strong sparsity weight closes every gate within the 60 finetune iterations;
    # without it the rendering loss alone keeps (nearly) all of them open
    cfg = TrainConfig(iters=100, freeze=True, schedule=fs, lrs=LearningRates(decay_iters=100), finetune_iters=60,
                      sh_mask_finetune=True, sh_mask_lr=0.2, sh_mask_lambda=lam, sh_mask_init=init)
    tr = Trainer(p, 3, cams, tgt, cfg, S.view_order(4, 100), ctx=ctx)
    tr.run(40)
    assert tr.shm is None and tr.sh_mask_stats() is None
    tr.step()                                         # iteration 40: the masks start, all open
    assert tr.shm is not None
    tr.run()
    torch.cuda.synchronize()
    assert tr.k == 100
    st = tr.sh_mask_stats()
    print("sh mask stats", st, flush=True)
    assert all(0 <= o <= n for o in st["open"])
    if lam > 0:
        assert st["open"] == [0, 0, 0] and st["sh_coeff_kept"] == pytest.approx(1 / 16)
    else:
        assert st["sh_coeff_kept"] > 0.95
    # the masked model renders as the stored model with its closed bands set to zero
    x = tr.shm["x"].cpu().numpy()
    gates = O.sh_band_gates(x, cfg.sh_mask_threshold)
    pz = tr.P.clone()
    for band in (1, 2, 3):
        closed = torch.as_tensor(gates[band - 1] == 0, device="cuda")
        for r in _sh_rows(band):
            pz[r] = torch.where(closed, torch.zeros_like(pz[r]), pz[r])
    img = torch.empty((1, 3, 40, 48), device="cuda")
    ctx.render_forward(pz, 3, [cams[2]], (0, 0, 0), img, 0)
    got = tr.render_views([2])
    torch.cuda.synchronize()
    assert torch.equal(img, got)
    assert np.isfinite(tr.evaluate())
