"""The torch.autograd binding (backward recomputes transmittance) against
FP64 finite differences of the oracle forward and the oracle gradient, on a
64-Gaussian 32x32 sub-scene; batched views at the c3 size against sampled
oracle pixels; the autotuner."""
import numpy as np
import pytest

import oracle as O
import synthetic as S
from tests.gpu_util import MARGIN_VALUE, compare_grads, dev

pytestmark = pytest.mark.gpu


def sub_scene(degree=3):
    p = S.make_scene(64, degree, seed=0).astype(np.float64)
    p[3:6] += 0.9
    cams = [S.look_at(10.0 + 35.0 * k, 20.0 + 70.0 * k, 32, 32) for k in range(2)]
    return p.astype(np.float32), cams


def _weights(p, D, cams, seed=31):
    w = np.random.default_rng(seed).standard_normal((len(cams), 3, 32, 32))
    for v, c in enumerate(cams):
        o = O.render(p, D, c)
        w[v][:, (o["m_value"] < MARGIN_VALUE) | (o["m_grad"] < MARGIN_VALUE)] = 0.0
    return w


@pytest.mark.parametrize("degree", [3, 0])
def test_autograd_matches_oracle_and_finite_differences(degree):
    import torch
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd.autograd import render
    p, cams = sub_scene(degree)
    w = _weights(p, degree, cams)
    ctx = G.Context(64, 2, 32, 32, 1 << 16, n_slots=2)
    P = dev(p).requires_grad_(True)
    img = render(P, cams, ctx, degree)
    loss = (img * dev(w.astype(np.float32))).sum()
    loss.backward()
    g = P.grad.cpu().numpy()
    ref, _, _ = O.render_backward(p, degree, cams, w)
    compare_grads(g, ref)
    # FP64 central differences of the oracle forward on a sample of parameters
    p64 = p.astype(np.float64)

    def L(pp):
        return sum((O.render(pp, degree, c)["image"] * w[v]).sum() for v, c in enumerate(cams))

    rng = np.random.default_rng(5)
    R = p.shape[0]
    gmax = np.abs(ref).max()
    checked = 0
    for _ in range(60):
        r, gid = int(rng.integers(R)), int(rng.integers(64))
        h = 1e-6 * max(abs(p64[r, gid]), 0.1)
        pp, pm = p64.copy(), p64.copy()
        pp[r, gid] += h
        pm[r, gid] -= h
        fd = (L(pp) - L(pm)) / (2 * h)
        if abs(fd - ref[r, gid]) > 1e-6 * gmax + 1e-5 * abs(ref[r, gid]):
            continue          # a decision flipped within +-h: not a smooth point
        assert abs(g[r, gid] - fd) <= 2e-3 * gmax + 2e-3 * abs(fd), (r, gid, g[r, gid], fd)
        checked += 1
    assert checked >= 50


def test_autograd_frozen_rows_get_zero_and_others_unchanged():
    import torch
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd.autograd import render
    p, cams = sub_scene(3)
    w = dev(_weights(p, 3, cams).astype(np.float32))
    ctx = G.Context(64, 2, 32, 32, 1 << 16, n_slots=2)
    frozen = (np.arange(64) % 4 == 1).astype(np.uint8)
    grads = []
    for fz in (None, dev(frozen)):
        P = dev(p).requires_grad_(True)
        (render(P, cams, ctx, 3, frozen=fz) * w).sum().backward()
        grads.append(P.grad.cpu().numpy())
    assert (grads[1][:, frozen == 1] == 0).all()
    np.testing.assert_array_equal(grads[1][:, frozen == 0], grads[0][:, frozen == 0])


def test_c3_batched_views_sampled_pixels():
    """1M Gaussians (SH degree 3), 4 views of 1080x1600 in one launch; 200
    sampled pixels per view against the brute-force oracle."""
    import torch
    import paper_2504_06716_amd as G
    c = S.CONFIGS["c3"]
    p = S.make_scene(c["n"], 3)
    cams = S.config_cameras("c3")[::25][:4]
    ctx = G.Context(c["n"], 4, c["height"], c["width"], instance_capacity=(1 << 31), n_slots=1)
    P = dev(p)
    img = torch.empty((4, 3, c["height"], c["width"]), device="cuda")
    ctx.render_forward(P, 3, cams, (0, 0, 0), img)
    st, need = ctx.check()
    assert st == 0, (st, need)
    from paper_2504_06716_amd import _lib as L
    Tf = torch.empty((4, c["height"], c["width"]), device="cuda")
    ctx.get_state(0, L.STATE_T_FINAL, Tf)
    img, Tf = img.cpu().numpy(), Tf.cpu().numpy()
    assert np.isfinite(img).all() and img.min() >= 0.0
    assert Tf.min() >= 1e-4 * (1 - 1e-6) and Tf.max() <= 1.0
    rng = np.random.default_rng(3)
    for v, cam in enumerate(cams):
        pix = np.stack([rng.integers(0, c["width"], 200), rng.integers(0, c["height"], 200)], 1)
        # sample around the centre of the image where the scene is
        pix[:150] = np.stack([rng.integers(600, 1000, 150), rng.integers(340, 740, 150)], 1)
        out, T, mv = O.render_pixels(p, 3, cam, pix)
        ok = mv >= MARGIN_VALUE
        got = img[v][:, pix[:, 1], pix[:, 0]].T
        assert ok.mean() > 0.95
        assert np.abs(got - out)[ok].max() <= 1e-4
        assert np.abs(Tf[v][pix[:, 1], pix[:, 0]] - T)[ok].max() <= 1e-4
        assert out[:, 0].max() > 0.05


def test_autotuner_picks_a_candidate(tmp_path):
    import torch
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd.autotune import tune
    from paper_2504_06716_amd.schedule import LearningRates
    from paper_2504_06716_amd.train import TrainConfig, render_targets
    p = S.make_scene(2000, 3, seed=2)
    cams = [S.look_at(10.0 * k, 45.0 * k, 64, 48) for k in range(4)]
    ctx = G.Context(2000, 4, 48, 64, 1 << 20)
    tgt = render_targets(ctx, S.perturb_scene(p, 3), 3, cams)
    cfg = TrainConfig(iters=40, freeze=False, lrs=LearningRates(decay_iters=40))
    cache = str(tmp_path / "tune.json")
    best = tune(p, 3, cams, tgt, S.view_order(4, 200), ctx, cfg, iters=8, cache_path=cache)
    assert best["fwd"] in (0, 1, 2, 4) and best["bwd"] in (1, 2, 4) and best["segment"] in (0, 64, 128, 256)
    assert best["variant"] in (0, 1)
    assert best["graph"] in (False, True)
    assert tune(p, 3, cams, tgt, S.view_order(4, 200), ctx, cfg, iters=8, cache_path=cache) == best


def test_views_per_step_gradient_is_the_batch_gradient():
    """Two views per step: the step's L1 gradient image is the sign of the
    residual over the whole batch, and the parameter gradient is the oracle's
    two-view gradient of that image."""
    import torch
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd.schedule import LearningRates
    from paper_2504_06716_amd.train import Trainer, TrainConfig, render_targets
    p = S.make_scene(1500, 3, seed=6)
    p[3:6] += 0.5
    cams = [S.look_at(-10.0 + 12 * k, 35.0 * k, 40, 32) for k in range(4)]
    ctx = G.Context(1500, 4, 32, 40, 1 << 20)
    tgt = render_targets(ctx, S.perturb_scene(p, 3), 3, cams)
    order = S.view_order(4, 20)
    cfg = TrainConfig(iters=10, freeze=False, lrs=LearningRates(decay_iters=10), views_per_step=2)
    tr = Trainer(p, 3, cams, tgt, cfg, order, ctx=ctx)
    tr.step()
    torch.cuda.synchronize()
    views = [int(order[0]), int(order[1])]
    img = tr.image.cpu().numpy()
    dL = tr.dL.cpu().numpy()
    t = tgt.cpu().numpy()[views]
    np.testing.assert_array_equal(dL, np.sign(img - t) * (np.float32(1) / np.float32(img.size)))
    img, dL = img.astype(np.float64), dL.astype(np.float64)
    for v in range(2):
        o = O.render(p, 3, cams[views[v]])
        ok = o["m_value"] >= MARGIN_VALUE
        assert np.abs(img[v] - o["image"])[:, ok].max() <= 1e-4
    ref, _, _ = O.render_backward(p, 3, [cams[v] for v in views], dL)
    compare_grads(tr.G.cpu().numpy(), ref)
