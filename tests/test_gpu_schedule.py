"""The trainer's schedule on the GPU (Algorithm 1; Section 3.2.2 eq. 7;
Section 3.2.3; Section 4.1): early stop fires, the plateau scheduler scales
the position learning rate the optimizer then uses, and training ends K_f
iterations after the freezing window closes -- all against the oracle's
lifecycle simulation fed with the trainer's own PSNRs."""
import numpy as np
import pytest

import oracle as O
import synthetic as S
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu


def _setup(n=1500, size=48, n_cams=4, seed=21):
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd.train import render_targets
    p = S.make_scene(n, 0, seed=seed)
    p[3:6] += 0.5
    cams = [S.look_at(-15.0 + 10 * k, 45.0 * k, size, size) for k in range(n_cams)]
    ctx = G.Context(n, n_cams, size, size, 1 << 20)
    tgt = render_targets(ctx, S.perturb_scene(p, 0), 0, cams)
    return p, cams, ctx, tgt


@pytest.mark.parametrize("graph", [False, True])
def test_early_stop_plateau_and_finetune_end(graph):
    import torch
    from paper_2504_06716_amd.schedule import FreezeSchedule, LearningRates, PlateauLR
    from paper_2504_06716_amd.train import Trainer, TrainConfig
    p, cams, ctx, tgt = _setup()
    K, Kf, every_eval = 200, 25, 10
    fs = FreezeSchedule(total_iters=K, warmup=10, every=5, reset_every=40, wait=5, window_end=150,
                        eps_xyz0=1e-5, eps_rgb0=1e-6)
    # eq. 7 with a 50 dB threshold fires at the third evaluation; the plateau
    # (improvement = more than 50 dB over the best) scales the position LR at it
    cfg = TrainConfig(iters=K, freeze=True, schedule=fs, lrs=LearningRates(decay_iters=K), eval_every=every_eval,
                      early_stop_eps=50.0, plateau=PlateauLR(0.75, 1, 50.0), finetune_iters=Kf, graph=graph,
                      device_sched=graph)
    order = S.view_order(len(cams), 400)
    tr = Trainer(p, 0, cams, tgt, cfg, order, ctx=ctx)
    tr.run(Kf + 3 * every_eval - 1)           # stops one iteration before the end
    assert not tr.finished
    P0, M0, V0 = tr.P.clone(), tr.M.clone(), tr.Vm.clone()
    frozen_before = tr.frozen.clone()
    tr.run()                                   # the last iteration
    torch.cuda.synchronize()
    sim = O.simulate_lifecycle(K, fs.warmup, fs.every, fs.reset_every, fs.wait, fs.window_end, Kf,
                               eval_every=every_eval, psnr_at=lambda k: tr.psnrs[k // every_eval - 1],
                               es_eps=50.0, plateau=O.PlateauLR(0.75, 1, 50.0))
    assert tr.stop_iter == sim["stop_iter"] == 3 * every_eval
    assert tr.k == sim["end"] == 3 * every_eval + Kf
    assert tr.finished
    acts = [a for _, a in tr.frozen_log]
    assert [(k, a) for k, a in tr.frozen_log] == [(k, a) for k, a in enumerate(sim["actions"]) if a != O.ACT_NONE]
    assert acts[-1] == O.ACT_RESET and int(tr.frozen.sum()) == 0 and int(frozen_before.sum()) == 0
    assert tr.scale_log == [(3 * every_eval, 0.75)] and sim["pos_scale"][-1] == 0.75
    # the last step's Adam used the scaled position LR: replay it on the oracle
    k_last = tr.k - 1
    lr = np.array(cfg.lrs.rows(k_last, 0, 0.75))
    g = tr.G.cpu().numpy()
    p_ref, _, _ = O.adam_masked(P0.cpu().numpy(), g, M0.cpu().numpy(), V0.cpu().numpy(), lr, 0.9, 0.999, 1e-15,
                                tr.step_count, None)
    got = tr.P.cpu().numpy()
    np.testing.assert_allclose(got, p_ref, rtol=1e-5, atol=1e-7)
    lr1 = np.array(cfg.lrs.rows(k_last, 0, 1.0))
    p_unscaled, _, _ = O.adam_masked(P0.cpu().numpy(), g, M0.cpu().numpy(), V0.cpu().numpy(), lr1, 0.9, 0.999,
                                     1e-15, tr.step_count, None)
    moved = np.abs(p_unscaled[0:3] - P0.cpu().numpy()[0:3]).max()
    assert np.abs(got[0:3] - p_unscaled[0:3]).max() > 0.1 * moved


def test_trainer_raises_on_device_flag():
    """An instance-capacity overflow during training (forced from the host
    with a tiny capacity; the kernels bound-check and flag it) stops the
    trainer at the next freeze-map change instead of training on."""
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd import _lib
    from paper_2504_06716_amd.schedule import FreezeSchedule, LearningRates
    from paper_2504_06716_amd.train import Trainer, TrainConfig
    p, cams, ctx, tgt = _setup()
    small = G.Context(p.shape[1], len(cams), 48, 48, 256)
    fs = FreezeSchedule(total_iters=40, warmup=4, every=2, reset_every=100, wait=2, window_end=30,
                        eps_xyz0=1e-5, eps_rgb0=1e-6)
    cfg = TrainConfig(iters=40, freeze=True, schedule=fs, lrs=LearningRates(decay_iters=40))
    tr = Trainer(p, 0, cams, tgt, cfg, S.view_order(len(cams), 40), ctx=small)
    with pytest.raises(_lib.GstaError) as ei:
        tr.run(10)
    assert ei.value.status == _lib.GSTA_ERR_CAPACITY
    assert tr.k == 4                    # raised at the first freeze update, before iteration 4 ran


def test_evaluate_psnr_from_library_sums_matches_oracle():
    """Validation PSNR (10 log10(count / SSE) of the clamped image, mean over
    views) computed from gsta_l1_loss's sums equals the oracle's PSNR of the
    same images."""
    import torch
    from paper_2504_06716_amd.schedule import LearningRates
    from paper_2504_06716_amd.train import Trainer, TrainConfig
    p, cams, ctx, tgt = _setup()
    cfg = TrainConfig(iters=5, freeze=False, lrs=LearningRates(decay_iters=5))
    tr = Trainer(p, 0, cams, tgt, cfg, S.view_order(len(cams), 5), ctx=ctx)
    tr.run(3)
    got = tr.evaluate([0, 2, 3])
    img = tr.render_views([0, 2, 3]).cpu().numpy().astype(np.float64)
    t = tgt.cpu().numpy().astype(np.float64)
    ref = np.mean([O.psnr(O.l1_loss(img[i], t[v])[2]) for i, v in enumerate([0, 2, 3])])
    assert got == pytest.approx(ref, abs=1e-9)
    torch.cuda.synchronize()
