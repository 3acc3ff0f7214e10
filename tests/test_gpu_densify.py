"""Densification, pruning and opacity reset through the C ABI against the
oracle: decisions and copies bit-exact, split children to float32 rounding;
the densification statistics accumulated by the backward to the gradient
tolerance."""
import math

import numpy as np
import pytest

import oracle as O
import synthetic as S
from tests.gpu_util import GRAD_REL, MARGIN_RECT_PX, MARGIN_VALUE, dev

pytestmark = pytest.mark.gpu

SPLIT_LS = math.log(0.01 * 4.0)
PRUNE_LG = math.log(0.005 / 0.995)
SHIFT = math.log(1.6)


def _case(n, degree=3, seed=0):
    rng = np.random.default_rng(seed)
    p = S.make_scene(n, degree, seed=seed).astype(np.float32)
    p[3:6] += rng.uniform(-0.5, 1.8, (1, n)).astype(np.float32)           # mix of small and big
    p[10] = rng.uniform(-6.5, 3.0, n).astype(np.float32)                  # some below the prune logit
    st = np.zeros((4, n), np.float32)
    st[1] = rng.integers(0, 4, n)
    st[0] = (rng.exponential(2e-4, n) * st[1]).astype(np.float32)
    st[3] = np.minimum(st[1], 2)
    st[2] = (rng.exponential(1e-6, n) * st[3]).astype(np.float32)
    frozen = (rng.random(n) < 0.15).astype(np.uint8)
    ema = rng.exponential(1e-4, (4, n)).astype(np.float32)
    M = rng.standard_normal(p.shape).astype(np.float32)
    V = np.abs(rng.standard_normal(p.shape)).astype(np.float32)
    noise = rng.standard_normal((6, n)).astype(np.float32)
    return p, M, V, ema, frozen, st, noise


def _cfg(thr=2e-4, rgb=1e-6, use_rgb=False):
    from paper_2504_06716_amd._lib import DensifyCfg
    return DensifyCfg(thr, rgb, int(use_rgb), SPLIT_LS, PRUNE_LG, SHIFT)


def _run(ctx, degree, p, M, V, ema, frozen, st, noise, cfg, cap, pad=0):
    """noise None: the kernel draws the children's normals (cfg.noise_seed, noise_draw)."""
    import torch
    R, n = p.shape
    ld = cap + pad
    outs = [torch.full((R, ld), -7.0, device="cuda")[:, :cap] for _ in range(3)]
    ema_o = torch.full((4 * cap,), -7.0, device="cuda")
    fz_o = torch.full((cap,), 9, dtype=torch.uint8, device="cuda")
    counts = torch.zeros(4, dtype=torch.int64, device="cuda")
    ins = [dev(x)[:, :n] if x.ndim == 2 else dev(x) for x in (p, M, V)]
    ctx.densify_prune(ins[0], ins[1], ins[2], degree, None if ema is None else dev(ema),
                      None if frozen is None else dev(frozen), dev(st), None if noise is None else dev(noise), cfg,
                      outs[0], outs[1], outs[2], ema_o, fz_o, counts)
    torch.cuda.synchronize()
    c = tuple(int(x) for x in counts.cpu())
    return c, [o.cpu().numpy() for o in outs], ema_o.cpu().numpy(), fz_o.cpu().numpy()


@pytest.mark.parametrize("n,degree,use_rgb,with_state", [(5003, 3, False, True), (5003, 3, True, True),
                                                         (257, 0, True, False), (1, 3, False, True)])
def test_densify_prune_matches_oracle(n, degree, use_rgb, with_state):
    import paper_2504_06716_amd as G
    p, M, V, ema, frozen, st, noise = _case(n, degree)
    if n == 1:
        st[:, 0] = [1.0, 1.0, 0.0, 1.0]
        p[3:6, 0], p[10, 0] = 0.0, 1.0          # big and live: split into two
        frozen[0] = 0
    if not with_state:
        ema, frozen = None, None
    ctx = G.Context(3 * n + 64, 1, 16, 16, 16)
    cfg = _cfg(use_rgb=use_rgb)
    cap = 3 * n + 5
    counts, (gP, gM, gV), gE, gF = _run(ctx, degree, p, M, V, ema, frozen, st, noise, cfg, cap, pad=3)
    oP, oM, oV, oE, oF, oc = O.densify_prune(p, M, V, ema, frozen, st, noise, 2e-4, 1e-6, use_rgb,
                                             SPLIT_LS, PRUNE_LG, SHIFT)
    assert counts == oc
    n_out, K, C, Sp = oc
    if n > 1:
        assert K > 0 and C > 0 and Sp > 0 and K + Sp < n            # every rule is exercised
    nc = K + C
    np.testing.assert_array_equal(gP[:, :nc], oP[:, :nc].astype(np.float32))
    np.testing.assert_array_equal(gM[:, :n_out], oM.astype(np.float32))
    np.testing.assert_array_equal(gV[:, :n_out], oV.astype(np.float32))
    np.testing.assert_array_equal(gE[:4 * n_out].reshape(4, n_out), oE.astype(np.float32))
    np.testing.assert_array_equal(gF[:n_out], oF)
    # children: copies exact, positions and log-scales to float32 rounding
    ch, oc_ = gP[:, nc:n_out].astype(np.float64), oP[:, nc:]
    np.testing.assert_array_equal(ch[6:], oc_[6:])
    assert np.all(np.abs(ch[0:3] - oc_[0:3]) <= 1e-6 * (np.abs(oc_[0:3]) + 1.0))
    np.testing.assert_allclose(ch[3:6], oc_[3:6], rtol=1e-6, atol=1e-6)
    # untouched tail of the outputs
    assert (gP[:, n_out:] == -7.0).all() and (gF[n_out:] == 9).all()


@pytest.mark.parametrize("draw", [0, 1234])
def test_densify_noise_drawn_in_kernel_matches_oracle(draw):
    """With noise NULL the split children's normals come from
    Philox4x64-10 (seed, draw, column) + Box-Muller in the kernel: children
    equal the oracle's, given the oracle's draws, to float32 rounding."""
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd._lib import DensifyCfg
    n = 1500
    p, M, V, ema, frozen, st, _ = _case(n, 3, seed=7)
    ctx = G.Context(3 * n + 64, 1, 16, 16, 16)
    cfg = DensifyCfg(2e-4, 1e-6, 0, SPLIT_LS, PRUNE_LG, SHIFT, 2 ** 40 + 9, draw)
    cap = 3 * n + 5
    counts, (gP, _, _), _, _ = _run(ctx, 3, p, M, V, ema, frozen, st, None, cfg, cap)
    noise = O.densify_noise(n, 2 ** 40 + 9, draw)
    oP, _, _, _, _, oc = O.densify_prune(p, M, V, ema, frozen, st, noise, 2e-4, 1e-6, False, SPLIT_LS, PRUNE_LG,
                                         SHIFT)
    assert counts == oc and oc[3] > 20
    n_out, K, C, _ = oc
    ch, oc_ = gP[:, K + C:n_out].astype(np.float64), oP[:, K + C:]
    np.testing.assert_array_equal(gP[:, :K + C], oP[:, :K + C].astype(np.float32))
    assert np.all(np.abs(ch[0:3] - oc_[0:3]) <= 1e-6 * (np.abs(oc_[0:3]) + 1.0))
    np.testing.assert_array_equal(ch[6:], oc_[6:])
    # the children moved away from their parents (non-trivial draws)
    _, split, live = O.densify_decisions(st, p, frozen, 2e-4, 1e-6, False, SPLIT_LS, PRUNE_LG)
    parents = p[0:3, np.flatnonzero(split & live)].astype(np.float64)
    S_ = parents.shape[1]
    assert np.abs(ch[0:3, :S_] - parents).max() > 1e-4 and np.abs(ch[0:3, S_:2 * S_] - parents).max() > 1e-4


def test_densify_capacity_overflow_writes_nothing_and_is_reported():
    import paper_2504_06716_amd as G
    p, M, V, ema, frozen, st, noise = _case(3000)
    oc = O.densify_prune(p, M, V, ema, frozen, st, noise, 2e-4, 1e-6, False, SPLIT_LS, PRUNE_LG, SHIFT)[5]
    ctx = G.Context(4000, 1, 16, 16, 16)
    counts, (gP, _, _), gE, gF = _run(ctx, 3, p, M, V, ema, frozen, st, noise, _cfg(), cap=oc[0] - 1)
    assert counts == oc
    assert (gP == -7.0).all() and (gE == -7.0).all() and (gF == 9).all()
    assert ctx.check()[0] == 2                      # GSTA_ERR_CAPACITY
    assert ctx.check()[0] == 0                      # flags are cleared by the report


def test_densify_empty_and_all_pruned():
    import torch
    import paper_2504_06716_amd as G
    ctx = G.Context(600, 1, 16, 16, 16)
    p, M, V, ema, frozen, st, noise = _case(500)
    p[10] = -9.0                                    # everything below the prune logit
    counts, (gP, _, _), _, _ = _run(ctx, 3, p, M, V, ema, frozen, st, noise, _cfg(), cap=600)
    assert counts == (0, 0, 0, 0) and (gP == -7.0).all()
    z = np.zeros((59, 0), np.float32)
    counts, *_ = _run(ctx, 3, z, z, z, np.zeros((4, 0), np.float32), np.zeros(0, np.uint8),
                      np.zeros((4, 0), np.float32), np.zeros((6, 0), np.float32), _cfg(), cap=10)
    assert counts == (0, 0, 0, 0)
    with pytest.raises(G.GstaError):                # output overlapping the input is refused
        P = dev(p)
        ctx.densify_prune(P, dev(M), dev(V), 3, None, None, dev(st), dev(noise), _cfg(), P, dev(M), dev(V),
                          None, None, torch.zeros(4, dtype=torch.int64, device="cuda"))


def test_opacity_reset_matches_oracle():
    import torch
    import paper_2504_06716_amd as G
    p, M, V, _, frozen, _, _ = _case(3001)
    ctx = G.Context(3001, 1, 16, 16, 16)
    P, Mt, Vt = dev(p), dev(M), dev(V)
    cap = math.log(0.01 / 0.99)
    ctx.opacity_reset(P, Mt, Vt, 3, dev(frozen), cap)
    torch.cuda.synchronize()
    oP, oM, oV = O.opacity_reset(p, M, V, frozen, cap)
    np.testing.assert_array_equal(P.cpu().numpy(), oP.astype(np.float32))
    np.testing.assert_array_equal(Mt.cpu().numpy(), oM.astype(np.float32))
    np.testing.assert_array_equal(Vt.cpu().numpy(), oV.astype(np.float32))


def test_densify_stats_match_oracle():
    """Two backward calls (two views each) accumulate the statistics."""
    import torch
    import paper_2504_06716_amd as G
    n = 300
    p = S.make_scene(n, 3, seed=3).astype(np.float64)
    p[3:6] += 0.7
    cams = [S.look_at(10.0 + 30.0 * k, 15.0 + 60.0 * k, 48, 40) for k in range(4)]
    rng = np.random.default_rng(9)
    frozen = (rng.random(n) < 0.2).astype(np.uint8)
    ctx = G.Context(n, 2, 40, 48, 1 << 18)
    P = dev(p.astype(np.float32))
    dst = torch.zeros((4, n), device="cuda")
    acc = np.zeros((4, n))
    excl = np.zeros(n, bool)
    for b in range(2):
        cs = cams[2 * b:2 * b + 2]
        w = rng.standard_normal((2, 3, 40, 48))
        for v, c in enumerate(cs):
            o = O.render(p, 3, c)
            w[v][:, (o["m_value"] < MARGIN_VALUE) | (o["m_grad"] < MARGIN_VALUE)] = 0.0
            rec = O.project(p, 3, c)
            excl |= rec[:, 27] < MARGIN_RECT_PX
        img = torch.empty((2, 3, 40, 48), device="cuda")
        ctx.render_forward(P, 3, cs, (0, 0, 0), img)
        grad = torch.zeros((59, n), device="cuda")
        ctx.render_backward(P, 3, cs, (0, 0, 0), 0, dev(w.astype(np.float32)), dev(frozen), grad, dstats=dst)
        g, g2, vis = O.render_backward(p, 3, cs, w, frozen)
        acc = O.densify_stats(acc, g2, vis, g, frozen, 48, 40)
    got = dst.cpu().numpy().astype(np.float64)
    keep = ~excl
    np.testing.assert_array_equal(got[1][keep], acc[1][keep])
    np.testing.assert_array_equal(got[3][keep], acc[3][keep])
    assert (got[:, frozen == 1] == 0).all()
    for r in (0, 2):
        a, b = got[r][keep], acc[r][keep]
        assert np.linalg.norm(a - b) <= GRAD_REL * np.linalg.norm(b)
        assert np.all(np.abs(a - b) <= GRAD_REL * np.abs(b) + GRAD_REL * np.abs(b).max())
    assert (acc[1] > 0).sum() > 100


def _dens_trainer(graph, iters=90, n=1500):
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd.schedule import DensifySchedule, FreezeSchedule, LearningRates
    from paper_2504_06716_amd.train import Trainer, TrainConfig, render_targets
    p = S.make_scene(n, 3, seed=11)
    cams = [S.look_at(-15.0 + 10 * k, 45.0 * k, 48, 40) for k in range(8)]
    ctx = G.Context(12 * n, 8, 40, 48, 1 << 20)
    tgt = render_targets(ctx, S.perturb_scene(p, 3, seed=12), 3, cams)
    ds = DensifySchedule(total_iters=iters, start=20, stop=60, every=20, reset_every=40, eps_xyz0=1e-4)
    fs = FreezeSchedule(total_iters=iters, warmup=10, every=10, reset_every=50, wait=10, window_end=70,
                        eps_xyz0=1e-6, eps_rgb0=1e-7)
    cfg = TrainConfig(iters=iters, freeze=True, schedule=fs, lrs=LearningRates(decay_iters=iters),
                      densify=ds, max_gaussians=12 * n, graph=graph, device_sched=True)
    tr = Trainer(p, 3, cams, tgt, cfg, S.view_order(8, iters), ctx=ctx)
    return tr


def test_trainer_densify_changes_n_and_graph_replay_matches_eager():
    """A densifying run (clone, split, prune, opacity reset, freezing) gives
    the same Gaussians eager and with HIP graphs captured again after every
    change of N."""
    import torch
    out = []
    for graph in (False, True):
        tr = _dens_trainer(graph)
        tr.run(41)                                   # densify at 20 and 40, opacity reset at 40
        p0 = tr.evaluate()
        tr.run(49)
        torch.cuda.synchronize()
        out.append((tr.n, tr.n_history, tr.P.cpu().numpy(), tr.frozen.cpu().numpy(), tr.evaluate(), p0))
    (n0, h0, P0, F0, e0, s0), (n1, h1, P1, F1, e1, _) = out
    print("N after each densify step:", h0, "PSNR after the reset", s0, "at the end", e0)
    assert len(h0) == 2 and h0 == h1 and n0 == n1
    assert any(b != a for (_, a), (_, b) in zip([(0, 1500)] + h0[:-1], h0))
    np.testing.assert_array_equal(P0, P1)
    np.testing.assert_array_equal(F0, F1)
    assert e0 > s0 + 1.0                             # it trains on after the reset


def test_c4_scale_training_with_densify_freeze_and_partition():
    """c4 sizes: 3M Gaussians (SH degree 3) at 1080x1920.  The first forward
    matches the brute-force oracle on sampled pixels; then a few training
    iterations with densification, a freeze update with the partitioned
    layout, and Adam run to finite parameters with the active Gaussians as
    the prefix."""
    import torch
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd.schedule import UPDATE, DensifySchedule, FreezeSchedule, LearningRates
    from paper_2504_06716_amd.train import Trainer, TrainConfig, render_targets, required_capacity
    c = S.CONFIGS["c4"]
    n, H, W = c["n"], c["height"], c["width"]
    p = S.make_scene(n, 3)
    cams = S.config_cameras("c4")[::30][:5]
    cap = 2 * n
    ctx = G.Context(cap, 1, H, W, instance_capacity=1 << 24, n_slots=1)
    pt = S.perturb_scene(p, 3)
    need = max(required_capacity(ctx, p, 3, cams), required_capacity(ctx, pt, 3, cams))
    print("c4 instances per view (max):", need, flush=True)
    ctx.reserve(instance_capacity=int(need * 1.5) + 4096)
    tgt = render_targets(ctx, pt, 3, cams)
    iters = 8
    ds = DensifySchedule(total_iters=iters, start=2, stop=6, every=2, reset_every=100, eps_xyz0=2e-4)
    fs = FreezeSchedule(total_iters=iters, warmup=3, every=2, reset_every=100, wait=1, window_end=7,
                        eps_xyz0=1e-7, eps_rgb0=1e-9)
    cfg = TrainConfig(iters=iters, freeze=True, schedule=fs, lrs=LearningRates(decay_iters=iters),
                      densify=ds, max_gaussians=cap, partition=True)
    tr = Trainer(p, 3, cams, tgt, cfg, np.arange(iters) % len(cams), ctx=ctx)
    # the first forward, on sampled pixels against the oracle
    img = tr.render_views([0])[0].cpu().numpy()
    rng = np.random.default_rng(5)
    pix = np.stack([rng.integers(700, 1220, 120), rng.integers(280, 800, 120)], 1)
    out, _, mv = O.render_pixels(p, 3, cams[0], pix)
    ok = mv >= MARGIN_VALUE
    assert ok.mean() > 0.95
    assert np.abs(img[:, pix[:, 1], pix[:, 0]].T - out)[ok].max() <= 1e-4
    checked = 0
    for k in range(iters):
        tr.step()
        if tr.frozen_log and tr.frozen_log[-1] == (k, UPDATE):
            torch.cuda.synchronize()
            f = tr.frozen.cpu().numpy()
            assert (np.diff(f.astype(np.int8)) >= 0).all()
            checked += 1
    torch.cuda.synchronize()
    print("N after each densify step:", tr.n_history, "frozen:", tr.freeze_history(), flush=True)
    assert checked >= 1 and len(tr.n_history) >= 1 and tr.n_history[0][1] != n
    assert np.isfinite(tr.P.cpu().numpy()).all()
    assert np.isfinite(tr.evaluate([0, 1]))
    st, _ = ctx.check()
    assert st == 0
