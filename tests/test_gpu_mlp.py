"""Learned freeze proposer through the C ABI against the oracle: trajectory
push, feature statistics and features, the bf16 matrix-core MLP forward,
BCE, weight gradients, Adam and the propose/veto step."""
import math

import numpy as np
import pytest

import oracle as O
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu


def bits(v):
    """bf16 bit patterns (as int16) of values that are already bf16."""
    return (np.asarray(v, np.float32).view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def from_bits(b):
    return (np.asarray(b).view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _weights(seed=0):
    rng = np.random.default_rng(seed)
    wf = np.zeros(O.MLP_COUNT)
    o = O.MLP_OFF
    wf[o["W1"]:o["b1"]] = rng.standard_normal(2048) / np.sqrt(32)
    wf[o["b1"]:o["W2"]] = 0.1 * rng.standard_normal(64)
    wf[o["W2"]:o["b2"]] = rng.standard_normal(4096) / 8.0
    wf[o["b2"]:o["w3"]] = 0.1 * rng.standard_normal(64)
    wf[o["w3"]:o["b3"]] = rng.standard_normal(64) / 8.0
    wf[o["b3"]] = 0.3
    return wf.astype(np.float32)


def _ctx():
    import paper_2504_06716_amd as G
    return G.Context(1024, 1, 16, 16, 16)


def _dev_weights(ctx, wf):
    import torch
    w = dev(wf.astype(np.float32))
    wb = torch.zeros(6144, dtype=torch.int16, device="cuda")
    ctx.mlp_sync_bf16(w, wb)
    return w, wb


def test_bf16_copy_and_push():
    import torch
    ctx = _ctx()
    wf = _weights()
    w, wb = _dev_weights(ctx, wf)
    o = O.MLP_OFF
    exp = np.concatenate([O.bf16_round(wf[o["W1"]:o["b1"]]), O.bf16_round(wf[o["W2"]:o["b2"]])])
    np.testing.assert_array_equal(from_bits(wb.cpu().numpy()), exp)
    n = 1001
    rng = np.random.default_rng(1)
    ema = (10.0 ** rng.uniform(-12, 2, (4, n))).astype(np.float32)
    ema[:, :5] = O.FLT_MAX                           # never seen
    ring = torch.zeros((8, 4, n), dtype=torch.int16, device="cuda")
    ctx.traj_push(dev(ema), ring, 3)
    got = from_bits(ring[3].cpu().numpy())
    np.testing.assert_array_equal(got, O.bf16_round(np.minimum(ema, np.float32(1e30))))
    assert (ring[2].cpu().numpy() == 0).all()


def _ring(n, seed=2):
    rng = np.random.default_rng(seed)
    vals = O.bf16_round(10.0 ** rng.uniform(-10, -2, (8, 4, n)))
    vals[:, :, :3] = 0.0
    return vals


def test_features_and_statistics():
    import torch
    ctx = _ctx()
    n = 3000
    ring = _ring(n)
    R = dev(bits(ring).reshape(8, 4, n))
    sums = torch.zeros(64, dtype=torch.float64, device="cuda")
    ctx.mlp_feature_stats(R, 5, sums)
    ctx.mlp_feature_stats(R, 2, sums)
    raw = []
    for h in (5, 2):
        x = np.zeros((n, 32))
        for j in range(8):
            for q in range(4):
                x[:, 4 * j + q] = np.log10(ring[(h - j) % 8, q] + 1e-12)
        raw.append(x)
    raw = np.concatenate(raw)
    s = sums.cpu().numpy()
    np.testing.assert_allclose(s[:32], raw.sum(0), rtol=1e-6)
    np.testing.assert_allclose(s[32:], (raw ** 2).sum(0), rtol=1e-6)
    mean = raw.mean(0).astype(np.float32)
    std = raw.std(0).astype(np.float32)
    x = torch.zeros((n, 32), dtype=torch.int16, device="cuda")
    ctx.mlp_features(R, 5, dev(mean), dev(std), x)
    got = from_bits(x.cpu().numpy())
    exp = O.traj_features(ring, 5, mean.astype(np.float64), std.astype(np.float64))
    # float32 log10 and division (relative error ~1e-7 of |log10 r| ~ 12, then
    # divided by std) vs float64, then the same bf16 rounding: one bf16 step
    # apart at most, or 1e-5 near zero
    tol = np.maximum(np.abs(exp) * 2.0 ** -7, 1e-5)
    assert (np.abs(got - exp) <= tol).all()
    assert (got == exp).mean() > 0.99


def _forward(ctx, wf, x, save=True):
    import torch
    n = x.shape[0]
    w, wb = _dev_weights(ctx, wf)
    X = dev(bits(x))
    z = torch.zeros(n, device="cuda")
    h1 = torch.zeros((n, 64), dtype=torch.int16, device="cuda") if save else None
    h2 = torch.zeros((n, 64), device="cuda") if save else None
    ctx.mlp_forward(wb, w, X, z, h1, h2)
    torch.cuda.synchronize()
    return w, wb, X, z, h1, h2


@pytest.mark.parametrize("n", [1, 17, 4099])
def test_mlp_forward_matches_oracle(n):
    ctx = _ctx()
    wf = _weights(3)
    x = O.bf16_round(np.random.default_rng(4).standard_normal((n, 32)))
    _, _, _, z, h1, h2 = _forward(ctx, wf, x)
    oz, oh1, oh2 = O.mlp_forward(x, wf.astype(np.float64))
    gh1 = from_bits(h1.cpu().numpy())
    # h1: float32 accumulation vs float64 may round to the neighbouring bf16 value
    assert (np.abs(gh1 - oh1) <= np.abs(oh1) * 2.0 ** -7).all()
    assert (gh1 == oh1).mean() > 0.999
    W1, b1, W2, b2, w3, b3 = O.mlp_unpack(wf)
    # one bf16 step of one h1 entry moves z by at most 2^-8 |h1_v| sum_u |w3_u W2b_uv|
    flip = 2.0 ** -8 * (np.abs(oh1) * (np.abs(w3) @ np.abs(O.bf16_round(W2)))[None, :]).max(1)
    tol = 1e-5 * (1.0 + np.abs(oh2) @ np.abs(w3)) + flip
    assert (np.abs(z.cpu().numpy() - oz) <= tol).all()
    exact = (gh1 == oh1).all(1)
    assert (np.abs(z.cpu().numpy() - oz)[exact] <= 1e-5 * (1.0 + np.abs(oh2[exact]) @ np.abs(w3))).all()


def test_mlp_bce_matches_oracle():
    import torch
    ctx = _ctx()
    n = 5000
    rng = np.random.default_rng(6)
    z = (rng.standard_normal(n) * 4).astype(np.float32)
    y = (rng.random(n) < 0.3).astype(np.uint8)
    dz = torch.zeros(n, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    ctx.mlp_bce(dev(z), dev(y), dz, loss)
    ol, odz = O.bce(z.astype(np.float64), y)
    assert float(loss.cpu()) == pytest.approx(ol, rel=1e-6)
    # sigmoid in float32 (relative error ~1e-7 of a value <= 1), minus y, over n
    assert (np.abs(dz.cpu().numpy() - odz) <= 1e-6 * np.abs(odz) + 2e-7 / n).all()


@pytest.mark.parametrize("n", [5, 5000, 33, 200_000])
def test_mlp_backward_matches_oracle(n):
    import torch
    ctx = _ctx()
    wf = _weights(5)
    rng = np.random.default_rng(8)
    x = O.bf16_round(rng.standard_normal((n, 32)))
    dzn = (rng.standard_normal(n) / n).astype(np.float32)
    w, wb, X, z, h1, h2 = _forward(ctx, wf, x)
    grad = torch.zeros(O.MLP_COUNT, device="cuda")
    ctx.mlp_backward(wb, w, X, h1, h2, dev(dzn), grad)
    g = grad.cpu().numpy().astype(np.float64)
    og = O.mlp_backward(x, wf.astype(np.float64), dzn.astype(np.float64))
    for name, (a, b) in {"W1": (0, 2048), "b1": (2048, 2112), "W2": (2112, 6208), "b2": (6208, 6272),
                         "w3": (6272, 6336), "b3": (6336, 6337)}.items():
        d = g[a:b] - og[a:b]
        assert np.linalg.norm(d) <= 1e-3 * np.linalg.norm(og[a:b]) + 1e-12, name
    grad2 = torch.zeros_like(grad)
    ctx.mlp_backward(wb, w, X, h1, h2, dev(dzn), grad2)
    assert torch.equal(grad, grad2)                  # fixed summation order


def test_mlp_adam_matches_oracle():
    import torch
    ctx = _ctx()
    rng = np.random.default_rng(9)
    wf = _weights(6)
    g = (rng.standard_normal(O.MLP_COUNT) * 1e-2).astype(np.float32)
    m0 = (rng.standard_normal(O.MLP_COUNT) * 1e-3).astype(np.float32)
    v0 = (np.abs(rng.standard_normal(O.MLP_COUNT)) * 1e-6).astype(np.float32)
    w, wb = _dev_weights(ctx, wf)
    m, v = dev(m0), dev(v0)
    ctx.mlp_adam(w, dev(g), m, v, 1e-3, 0.9, 0.999, 1e-8, 3, wb)
    torch.cuda.synchronize()
    P, M, V = O.adam_masked(wf[None].astype(np.float64), g[None].astype(np.float64), m0[None].astype(np.float64),
                            v0[None].astype(np.float64), np.array([1e-3]), float(np.float32(0.9)),
                            float(np.float32(0.999)), 1e-8, 3)
    np.testing.assert_allclose(w.cpu().numpy(), P[0], rtol=1e-6, atol=1e-9)
    # m = b1 m + (1 - b1) g in float32: bounded by the operands, not the (cancelling) result
    b1 = float(np.float32(0.9))
    assert (np.abs(m.cpu().numpy() - M[0]) <= 4e-7 * (b1 * np.abs(m0) + (1 - b1) * np.abs(g))).all()
    o = O.MLP_OFF
    wn = w.cpu().numpy()
    np.testing.assert_array_equal(from_bits(wb.cpu().numpy())[:2048], O.bf16_round(wn[:2048]))
    np.testing.assert_array_equal(from_bits(wb.cpu().numpy())[2048:], O.bf16_round(wn[o["W2"]:o["b2"]]))


def test_mlp_propose_matches_oracle():
    import torch
    ctx = _ctx()
    n = 2049
    rng = np.random.default_rng(7)
    z = rng.standard_normal(n).astype(np.float32) * 3
    sx = (10.0 ** rng.uniform(-7, -3, n)).astype(np.float32)
    sr = (10.0 ** rng.uniform(-8, -2, n)).astype(np.float32)
    thr = math.log(9.0)
    prop = torch.zeros(n, dtype=torch.uint8, device="cuda")
    ctx.mlp_propose(dev(z), dev(sx), dev(sr), thr, 9e-5, 3e-4, prop)
    exp = O.propose(z, sx, sr, thr, 9e-5, 3e-4)
    np.testing.assert_array_equal(prop.cpu().numpy(), exp)
    assert 0 < exp.sum() < n


def test_proposer_end_to_end_training_run():
    """Log a rule-only run, train the proposer on the rule's own future
    decisions, then train again with proposals: the BCE falls, accepted
    proposals only add to the rule's map, and the vetoed ones stay out."""
    import torch
    import paper_2504_06716_amd as G
    import synthetic as S
    from paper_2504_06716_amd.proposer import Proposer, ProposerDataset
    from paper_2504_06716_amd.schedule import FreezeSchedule, LearningRates, UPDATE
    from paper_2504_06716_amd.train import Trainer, TrainConfig, render_targets
    n, iters = 3000, 300
    p = S.make_scene(n, 3, seed=13)
    p[3:6] += 0.4
    cams = [S.look_at(-20.0 + 8 * k, 45.0 * k, 48, 40) for k in range(8)]
    ctx = G.Context(n, 8, 40, 48, 1 << 20)
    tgt = render_targets(ctx, S.perturb_scene(p, 3, seed=14), 3, cams)
    order = S.view_order(8, iters)
    sched = FreezeSchedule(total_iters=iters, warmup=60, every=20, reset_every=200, wait=20, window_end=260,
                           eps_xyz0=2e-6, eps_rgb0=5e-8)

    def cfg(**kw):
        return TrainConfig(iters=iters, freeze=True, schedule=sched, lrs=LearningRates(decay_iters=iters),
                           traj_every=5, **kw)

    ds = ProposerDataset(ctx, n)
    tr = Trainer(p, 3, cams, tgt, cfg(dataset=ds), order, ctx=ctx)
    tr.run(iters)
    prop = Proposer(ctx)
    x, y = ds.build(prop)
    assert 0.02 < float(y.float().mean()) < 0.98
    hist = prop.fit(x, y, epochs=150, lr=3e-3)
    print("bce", hist[0], hist[-1])
    assert hist[-1][1] < 0.8 * hist[0][1]
    # one update with proposals on the logged state: proposals only add, vetoes hold
    t2 = Trainer(p, 3, cams, tgt, cfg(proposer=prop), order, ctx=ctx)
    t2.run(sched.warmup)                     # up to the first update
    ema = t2.ema.clone()
    ex, er = sched.thresholds(sched.warmup, sched.window_close())
    assert sched.action(sched.warmup) == UPDATE
    t2.run(1)
    torch.cuda.synchronize()
    frz = t2.frozen.cpu().numpy()
    e = ema.cpu().numpy()
    rule = ((e[0] < np.float32(ex)) & (e[1] < np.float32(er))).astype(np.uint8)   # the rule's own condition
    assert (frz >= rule).all()
    extra = (frz == 1) & (rule == 0)
    assert (e[0][extra] < np.float32(3 * ex)).all() and (e[1][extra] < np.float32(3 * er)).all()
    print("rule froze", int(rule.sum()), "proposals added", int(extra.sum()))
    t2.run(iters - sched.warmup - 1)
    assert np.isfinite(t2.evaluate())


def test_proposer_inference_at_c5_scale():
    """The c5 workload's proposer step at its size: features of 3M Gaussians
    from an 8-deep ring and logits on the matrix cores, against the oracle
    on 4000 sampled Gaussians (features within one bf16 step, logits to the
    forward test's bound)."""
    import time
    import torch
    n = 3_000_000
    ctx = _ctx()
    rng = np.random.default_rng(17)
    ring_v = O.bf16_round(np.exp(rng.normal(-9.0, 2.0, (8, 4, n))))
    ring = dev(bits(ring_v))
    mean_np = rng.normal(-4.0, 0.1, 32).astype(np.float32)
    std_np = rng.uniform(0.5, 1.5, 32).astype(np.float32)
    wf = _weights(7)
    w, wb = _dev_weights(ctx, wf)
    x = torch.empty((n, 32), dtype=torch.int16, device="cuda")
    z = torch.empty(n, device="cuda")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.mlp_features(ring, 5, dev(mean_np), dev(std_np), x)
    ctx.mlp_forward(wb, w, x, z)
    torch.cuda.synchronize()
    print(f"c5 proposer inference: {n} Gaussians in {(time.perf_counter() - t0) * 1e3:.2f} ms", flush=True)
    idx = rng.choice(n, 4000, replace=False)
    xo = O.traj_features(ring_v[:, :, idx], 5, mean_np.astype(np.float64), std_np.astype(np.float64))
    xg = from_bits(x.cpu().numpy()[idx])
    assert (np.abs(xg - xo) <= np.maximum(np.abs(xo) * 2.0 ** -7, 1e-5)).all()
    oz, oh1, oh2 = O.mlp_forward(xg, wf.astype(np.float64))
    W1, b1, W2, b2, w3, b3 = O.mlp_unpack(wf)
    flip = 2.0 ** -8 * (np.abs(oh1) * (np.abs(w3) @ np.abs(O.bf16_round(W2)))[None, :]).max(1)
    tol = 1e-5 * (1.0 + np.abs(oh2) @ np.abs(w3)) + flip
    assert (np.abs(z.cpu().numpy()[idx] - oz) <= tol).all()
