"""The ablation's freezing rules on the GPU (Section 4.3, Table 3: "+mingrad"
and "+random") against the oracle, bit for bit: masks, counts, both
accumulation modes, ties, never-seen Gaussians, empty and ragged sizes; and
a training run with each rule."""
import numpy as np
import pytest

import oracle as O
import synthetic as S
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu


def _scores(n, seed):
    rng = np.random.default_rng(seed)
    s = (np.round(rng.random(n) * 40) / 4000).astype(np.float32)      # many equal values
    s[rng.random(n) < 0.1] = np.float32(O.FLT_MAX)                     # never seen
    s[rng.random(n) < 0.05] = np.float32(0.0)
    neg0 = rng.random(n) < 0.05
    s[neg0] = np.float32(-0.0)                                          # equal to +0: ties by index
    return s


@pytest.mark.parametrize("n", [0, 1, 7, 257, 3001, 100_000])
@pytest.mark.parametrize("fraction", [0.0, 0.25, 0.5, 1.0])
@pytest.mark.parametrize("mode", [0, 2])
def test_mingrad_matches_oracle(n, fraction, mode):
    import torch
    import paper_2504_06716_amd as G
    print(f"mingrad n={n} fraction={fraction} mode={mode}", flush=True)
    ctx = G.Context(max(n, 1), 1, 16, 16, 16)
    s = _scores(n, 100 + n)
    old = (np.random.default_rng(n).random(n) < 0.3).astype(np.uint8)
    fz = dev(old.copy())
    cnt = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    ctx.update_freeze_mask_rule("mingrad", dev(s), fraction, 0, 0, mode, fz, n_frozen=cnt)
    torch.cuda.synchronize()
    ref = O.apply_freeze(old, O.freeze_mingrad(s, fraction), mode)
    got = fz.cpu().numpy()
    assert np.array_equal(got, ref)
    assert int(cnt.item()) == int(ref.sum())
    assert ctx.check()[0] == 0


@pytest.mark.parametrize("n", [0, 1, 1000, 20_000])
@pytest.mark.parametrize("fraction", [0.0, 0.25, 1.0])
def test_random_matches_oracle(n, fraction):
    import torch
    import paper_2504_06716_amd as G
    print(f"random n={n} fraction={fraction}", flush=True)
    ctx = G.Context(max(n, 1), 1, 16, 16, 16)
    for draw, seed, mode in [(0, 5, 2), (1234, 5, 0), (1234, 2 ** 63 + 7, 2)]:
        old = (np.random.default_rng(draw).random(n) < 0.2).astype(np.uint8)
        fz = dev(old.copy())
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        ctx.update_freeze_mask_rule("random", None, fraction, seed, draw, mode, fz, n_frozen=cnt)
        torch.cuda.synchronize()
        ref = O.apply_freeze(old, O.freeze_random(n, fraction, seed, draw), mode)
        assert np.array_equal(fz.cpu().numpy(), ref)
        assert int(cnt.item()) == int(ref.sum())


def test_rule_arguments_rejected():
    import torch
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd import _lib
    ctx = G.Context(100, 1, 16, 16, 16)
    fz = torch.zeros(100, dtype=torch.uint8, device="cuda")
    s = torch.zeros(100, device="cuda")
    L = _lib.load()
    st = torch.cuda.current_stream().cuda_stream
    for rule, frac, mode in [(0, 0.25, 0), (3, 0.25, 0), (1, -0.1, 0), (1, 1.5, 0), (2, float("nan"), 0),
                             (1, 0.25, 3)]:
        assert L.gsta_update_freeze_mask_rule(ctx.h, rule, s.data_ptr(), 100, frac, 0, 0, mode, fz.data_ptr(),
                                              None, st) == _lib.GSTA_ERR_INVALID
    assert L.gsta_update_freeze_mask_rule(ctx.h, 1, None, 100, 0.25, 0, 0, 0, fz.data_ptr(), None,
                                          st) == _lib.GSTA_ERR_INVALID
    assert L.gsta_update_freeze_mask_rule(ctx.h, 1, s.data_ptr(), 101, 0.25, 0, 0, 0, fz.data_ptr(), None,
                                          st) == _lib.GSTA_ERR_INVALID


@pytest.mark.parametrize("rule", ["mingrad", "random"])
def test_training_with_ablation_rule(rule):
    """The trainer applies the rule at each update of the lifecycle: at the
    first update the map is exactly the oracle's rule on the averages the
    GPU held just before it; the map is reset at the window close."""
    import torch
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd.schedule import FreezeSchedule, LearningRates
    from paper_2504_06716_amd.train import Trainer, TrainConfig, render_targets
    n = 3000
    p = S.make_scene(n, 3, seed=4)
    p[3:6] += 0.4
    cams = [S.look_at(-20.0 + 10 * k, 40.0 * k, 48, 40) for k in range(4)]
    ctx = G.Context(n, 4, 40, 48, 1 << 20)
    tgt = render_targets(ctx, S.perturb_scene(p, 3), 3, cams)
    fs = FreezeSchedule(total_iters=60, warmup=10, every=5, reset_every=30, wait=5, window_end=50,
                        rule=rule, fraction=0.25, seed=9)
    cfg = TrainConfig(iters=60, freeze=True, schedule=fs, lrs=LearningRates(decay_iters=60), finetune_iters=10)
    tr = Trainer(p, 3, cams, tgt, cfg, S.view_order(4, 60), ctx=ctx)
    tr.run(10)
    ema = tr.ema[0].cpu().numpy()
    tr.step()                                   # the update before iteration 10, then iteration 10
    torch.cuda.synchronize()
    cond = O.freeze_mingrad(ema, 0.25) if rule == "mingrad" else O.freeze_random(n, 0.25, 9, 10)
    assert np.array_equal(tr.frozen.cpu().numpy(), cond)
    tr.run()
    torch.cuda.synchronize()
    assert tr.k == 60 and int(tr.frozen.sum()) == 0
    hist = tr.freeze_history()
    assert max(c for *_, c in hist) > 0.2 * n
