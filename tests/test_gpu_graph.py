"""The C-ABI graph capture (gsta_graph_begin/end/launch/destroy) and
autotuner (gsta_autotune): a captured iteration replayed several times with
eager work and synchronisations in between equals the eager iterations bit
for bit; multi-view steps from fixed batches captured per batch equal eager
ones; the tuned options leave results unchanged; misuse is refused."""
import ctypes

import numpy as np
import pytest

import synthetic as S
from tests.gpu_util import dev

pytestmark = pytest.mark.gpu


def _scene(n=2500, degree=3, H=40, W=48, n_cams=4, seed=4):
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd.train import render_targets
    p = S.make_scene(n, degree, seed=seed)
    p[3:6] += 0.4
    cams = [S.look_at(-20.0 + 10 * k, 40.0 * k, W, H) for k in range(n_cams)]
    ctx = G.Context(n, n_cams, H, W, 1 << 20)
    tgt = render_targets(ctx, S.perturb_scene(p, degree), degree, cams)
    return p, cams, ctx, tgt


def test_captured_iteration_replays_equal_eager_calls():
    import torch
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd.core import adam_sched_tensor
    from paper_2504_06716_amd.schedule import LearningRates
    p, cams, ctx, tgt = _scene()
    lrs = LearningRates(decay_iters=20)
    carr = G.camera_array(cams[:1])
    runs = []
    for mode in ("eager", "graph"):
        P = dev(p.copy())
        M, V, Gr = torch.zeros_like(P), torch.zeros_like(P), torch.zeros_like(P)
        img = torch.empty((1, 3, 40, 48), device="cuda")
        dL = torch.empty_like(img)
        sums = torch.zeros(2, dtype=torch.float64, device="cuda")
        sched = adam_sched_tensor(1, 0.9, 0.999, 1e-15, lrs.rows(0, 3), lrs.extent * lrs.pos_init,
                                  lrs.extent * lrs.pos_final, lrs.decay_iters)

        def body():
            ctx.render_forward_l1(P, 3, carr, (0, 0, 0), tgt[0:1], img, dL, sums, 0)
            ctx.render_backward(P, 3, carr, (0, 0, 0), 0, dL, None, Gr)
            ctx.adam_masked_sched(P, Gr, M, V, 3, sched, None)

        snaps = []
        if mode == "eager":
            for _ in range(4):
                body()
                torch.cuda.synchronize()
                snaps.append(P.cpu().numpy().copy())
        else:
            side = torch.cuda.Stream()
            side.wait_stream(torch.cuda.current_stream())
            with torch.cuda.stream(side):
                g = ctx.capture(body)
            torch.cuda.current_stream().wait_stream(side)
            for r in range(4):
                g.launch()
                # eager work of the program between replays, then a synchronisation
                junk = torch.ones(1 << 16, device="cuda").sum()
                torch.cuda.synchronize()
                snaps.append(P.cpu().numpy().copy())
                assert junk.item() == float(1 << 16)
            g.close()
        runs.append(snaps)
    for a, b in zip(*runs):
        assert np.array_equal(a, b)
    assert ctx.check()[0] == 0


def test_graph_misuse_is_refused():
    import torch
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd import _lib
    L = _lib.load()
    ctx = G.Context(100, 1, 16, 16, 1024)
    assert L.gsta_graph_begin(ctx.h, None) == _lib.GSTA_ERR_INVALID            # the null stream
    s = torch.cuda.Stream()
    ctx.set_profiling(["adam"])
    assert L.gsta_graph_begin(ctx.h, s.cuda_stream) == _lib.GSTA_ERR_INVALID   # profiling on
    ctx.set_profiling([])
    assert L.gsta_graph_begin(ctx.h, s.cuda_stream) == _lib.GSTA_OK
    assert L.gsta_graph_begin(ctx.h, s.cuda_stream) == _lib.GSTA_ERR_INVALID   # nested
    mi = ctypes.c_int64(0)
    assert L.gsta_check(ctx.h, s.cuda_stream, ctypes.byref(mi)) == _lib.GSTA_ERR_INVALID
    out = ctypes.c_void_p()
    assert L.gsta_graph_end(ctx.h, s.cuda_stream, ctypes.byref(out)) == _lib.GSTA_OK   # an empty graph
    assert L.gsta_graph_launch(out, s.cuda_stream) == _lib.GSTA_OK
    s.synchronize()
    L.gsta_graph_destroy(out)
    assert L.gsta_graph_end(ctx.h, s.cuda_stream, ctypes.byref(out)) == _lib.GSTA_ERR_INVALID
    assert ctx.check()[0] == 0


@pytest.mark.parametrize("vb", [2, 4])
def test_multiview_fixed_batches_graph_equals_eager(vb):
    """Several views per step captured once per fixed batch and replayed
    (with freezing and the partitioned layout) train exactly like the same
    batches run eagerly."""
    import torch
    from paper_2504_06716_amd.schedule import FreezeSchedule, LearningRates
    from paper_2504_06716_amd.train import Trainer, TrainConfig
    p, cams, ctx, tgt = _scene(n_cams=8, seed=9)
    import paper_2504_06716_amd as G
    ctx = G.Context(p.shape[1], 8, 40, 48, 1 << 21)
    from paper_2504_06716_amd.train import render_targets
    tgt = render_targets(ctx, S.perturb_scene(p, 3), 3, cams)
    perm = list(S.view_order(8, 8, seed=3))
    batches = [perm[i:i + vb] for i in range(0, 8, vb)]
    order = S.view_order(len(batches), 40, seed=5)
    fs = FreezeSchedule(total_iters=40, warmup=8, every=4, reset_every=20, wait=4, window_end=32,
                        eps_xyz0=1e-6, eps_rgb0=1e-7)
    out = []
    for graph in (False, True):
        cfg = TrainConfig(iters=40, freeze=True, schedule=fs, lrs=LearningRates(decay_iters=40), device_sched=True,
                          graph=graph, batches=batches, partition=True, finetune_iters=8)
        tr = Trainer(p, 3, cams, tgt, cfg, order, ctx=ctx)
        tr.run()
        torch.cuda.synchronize()
        out.append((tr.in_original_order(tr.P).cpu().numpy(), tr.freeze_history(), tr.k))
    assert out[0][2] == out[1][2] == 40
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1]


def test_autotune_sets_options_without_changing_results():
    import torch
    import paper_2504_06716_amd as G
    p, cams, ctx, tgt = _scene(n=4000, H=64, W=80)
    ctx = G.Context(4000, 2, 64, 80, 1 << 21)
    P = dev(p)
    carr = G.camera_array(cams[:2])
    img = torch.empty((2, 3, 64, 80), device="cuda")
    dLs = torch.full_like(img, 1e-3)
    grad = torch.empty_like(P)
    rng = np.random.default_rng(2)
    dL = dev(rng.standard_normal((2, 3, 64, 80)).astype(np.float32))

    def run():
        out = torch.empty_like(img)
        g = torch.zeros_like(P)
        ctx.render_forward(P, 3, carr, (0, 0, 0), out, 0)
        ctx.render_backward(P, 3, carr, (0, 0, 0), 0, dL, None, g)
        torch.cuda.synchronize()
        return out.cpu().numpy(), g.cpu().numpy()

    a = run()
    frozen = dev((rng.random(4000) < 0.5).astype(np.uint8))
    t = ctx.autotune(P, 3, carr, (0, 0, 0), img, dLs, grad, repeats=2, frozen=frozen)
    assert t["candidates"] == 20          # 4 forward shapes; (3 waves + the per-splat variant) x 4 segments
    assert t["fwd_waves"] in (0, 1, 2, 4) and t["bwd_waves"] in (1, 2, 4) and t["bwd_segment"] in (0, 64, 128, 256)
    assert t["bwd_variant"] in (0, 1)
    assert 0 < t["fwd_ms"] < 1000 and 0 < t["step_ms"] < 1000
    b = run()
    assert np.array_equal(a[0], b[0])                   # images: bit-identical for every option
    # gradients: the backward's waves per tile and variant change the order of its float additions
    np.testing.assert_allclose(b[1], a[1], rtol=1e-4, atol=1e-6 * np.abs(a[1]).max())
    assert ctx.check()[0] == 0
