"""GPU (libgsta through the C ABI) versus the FP64 oracle, element by element.

Bars: depth keys, depth order, tile lists and freeze masks bit-exact (a
Gaussian whose tile-rectangle edge or near-plane test lies within float32
reach of its threshold may differ, and is left out); images within 1e-4 on
pixels whose decisions are not within 1e-5 relative of a threshold;
gradients within 1e-3 relative per parameter group."""
import numpy as np
import pytest

import oracle as O
import synthetic as S
from tests.gpu_util import (IMAGE_ATOL, MARGIN_NEAR, MARGIN_RECT_PX, MARGIN_VALUE, GpuScene,
                            compare_grads, dev)

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2504_06716_amd import _lib
    return _lib


def scene(kind):
    """(params, degree, cams) for a named parity case."""
    if kind == "tiny":
        p = S.make_scene(64, 3, seed=0)
        p[3:6] += 0.9
        cams = [S.look_at(10.0 + 35.0 * k, 20.0 + 70.0 * k, 32, 32) for k in range(2)]
        return p, 3, cams
    if kind == "c1":
        c = S.CONFIGS["c1"]
        return S.make_scene(c["n"], 0), 0, S.config_cameras("c1")
    if kind == "ragged":
        p = S.make_scene(3000, 3, seed=5)
        p[3:6] += 0.5
        cams = [S.look_at(25.0, 130.0, 50, 37), S.look_at(-40.0, 10.0, 50, 37)]
        return p, 3, cams
    if kind == "deg1":
        p = S.make_scene(1500, 1, seed=6)
        p[3:6] += 0.6
        return p, 1, [S.look_at(5.0, 60.0, 48, 48)]
    if kind == "c2view":
        c = S.CONFIGS["c2"]
        return S.make_scene(c["n"], 3), 3, S.config_cameras("c2")[:1]
    raise KeyError(kind)


CASES = ["tiny", "c1", "ragged", "deg1"]


def _margins(p, degree, cams):
    recs = [O.project(p, degree, c) for c in cams]
    marg = np.zeros(p.shape[1], bool)
    for r in recs:
        marg |= (r[:, 27] < MARGIN_RECT_PX) | (r[:, 25] < MARGIN_NEAR) | (r[:, 26] < MARGIN_NEAR)
    return recs, marg


@pytest.mark.parametrize("kind", CASES + ["c2view"])
def test_preprocess_records(kind):
    p, D, cams = scene(kind)
    g = GpuScene(p, D, cams)
    g.forward()
    n, V = p.shape[1], len(cams)
    from paper_2504_06716_amd import _lib as L
    import torch
    geo = g.state(L.STATE_REC_GEO, torch.float32, (V, n, 4))
    col = g.state(L.STATE_REC_COL, torch.float32, (V, n, 4))
    rgb = g.state(L.STATE_REC_RGB, torch.float32, (V, n, 4))
    rect = g.state(L.STATE_RECT, torch.int16, (V, n, 4)).astype(np.int64) & 0xFFFF
    recs, marg = _margins(p, D, cams)
    for v in range(V):
        r = recs[v]
        gvis = rect[v, :, 0] < rect[v, :, 1]
        ovis = r[:, 0] == 1
        assert np.array_equal(gvis[~marg], ovis[~marg])
        both = gvis & ovis
        assert both.sum() > 0
        # depth key: the correctly rounded float32 depth, bit-exact
        assert np.array_equal(rgb[v, both, 3], r[both, 4].astype(np.float32))
        # the whole-wave skip extent covers every possible member pixel
        rb = r[both]
        can = 255.0 * rb[:, 24] > 1.0 + 1e-5
        kf = np.sqrt(2.0 * np.minimum(4.5, np.log(255.0 * rb[can, 24])))
        assert (col[v, both, 2][can] >= kf * np.sqrt(rb[can, 5]) - 1e-3).all()
        assert (col[v, both, 3][can] >= kf * np.sqrt(rb[can, 7]) - 1e-3).all()
        np.testing.assert_allclose(geo[v, both, 0], r[both, 1], atol=2e-4, rtol=1e-6)
        np.testing.assert_allclose(geo[v, both, 1], r[both, 2], atol=2e-4, rtol=1e-6)
        # the records hold the conic scaled for a base-2 exponent:
        # (A, B, C) = (-a/2, -b, -c/2) * log2(e)
        l2e = np.log2(np.e)
        conic = [geo[v, both, 2] / (-0.5 * l2e), geo[v, both, 3] / -l2e, col[v, both, 0] / (-0.5 * l2e)]
        cmax = np.maximum(np.abs(r[both, 9]), np.abs(r[both, 11]))
        for got, j in zip(conic, (9, 10, 11)):
            assert (np.abs(got - r[both, j]) <= 1e-4 * cmax).all()
        np.testing.assert_allclose(col[v, both, 1], r[both, 24], atol=1e-6)
        np.testing.assert_allclose(rgb[v, both, :3], r[both, 18:21], atol=2e-5)
        ok = ~marg
        assert np.array_equal(rect[v, ok & ovis], r[ok & ovis, 14:18].astype(np.int64))


@pytest.mark.parametrize("kind", CASES + ["c2view"])
def test_depth_order_and_tile_lists(kind):
    p, D, cams = scene(kind)
    g = GpuScene(p, D, cams)
    g.forward()
    import torch
    from paper_2504_06716_amd import _lib as L
    n, V = p.shape[1], len(cams)
    order = g.state(L.STATE_DEPTH_ORDER, torch.int32, (V, n)).astype(np.int64)
    ninst = int(g.state(L.STATE_N_INSTANCES, torch.int64, (1,))[0])
    cam0 = cams[0]
    ntx, nty = (cam0.width + 15) // 16, (cam0.height + 15) // 16
    T = ntx * nty
    keys = g.state(L.STATE_INST_KEYS, torch.int32, (ninst,)).astype(np.int64) & 0xFFFFFFFF
    eidx = g.state(L.STATE_INST_IDS, torch.int32, (ninst,)).astype(np.int64)
    egid = g.state(L.STATE_INST_GID, torch.int32, (ninst,)).astype(np.int64)
    ids = egid[eidx]
    # the expansion lists Gaussians in depth order, each one's tiles contiguous
    assert sorted(eidx.tolist()) == list(range(ninst))
    ranges = g.state(L.STATE_RANGES, torch.int32, (V * T, 2)).astype(np.int64)
    assert (np.diff(keys) >= 0).all()
    _, marg = _margins(p, D, cams)
    mset = set(np.nonzero(marg)[0].tolist())
    total = 0
    for v, cam in enumerate(cams):
        counts, oids, oorder = O.bin_tiles(p, D, cam)
        nvis = len(oorder)
        got = [x for x in order[v, :nvis] if x not in mset]
        exp = [x for x in oorder if x not in mset]
        assert got == exp
        pos = 0
        for t in range(T):
            a, b = ranges[v * T + t]
            glist = [x for x in ids[a:b] if x not in mset]
            olist = [x for x in oids[pos:pos + counts[t]] if x not in mset]
            pos += counts[t]
            assert glist == olist, (v, t)
            assert (keys[a:b] == v * T + t).all()
        total += counts.sum()
    if not mset:
        assert ninst == total


def _forward_compare(p, D, cams, bg=(0.0, 0.0, 0.0)):
    g = GpuScene(p, D, cams, bg=bg)
    img = g.forward()
    import torch
    from paper_2504_06716_amd import _lib as L
    V, H, W = len(cams), cams[0].height, cams[0].width
    Tf = g.state(L.STATE_T_FINAL, torch.float32, (V, H, W))
    excluded = 0
    outs = []
    for v, cam in enumerate(cams):
        o = O.render(p, D, cam, bg=bg)
        ok = o["m_value"] >= MARGIN_VALUE
        excluded += (~ok).sum()
        d = np.abs(img[v] - o["image"])
        assert d[:, ok].max() <= IMAGE_ATOL, d[:, ok].max()
        assert np.abs(Tf[v] - o["T_final"])[ok].max() <= IMAGE_ATOL
        outs.append(o)
    return g, img, outs, excluded / (V * H * W)


@pytest.mark.parametrize("kind", CASES + ["c2view"])
def test_forward_image(kind):
    p, D, cams = scene(kind)
    _, img, outs, frac = _forward_compare(p, D, cams)
    assert frac < 0.01
    assert img.max() > 0.05


def test_forward_background_and_partial_tiles():
    p, D, cams = scene("ragged")
    _forward_compare(p, D, cams, bg=(0.3, 0.6, 0.1))


def _backward_case(p, D, cams, frozen=None, bg=(0.0, 0.0, 0.0), seed=21):
    g, img, outs, _ = _forward_compare(p, D, cams, bg=bg)
    V, H, W = len(cams), cams[0].height, cams[0].width
    rng = np.random.default_rng(seed)
    dL = rng.standard_normal((V, 3, H, W))
    for v, o in enumerate(outs):
        bad = (o["m_value"] < MARGIN_VALUE) | (o["m_grad"] < MARGIN_VALUE)
        dL[v][:, bad] = 0.0
    dL = dL.astype(np.float32)
    grad, g2, _ = g.backward(dL, frozen=frozen, sentinel=7.0)
    ref, ref2, _ = O.render_backward(p, D, cams, dL.astype(np.float64), frozen=frozen, bg=bg)
    recs, marg = _margins(p, D, cams)
    for r in recs:
        marg |= (r[:, 28] < 1e-4) | (r[:, 29] < 1e-4)
    act = np.ones(p.shape[1], bool) if frozen is None else frozen == 0
    rep = compare_grads(grad[:, act], ref[:, act], exclude_cols=marg[act])
    if frozen is not None:
        assert (grad[:, ~act] == 7.0).all()
    return grad, ref, rep


@pytest.mark.parametrize("kind", CASES + ["c2view"])
def test_backward_gradients(kind):
    p, D, cams = scene(kind)
    _backward_case(p, D, cams)


def test_backward_with_background():
    p, D, cams = scene("ragged")
    _backward_case(p, D, cams, bg=(0.3, 0.6, 0.1))


@pytest.mark.parametrize("kind", ["tiny", "c1", "ragged"])
def test_backward_frozen_skip(kind):
    p, D, cams = scene(kind)
    frozen = (np.random.default_rng(3).random(p.shape[1]) < 0.4).astype(np.uint8)
    grad_f, _, _ = _backward_case(p, D, cams, frozen=frozen)
    grad_a, _, _ = _backward_case(p, D, cams)
    act = frozen == 0
    # active rows do not depend on which other Gaussians are frozen
    np.testing.assert_allclose(grad_f[:, act], grad_a[:, act], rtol=1e-5,
                               atol=1e-6 * np.abs(grad_a[:, act]).max())


def test_ema_scores():
    p, D, cams = scene("ragged")
    g, img, outs, _ = _forward_compare(p, D, cams)
    n = p.shape[1]
    rng = np.random.default_rng(4)
    big = np.finfo(np.float32).max
    ema0 = np.where(rng.random((4, n)) < 0.3, big, rng.random((4, n)) * 1e-3).astype(np.float32)
    frozen = (rng.random(n) < 0.2).astype(np.uint8)
    dL = rng.standard_normal((len(cams), 3, cams[0].height, cams[0].width)).astype(np.float32)
    for v, o in enumerate(outs):
        dL[v][:, (o["m_value"] < MARGIN_VALUE) | (o["m_grad"] < MARGIN_VALUE)] = 0.0
    _, _, ema = g.backward(dL, frozen=frozen, ema=ema0, beta=0.9)
    ref, _, vis = O.render_backward(p, D, cams, dL.astype(np.float64), frozen=frozen)
    sc = O.scores(ref)
    visany = vis.any(0)
    for k in range(4):
        exp = O.ema_update(ema0[k].astype(np.float64), sc[k], visany, frozen, 0.9)
        same = exp >= big
        assert np.array_equal(ema[k] >= big, same)
        np.testing.assert_allclose(ema[k][~same], exp[~same], rtol=2e-3,
                                   atol=1e-3 * np.abs(exp[~same]).max())


def test_multiview_batch_equals_single_views():
    p = S.make_scene(2500, 3, seed=8)
    p[3:6] += 0.5
    cams = [S.look_at(-50.0 + 14.0 * k, 45.0 * k, 40, 40) for k in range(8)]
    gb = GpuScene(p, 3, cams)
    batch = gb.forward()
    for v in range(8):
        single = GpuScene(p, 3, cams[v:v + 1]).forward()
        assert np.array_equal(batch[v], single[0])
    _backward_case(p, 3, cams[:4])


def test_empty_and_culled_scenes():
    bg = (0.3, 0.6, 0.1)
    cam = S.look_at(0.0, 0.0, 40, 24)
    # no Gaussians
    g = GpuScene(np.zeros((14, 0), np.float32), 0, [cam], bg=bg)
    img = g.forward()
    assert np.allclose(img[0], np.array(bg, np.float32)[:, None, None])
    # every Gaussian behind the camera (camera at (3,0,0) looking along -x)
    p = S.make_scene(50, 0, seed=2)
    p[0] += 5.0
    g = GpuScene(p, 0, [cam], bg=bg)
    img = g.forward()
    assert np.allclose(img[0], np.array(bg, np.float32)[:, None, None])
    dL = np.ones((1, 3, 24, 40), np.float32)
    big = np.finfo(np.float32).max
    grad, _, ema = g.backward(dL, ema=np.full((4, 50), big, np.float32))
    assert (grad == 0).all()
    assert (ema == big).all()


def test_capacity_overflow_is_reported():
    import paper_2504_06716_amd as G
    p, D, cams = scene("c1")
    ctx = G.Context(p.shape[1], 1, 64, 64, instance_capacity=200)
    g = GpuScene(p, D, cams[:1], ctx=ctx)
    g.forward()
    st, need = ctx.check()
    assert st == _lib().GSTA_ERR_CAPACITY and need > 200
    ctx.reserve(instance_capacity=int(need))
    g.forward()
    st, _ = ctx.check()
    assert st == _lib().GSTA_OK


def test_invalid_arguments_rejected():
    import torch
    import paper_2504_06716_amd as G
    p, D, cams = scene("tiny")
    ctx = G.Context(64, 2, 32, 32, 1 << 16)
    P = dev(p)
    img = torch.empty((2, 3, 32, 32), device="cuda")
    with pytest.raises(G.GstaError):                     # backward before any forward
        ctx.render_backward(P, D, cams, (0, 0, 0), 0, img, None, torch.empty_like(P))
    with pytest.raises(G.GstaError):                     # slot out of range
        ctx.render_forward(P, D, cams, (0, 0, 0), img, slot=3)
    big = S.look_at(0.0, 0.0, 64, 64)
    with pytest.raises(G.GstaError):                     # image larger than reserved
        ctx.render_forward(P, D, [big], (0, 0, 0), torch.empty((1, 3, 64, 64), device="cuda"))
    with pytest.raises(ValueError):                      # image shape does not match the views
        ctx.render_forward(P, D, [big], (0, 0, 0), img)
    ctx.render_forward(P, D, cams, (0, 0, 0), img)
    with pytest.raises(G.GstaError):                     # cameras differ from the forward
        ctx.render_backward(P, D, cams[::-1], (0, 0, 0), 0, img, None, torch.empty_like(P))
    with pytest.raises(G.GstaError):                     # 65 Gaussians > reserved 64
        ctx.render_forward(dev(S.make_scene(65, 3)), D, cams, (0, 0, 0), img)


@pytest.mark.parametrize("ld_pad", [0, 1])
def test_adam_masked_matches_oracle(ld_pad):
    import torch
    import paper_2504_06716_amd as G
    rng = np.random.default_rng(5)
    R, n = 59, 1003
    ctx = G.Context(n + ld_pad, 1, 16, 16, 16)
    blocks = [rng.standard_normal((R, n + ld_pad)).astype(np.float32) for _ in range(4)]
    blocks[3] = np.abs(blocks[3])
    frozen = (rng.random(n) < 0.3).astype(np.uint8)
    lr = np.linspace(1e-3, 1e-2, R).astype(np.float32)
    t = [dev(b)[:, :n] for b in blocks]
    p, g, m, v = t
    ctx.adam_masked(p, g, m, v, 3, lr, 0.9, 0.999, 1e-15, 7, dev(frozen))
    torch.cuda.synchronize()
    # the oracle takes the float32 hyper-parameters the GPU receives
    b1, b2 = float(np.float32(0.9)), float(np.float32(0.999))
    P, Mm, Vv = O.adam_masked(blocks[0][:, :n], blocks[1][:, :n], blocks[2][:, :n], blocks[3][:, :n],
                              lr.astype(np.float64), b1, b2, 1e-15, 7, frozen)
    gp, gm, gv = p.cpu().numpy(), m.cpu().numpy(), v.cpu().numpy()
    fz = frozen == 1
    assert np.array_equal(gp[:, fz], blocks[0][:, :n][:, fz])
    assert np.array_equal(gm[:, fz], blocks[2][:, :n][:, fz])
    assert np.array_equal(gv[:, fz], blocks[3][:, :n][:, fz])
    # p: a few float32 ulps of p plus a relative error of the applied update
    p0 = blocks[0][:, :n].astype(np.float64)
    err = np.abs(gp[:, ~fz] - P[:, ~fz])
    assert (err <= 4e-7 * np.abs(P[:, ~fz]) + 1e-5 * np.abs(P - p0)[:, ~fz] + 1e-12).all()
    # m = b1 m + (1 - b1) g may cancel: bound by the float32 rounding of the operands
    m0, g0, v0 = (blocks[k][:, :n].astype(np.float64) for k in (2, 1, 3))
    mb = 4e-7 * (0.9 * np.abs(m0) + 0.1 * np.abs(g0)) + 1e-12
    assert (np.abs(gm - Mm)[:, ~fz] <= mb[:, ~fz]).all()
    vb = 4e-7 * (0.999 * v0 + 0.001 * g0 * g0) + 1e-12
    assert (np.abs(gv - Vv)[:, ~fz] <= vb[:, ~fz]).all()


def test_adam_nonfinite_flag():
    import torch
    import paper_2504_06716_amd as G
    ctx = G.Context(64, 1, 16, 16, 16)
    blocks = [torch.zeros((14, 64), device="cuda") for _ in range(4)]
    blocks[1][3, 5] = float("nan")
    ctx.adam_masked(*blocks, 0, [1e-3] * 14, 0.9, 0.999, 1e-15, 1)
    st, _ = ctx.check()
    assert st == _lib().GSTA_ERR_NONFINITE
    assert ctx.check()[0] == _lib().GSTA_OK


def test_freeze_mask_bit_exact():
    import torch
    import paper_2504_06716_amd as G
    rng = np.random.default_rng(6)
    n = 100_003
    ctx = G.Context(16, 1, 16, 16, 16)
    sx = (rng.random(n) * 6e-5).astype(np.float32)
    sr = (rng.random(n) * 2e-4).astype(np.float32)
    sx[:100] = np.float32(3e-5)                      # exactly at the threshold: not frozen (strict)
    sr[100:200] = np.float32(1e-4)
    sx[200:300] = np.finfo(np.float32).max            # never seen
    old = (rng.random(n) < 0.1).astype(np.uint8)
    prop = (rng.random(n) < 0.05).astype(np.uint8)
    for mode in (0, 1, 2):
        for proposal in (None, prop):
            fz = dev(old.copy())
            cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
            ctx.update_freeze_mask(dev(sx), dev(sr), 3e-5, 1e-4, mode, fz,
                                   proposal=None if proposal is None else dev(proposal), n_frozen=cnt)
            torch.cuda.synchronize()
            exp = O.freeze_update(old, sx, sr, 3e-5, 1e-4, mode, proposal)
            got = fz.cpu().numpy()
            assert np.array_equal(got, exp)
            assert int(cnt.item()) == int(exp.sum())


def test_l1_loss_matches_oracle():
    import torch
    import paper_2504_06716_amd as G
    rng = np.random.default_rng(7)
    ctx = G.Context(16, 1, 16, 16, 16)
    img = rng.uniform(-0.2, 1.2, (2, 3, 37, 50)).astype(np.float32)
    tgt = rng.random((2, 3, 37, 50)).astype(np.float32)
    tgt[0, 0, 0, :5] = img[0, 0, 0, :5]              # sign(0) = 0
    dL = torch.empty(img.shape, device="cuda")
    sums = torch.zeros(2, dtype=torch.float64, device="cuda")
    ctx.l1_loss(dev(img), dev(tgt), dL, sums)
    torch.cuda.synchronize()
    loss, dref, mse = O.l1_loss(img, tgt)
    s = sums.cpu().numpy()
    assert s[0] / img.size == pytest.approx(loss, rel=1e-6)
    assert s[1] / img.size == pytest.approx(mse, rel=1e-6)
    np.testing.assert_allclose(dL.cpu().numpy(), dref, rtol=1e-6)
    assert (dL.cpu().numpy()[0, 0, 0, :5] == 0).all()


@pytest.mark.parametrize("fwd,bwd", [(1, 1), (2, 2), (4, 4), (4, 1), (1, 4), (0, 4), (0, 2)])
def test_waves_per_tile_options(fwd, bwd):
    """Waves per tile change the thread mapping only: images are bit-identical,
    gradients agree to rounding of the reduction order."""
    p, D, cams = scene("ragged")
    ref = GpuScene(p, D, cams)
    img_ref = ref.forward()
    dL = np.random.default_rng(9).standard_normal((len(cams), 3, 37, 50)).astype(np.float32)
    g_ref, _, _ = ref.backward(dL)
    g = GpuScene(p, D, cams)
    g.ctx.set_waves(fwd=fwd, bwd=bwd)
    img = g.forward()
    assert np.array_equal(img, img_ref)
    grad, _, _ = g.backward(dL)
    np.testing.assert_allclose(grad, g_ref, rtol=1e-4, atol=1e-6 * np.abs(g_ref).max())


@pytest.mark.parametrize("kind", ["ragged", "c2view"])
def test_quadrant_forward_checkpoints_equal_tile_mode(kind):
    """The quadrant-mode forward (one workgroup per 8x8 quarter) takes the
    same per-pixel steps as the tile mode and writes its own quarter's
    checkpoints: image, final state and segmented-backward gradients are
    bit-identical."""
    import torch
    from paper_2504_06716_amd import _lib as L
    p, D, cams = scene(kind)
    H, W = cams[0].height, cams[0].width
    dL = np.random.default_rng(5).standard_normal((len(cams), 3, H, W)).astype(np.float32)
    out = []
    for fwd in (4, 0):
        print(f"quadrant checkpoints {kind}: forward waves {fwd}", flush=True)
        g = GpuScene(p, D, cams)
        g.ctx.set_waves(fwd=fwd, bwd=2)
        img = g.forward()
        last = g.state(L.STATE_LAST, torch.int32, (len(cams), H, W))
        grad, g2, _ = g.backward(dL)
        assert g.ctx.check()[0] == 0
        out.append((img, last, grad, g2))
    assert int(out[0][1].max()) > 64          # several segments per tile
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("kind", ["ragged", "c2view"])
def test_backward_segments_agree(kind):
    """Splitting each tile's backward walk into segments that resume from
    the forward's checkpoints changes the schedule, and where a segment
    starts, how the dot product of dL/dC with the colour behind is formed
    (from the checkpointed colour instead of step by step): images are
    bit-identical to the unsegmented walk and gradients agree to rounding,
    for every forward / backward wave shape; with the same segment length,
    every forward mode gives bit-identical gradients."""
    from paper_2504_06716_amd import _lib as L
    p, D, cams = scene(kind)
    H, W = cams[0].height, cams[0].width
    dL = np.random.default_rng(12).standard_normal((len(cams), 3, H, W)).astype(np.float32)
    g = GpuScene(p, D, cams)
    g.ctx.set_option(L.OPT_BWD_SEGMENT, 0)
    g.ctx.set_waves(fwd=4, bwd=2)
    img0 = g.forward()
    ref, ref2, _ = g.backward(dL)
    import torch
    tl = g.state(L.STATE_LAST, torch.int32, (len(cams), H, W))
    print(kind, "largest last", int(tl.max()))
    res = {}
    for seg, fwd, bwd in [(64, 4, 2), (128, 4, 2), (4096, 4, 2), (64, 1, 2), (128, 2, 1), (64, 0, 4), (128, 4, 4),
                          (64, 0, 2), (128, 0, 2), (512, 0, 2), (4096, 0, 2)]:
        g.ctx.set_option(L.OPT_BWD_SEGMENT, seg)
        g.ctx.set_waves(fwd=fwd, bwd=bwd)
        img = g.forward()
        grad, g2, _ = g.backward(dL)
        assert np.array_equal(img, img0)
        np.testing.assert_allclose(grad, ref, rtol=1e-4, atol=1e-6 * np.abs(ref).max(), err_msg=str((seg, fwd, bwd)))
        if bwd == 2:
            np.testing.assert_allclose(g2, ref2, rtol=1e-4, atol=1e-6 * np.abs(ref2).max())
        if (seg, bwd) == (64, 2):
            res[fwd] = grad
    # the same segments and backward: every forward mode's checkpoints give the same gradients
    assert np.array_equal(res[4], res[1]) and np.array_equal(res[4], res[0])
    assert g.ctx.check()[0] == 0


def test_backward_is_deterministic():
    p, D, cams = scene("c2view")
    g = GpuScene(p, D, cams)
    g.forward()
    dL = np.random.default_rng(10).standard_normal((1, 3, 480, 640)).astype(np.float32)
    a, a2, _ = g.backward(dL)
    b, b2, _ = g.backward(dL)
    assert np.array_equal(a, b) and np.array_equal(a2, b2)


def test_adam_device_schedule_matches_host_adam():
    import torch
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd.core import adam_sched_tensor
    from paper_2504_06716_amd.schedule import LearningRates
    rng = np.random.default_rng(11)
    R, n = 59, 777
    ctx = G.Context(n, 1, 16, 16, 16)
    lrs = LearningRates(decay_iters=100)
    base = [rng.standard_normal((R, n)).astype(np.float32) for _ in range(4)]
    base[3] = np.abs(base[3])
    frozen = (rng.random(n) < 0.25).astype(np.uint8)
    host = [dev(b) for b in base]
    devs = [dev(b) for b in base]
    sched = adam_sched_tensor(1, 0.9, 0.999, 1e-15, lrs.rows(0, 3), lrs.extent * lrs.pos_init,
                              lrs.extent * lrs.pos_final, lrs.decay_iters)
    fz = dev(frozen)
    for k in range(5):
        g = dev(rng.standard_normal((R, n)).astype(np.float32))
        host[1].copy_(g)
        devs[1].copy_(g)
        ctx.adam_masked(host[0], host[1], host[2], host[3], 3, lrs.rows(k, 3), 0.9, 0.999, 1e-15, k + 1, fz)
        ctx.adam_masked_sched(devs[0], devs[1], devs[2], devs[3], 3, sched, fz)
    torch.cuda.synchronize()
    assert int(sched[:4].view(torch.int32).item()) == 6
    for a, b in zip(host, devs):
        np.testing.assert_allclose(b.cpu().numpy(), a.cpu().numpy(), rtol=2e-5, atol=1e-6)


def test_graph_replay_matches_eager_training():
    """A HIP-graph-captured iteration (one graph per view, replayed) trains
    exactly like the eager calls, freezing included."""
    import torch
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd.schedule import FreezeSchedule, LearningRates
    from paper_2504_06716_amd.train import Trainer, TrainConfig, render_targets
    p = S.make_scene(3000, 3, seed=4)
    p[3:6] += 0.4
    cams = [S.look_at(-20.0 + 10 * k, 40.0 * k, 48, 40) for k in range(4)]
    ctx = G.Context(3000, 4, 40, 48, 1 << 20)
    tgt = render_targets(ctx, S.perturb_scene(p, 3), 3, cams)
    order = S.view_order(4, 60)
    sched = FreezeSchedule(total_iters=60, warmup=10, every=5, reset_every=30, wait=5, window_end=50,
                           eps_xyz0=1e-6, eps_rgb0=1e-7)
    out = []
    for graph in (False, True):
        cfg = TrainConfig(iters=60, freeze=True, schedule=sched, lrs=LearningRates(decay_iters=60),
                          device_sched=True, graph=graph)
        tr = Trainer(p, 3, cams, tgt, cfg, order, ctx=ctx)
        tr.run(60)
        torch.cuda.synchronize()
        out.append((tr.P.cpu().numpy(), tr.frozen_log, [c for *_, c in tr.freeze_history()]))
    assert np.array_equal(out[0][0], out[1][0])
    assert out[0][1] == out[1][1] and out[0][2] == out[1][2]


def test_trainer_ema_rows_match_the_step_gradient():
    """Regression: with n not a multiple of 64 the trainer's EMA rows must be
    the scores of the same Gaussians as the gradient block (first step: the
    EMA equals the score)."""
    import torch
    import paper_2504_06716_amd as G
    from paper_2504_06716_amd.schedule import LearningRates
    from paper_2504_06716_amd.train import Trainer, TrainConfig, render_targets
    n = 1499
    p = S.make_scene(n, 3, seed=8)
    p[3:6] += 0.5
    cams = [S.look_at(5.0 * k, 30.0 * k, 40, 32) for k in range(2)]
    ctx = G.Context(n, 2, 32, 40, 1 << 20)
    tgt = render_targets(ctx, S.perturb_scene(p, 3), 3, cams)
    cfg = TrainConfig(iters=4, freeze=False, track_ema=True, lrs=LearningRates(decay_iters=4))
    tr = Trainer(p, 3, cams, tgt, cfg, S.view_order(2, 4), ctx=ctx)
    tr.step()
    torch.cuda.synchronize()
    g = tr.G.cpu().numpy().astype(np.float64)
    ema = tr.ema.cpu().numpy().astype(np.float64)
    seen = ema[0] < O.FLT_MAX
    assert seen.sum() > 100
    sc = [np.linalg.norm(g[0:3], axis=0), np.linalg.norm(g[11:14], axis=0), np.abs(g[10]),
          np.linalg.norm(g[3:6], axis=0)]
    for k in range(4):
        np.testing.assert_allclose(ema[k][seen], sc[k][seen], rtol=1e-5, atol=1e-30)
