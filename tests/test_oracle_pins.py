"""Pins of the FP64 oracle against facts that do not come from the oracle:
closed forms, quadrature, symmetry, brute force, finite differences, an
independent torch-autograd route and torch's Adam.  All CPU."""
import math

import numpy as np
import pytest
import torch

import oracle as O
import synthetic as S
from tests.dense_torch import render_dense

Y00 = 1.0 / (2.0 * math.sqrt(math.pi))


def tiny_scene(n=64, degree=3, seed=0, log_s_shift=0.0, size=32, n_cams=2):
    p = S.make_scene(n, degree, seed=seed).astype(np.float64)
    p[3:6] += log_s_shift
    cams = [S.look_at(10.0 + 35.0 * k, 20.0 + 70.0 * k, size, size) for k in range(n_cams)]
    return p, cams


# ---------------------------------------------------------------------------
# Spherical harmonics (Section 3.1: SH colour up to 3 bands)
# ---------------------------------------------------------------------------

def test_sh_constants_textbook():
    # textbook normalisation constants of the real SH basis (positive sign)
    d = np.array([[0.0, 0.0, 1.0]])
    B = O.sh_basis(3, d)[0]
    assert B[0] == pytest.approx(0.2820948, abs=1e-7)
    assert B[2] == pytest.approx(0.4886025, abs=1e-7)              # z
    assert B[6] == pytest.approx(2 * 0.3153916, abs=1e-7)          # 2z^2 - x^2 - y^2 at z=1
    assert B[12] == pytest.approx(2 * 0.3731763, abs=1e-7)         # z(2z^2 - ...) at z=1
    s = 1 / math.sqrt(3)
    B = O.sh_basis(3, np.array([[s, s, s]]))[0]
    assert B[4] == pytest.approx(1.0925484 * s * s, abs=1e-7)      # xy
    assert B[10] == pytest.approx(2.8906114 * s ** 3, abs=1e-7)    # xyz
    d = np.array([[1.0, 0.0, 0.0]])
    B = O.sh_basis(3, d)[0]
    assert B[8] == pytest.approx(0.5462742, abs=1e-7)              # x^2 - y^2
    assert B[15] == pytest.approx(0.5900436, abs=1e-7)             # x(x^2 - 3y^2)
    assert B[13] == pytest.approx(-0.4570458, abs=1e-7)            # x(4z^2 - x^2 - y^2)
    d = np.array([[math.sqrt(0.5), 0.0, math.sqrt(0.5)]])
    B = O.sh_basis(3, d)[0]
    assert B[14] == pytest.approx(1.4453057 * math.sqrt(0.5) * 0.5, abs=1e-7)  # z(x^2 - y^2)


def _sphere_quadrature(n_theta=12, n_phi=24):
    # Gauss-Legendre in cos(theta) x uniform phi: exact for polynomials of degree <= 6
    xg, wg = np.polynomial.legendre.leggauss(n_theta)
    phi = 2 * np.pi * np.arange(n_phi) / n_phi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    w = (np.repeat(wg[:, None], n_phi, 1) * (2 * np.pi / n_phi)).reshape(-1)
    return dirs, w


def test_sh_orthonormal_quadrature():
    dirs, w = _sphere_quadrature()
    B = O.sh_basis(3, dirs)
    G = (B * w[:, None]).T @ B
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_parity():
    rng = np.random.default_rng(3)
    d = rng.standard_normal((50, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    B1, B2 = O.sh_basis(3, d), O.sh_basis(3, -d)
    band = np.array([0] + [1] * 3 + [2] * 5 + [3] * 7)
    np.testing.assert_allclose(B2, B1 * (-1.0) ** band, atol=1e-15)


def test_sh_gradient_fd():
    rng = np.random.default_rng(4)
    d = rng.standard_normal((20, 3))
    _, g = O.sh_basis(3, d, with_grad=True)
    h = 1e-6
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fd = (O.sh_basis(3, d + e) - O.sh_basis(3, d - e)) / (2 * h)
        np.testing.assert_allclose(g[:, :, a], fd, atol=1e-8)


# ---------------------------------------------------------------------------
# Projection (eq. 1, EWA) closed forms
# ---------------------------------------------------------------------------

def _single(mu, log_s, q=(1.0, 0, 0, 0), logit=0.0, rgb=(0.2, 0.5, 0.9)):
    p = np.zeros((14, 1))
    p[0:3, 0] = mu
    p[3:6, 0] = log_s
    p[6:10, 0] = q
    p[10, 0] = logit
    p[11:14, 0] = (np.asarray(rgb) - 0.5) / Y00
    return p


def test_isotropic_on_axis_closed_form():
    cam = S.config_cameras("c1")[0]               # at (3, 0, 0) looking at the origin
    s = 0.05
    rng = np.random.default_rng(5)
    for _ in range(5):
        q = rng.standard_normal(4)
        p = _single([0.0, 0.0, 0.0], [math.log(s)] * 3, q)
        r = O.project(p, 0, cam)[0]
        z = 3.0
        sig2 = (cam.fx * s / z) ** 2 + 0.3
        assert r[0] == 1
        assert r[3] == pytest.approx(z, abs=1e-12)
        assert r[1] == pytest.approx(cam.cx, abs=1e-9) and r[2] == pytest.approx(cam.cy, abs=1e-9)
        assert r[5] == pytest.approx(sig2, rel=1e-12)
        assert r[7] == pytest.approx(sig2, rel=1e-12)
        assert abs(r[6]) < 1e-12
        np.testing.assert_allclose(r[9:12], [1 / sig2, 0.0, 1 / sig2], atol=1e-12)


def test_ewa_off_axis_matches_pinhole_jacobian():
    """Eq. 1 away from the optical axis: Sigma' - 0.3 I must equal D Sigma D^T
    with D the Jacobian of the pinhole map (world point -> pixel) at the
    mean, taken here by central differences of u = fx x/z + cx, v = fy y/z +
    cy, and Sigma = R S^2 R^T with R from scipy's quaternion rotation.  A sign
    or index slip in the perspective Jacobian's third column (zero on the
    axis) or in the quaternion rotation fails this."""
    from scipy.spatial.transform import Rotation
    cam = S.look_at(25.0, 40.0, 96, 80)
    rng = np.random.default_rng(11)
    tested = 0
    for _ in range(30):
        mu = rng.uniform(-0.7, 0.7, 3)
        log_s = rng.normal(-2.5, 0.5, 3)
        q = rng.standard_normal(4)
        p = _single(mu, log_s, q)
        r = O.project(p, 0, cam)[0]
        xc = cam.R @ mu + cam.t
        if r[30] or r[31] or abs(xc[0] / xc[2]) < 0.05 or abs(xc[1] / xc[2]) < 0.05:
            continue                      # tangent clamp active, or too close to the axis to matter

        def pix(x):
            c = cam.R @ x + cam.t
            return np.array([cam.fx * c[0] / c[2] + cam.cx, cam.fy * c[1] / c[2] + cam.cy])

        h = 1e-6
        D = np.stack([(pix(mu + h * e) - pix(mu - h * e)) / (2 * h) for e in np.eye(3)], axis=1)
        Rm = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        Sig = Rm @ np.diag(np.exp(2 * log_s)) @ Rm.T
        S2 = D @ Sig @ D.T + 0.3 * np.eye(2)
        np.testing.assert_allclose([r[5], r[6], r[7]], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-6, atol=1e-9)
        np.testing.assert_allclose([r[1], r[2]], pix(mu), rtol=0, atol=1e-9)
        assert r[3] == pytest.approx(xc[2], rel=1e-14)
        tested += 1
    assert tested >= 10


def test_near_plane_cull():
    cam = S.config_cameras("c1")[0]
    # camera at (3,0,0), forward -x: world x = 3 - z_cam
    p = np.concatenate([_single([3.0 - 0.19, 0, 0], [-3] * 3), _single([3.0 - 0.21, 0, 0], [-3] * 3)], 1)
    r = O.project(p, 0, cam)
    assert r[0, 0] == 0 and r[1, 0] == 1


def test_single_gaussian_image_closed_form():
    cam = S.config_cameras("c1")[0]
    s, logit, rgb = 0.08, 0.7, np.array([0.2, 0.5, 0.9])
    p = _single([0.0, 0.0, 0.0], [math.log(s)] * 3, logit=logit, rgb=rgb)
    out = O.render(p, 0, cam)
    sig2 = (cam.fx * s / 3.0) ** 2 + 0.3
    o = 1 / (1 + math.exp(-logit))
    py, px = np.mgrid[0:cam.height, 0:cam.width].astype(np.float64)
    qf = ((px - cam.cx) ** 2 + (py - cam.cy) ** 2) / sig2
    power = -0.5 * qf
    alpha = np.minimum(0.99, o * np.exp(power))
    mem = (power >= -4.5) & (alpha >= 1 / 255)
    exp_img = rgb[:, None, None] * np.where(mem, alpha, 0.0)[None]
    np.testing.assert_allclose(out["image"], exp_img, atol=1e-13)
    np.testing.assert_allclose(out["T_final"], np.where(mem, 1 - alpha, 1.0), atol=1e-13)
    assert mem.sum() > 20 and (~mem).sum() > 20


def test_two_gaussian_blend_closed_form():
    cam = S.config_cameras("c1")[0]
    c1, c2 = np.array([0.9, 0.1, 0.3]), np.array([0.2, 0.8, 0.6])
    p = np.concatenate([_single([0.5, 0, 0], [math.log(0.06)] * 3, logit=0.3, rgb=c1),     # z = 2.5
                        _single([-0.5, 0, 0], [math.log(0.09)] * 3, logit=1.2, rgb=c2)], 1)  # z = 3.5
    out = O.render(p, 0, cam)
    py, px = np.mgrid[0:cam.height, 0:cam.width].astype(np.float64)
    r2 = (px - cam.cx) ** 2 + (py - cam.cy) ** 2

    def alpha(s, z, logit):
        sig2 = (cam.fx * s / z) ** 2 + 0.3
        power = -0.5 * r2 / sig2
        a = np.minimum(0.99, np.exp(power) / (1 + math.exp(-logit)))
        return np.where((power >= -4.5) & (a >= 1 / 255), a, 0.0)

    a1, a2 = alpha(0.06, 2.5, 0.3), alpha(0.09, 3.5, 1.2)
    exp_img = c1[:, None, None] * a1 + c2[:, None, None] * (a2 * (1 - a1))
    np.testing.assert_allclose(out["image"], exp_img, atol=1e-13)


def test_tangent_clamp_and_rect_definition():
    # Gaussians far off-axis exercise the tangent clamp; the rect must equal
    # the per-tile interval test written out directly.
    cam = S.look_at(0.0, 0.0, 64, 48)
    rng = np.random.default_rng(7)
    n = 300
    p = np.zeros((14, n))
    p[0] = rng.uniform(-1, 1.5, n)
    p[1] = rng.uniform(-4, 4, n)
    p[2] = rng.uniform(-3, 3, n)
    p[3:6] = rng.normal(-2.5, 0.5, (3, n))
    p[6:10] = rng.standard_normal((4, n))
    rec = O.project(p, 0, cam, tile=16)
    assert rec[:, 30].sum() > 10                       # some tangent clamps fired
    ntx, nty = 4, 3
    for g in range(n):
        r = rec[g]
        if r[3] <= 0.2 or r[8] <= 0:
            assert r[0] == 0
            continue
        u, v, ex, ey = r[1], r[2], r[12], r[13]
        tx = [t for t in range(ntx) if 16 * t <= u + ex and 16 * t + 15 >= u - ex]
        ty = [t for t in range(nty) if 16 * t <= v + ey and 16 * t + 15 >= v - ey]
        if tx and ty:
            assert (r[14], r[15]) == (tx[0], tx[-1] + 1)
            assert (r[16], r[17]) == (ty[0], ty[-1] + 1)
            assert r[0] == 1
        else:
            assert r[0] == 0


def test_ellipse_bounding_box_is_tight():
    # ex = 3 sqrt(Sigma'_xx) is the exact half-width of the ellipse d^T K d = 9
    p, cams = tiny_scene(n=30, degree=0, log_s_shift=1.0)
    rec = O.project(p, 0, cams[0])
    th = np.linspace(0, 2 * np.pi, 20001)
    for r in rec[rec[:, 0] == 1]:
        A = np.array([[r[5], r[6]], [r[6], r[7]]])
        L = np.linalg.cholesky(A)
        d = 3.0 * (L @ np.stack([np.cos(th), np.sin(th)]))
        assert np.abs(d[0]).max() == pytest.approx(r[12], rel=1e-6)
        assert np.abs(d[1]).max() == pytest.approx(r[13], rel=1e-6)
        K = np.array([[r[9], r[10]], [r[10], r[11]]])
        np.testing.assert_allclose(np.einsum("ij,ik,kj->j", d, K, d), 9.0, rtol=1e-9)


# ---------------------------------------------------------------------------
# Binning, order, brute force, invariants (eq. 2, depth-ordered blending)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("degree,n,size", [(0, 400, 48), (3, 300, 40)])
def test_bin_lists_match_direct_filter(degree, n, size):
    p, cams = tiny_scene(n=n, degree=degree, size=size, log_s_shift=0.7)
    cam = cams[0]
    rec = O.project(p, degree, cam)
    counts, ids, order = O.bin_tiles(p, degree, cam)
    ntx = (cam.width + 15) // 16
    pos = 0
    for t in range(len(counts)):
        tx, ty = t % ntx, t // ntx
        exp = [g for g in range(n) if rec[g, 0] == 1 and rec[g, 14] <= tx < rec[g, 15]
               and rec[g, 16] <= ty < rec[g, 17]]
        exp.sort(key=lambda g: (np.float32(rec[g, 3]), g))
        got = list(ids[pos:pos + counts[t]])
        pos += counts[t]
        assert got == exp


@pytest.mark.parametrize("degree,seed", [(0, 0), (3, 1), (3, 2)])
def test_tiled_equals_brute_force(degree, seed):
    p, cams = tiny_scene(n=500, degree=degree, seed=seed, size=48, log_s_shift=0.8)
    for cam in cams:
        a = O.render(p, degree, cam)
        b = O.render(p, degree, cam, brute=True)
        for k in ("image", "T_final", "n_members", "hash"):
            assert np.array_equal(a[k], b[k]), k
        assert a["n_members"].max() > 5


def test_tile_size_invariance():
    p, cams = tiny_scene(n=500, degree=3, size=48, log_s_shift=0.8)
    ref = O.render(p, 3, cams[0], tile=16)
    for tile in (8, 32, 48):
        o = O.render(p, 3, cams[0], tile=tile)
        assert np.array_equal(o["image"], ref["image"])
        assert np.array_equal(o["T_final"], ref["T_final"])


def test_weights_plus_transmittance_is_one():
    p, cams = tiny_scene(n=500, degree=0, size=48, log_s_shift=0.8)
    p[11:14] = 0.5 / Y00                    # colour exactly 1 in every channel
    o = O.render(p, 0, cams[0])
    np.testing.assert_allclose(o["image"] + o["T_final"][None], 1.0, atol=1e-12)
    assert o["T_final"].min() < 0.01 and o["n_members"].max() > 10


def test_relabel_invariance():
    p, cams = tiny_scene(n=400, degree=3, size=40, log_s_shift=0.8)
    perm = np.random.default_rng(9).permutation(p.shape[1])
    a = O.render(p, 3, cams[0])
    b = O.render(p[:, perm], 3, cams[0])
    assert (a["ztie"] > 0).all()            # no exact depth ties
    np.testing.assert_allclose(a["image"], b["image"], atol=1e-15)


def test_termination_floor():
    # a stack of opaque Gaussians on the axis: the walk must stop before
    # transmittance drops below 1e-4 (0.01^2 = 1e-4 is not below, 0.01^3 is)
    cam = S.config_cameras("c1")[0]
    gs = [_single([0.5 - 0.1 * k, 0, 0], [math.log(0.5)] * 3, logit=12.0, rgb=(1, 1, 1)) for k in range(5)]
    p = np.concatenate(gs, 1)
    o = O.render(p, 0, cam)
    c = (cam.height // 2, cam.width // 2)
    assert o["n_members"][c] == 2
    assert o["T_final"][c] == pytest.approx(1e-4, rel=1e-9)


# ---------------------------------------------------------------------------
# Backward (Section 3.2.4): finite differences and torch autograd
# ---------------------------------------------------------------------------

def _decisions(p, degree, cams):
    sig = []
    for cam in cams:
        r = O.render(p, degree, cam)
        rec = O.project(p, degree, cam)
        sig.append((r["hash"].copy(), rec[:, [0, 14, 15, 16, 17, 21, 22, 23, 30, 31]].copy()))
    return sig


def _same(a, b):
    return all(np.array_equal(x[0], y[0]) and np.array_equal(x[1], y[1]) for x, y in zip(a, b))


@pytest.mark.parametrize("degree,shift", [(3, 0.9), (0, 1.2)])
def test_backward_matches_finite_differences(degree, shift):
    p, cams = tiny_scene(n=64, degree=degree, size=32, log_s_shift=shift)
    rng = np.random.default_rng(11)
    wimg = rng.standard_normal((len(cams), 3, 32, 32))

    def loss(pp):
        return sum((O.render(pp, degree, c)["image"] * wimg[v]).sum() for v, c in enumerate(cams))

    grads, _, _ = O.render_backward(p, degree, cams, wimg)
    base = _decisions(p, degree, cams)
    R, n = p.shape
    checked = skipped = 0
    gmax = np.abs(grads).max()
    for g in range(0, n, 3):
        for row in range(R):
            h = 1e-6 * max(abs(p[row, g]), 0.1)
            pp, pm = p.copy(), p.copy()
            pp[row, g] += h
            pm[row, g] -= h
            if not (_same(_decisions(pp, degree, cams), base) and _same(_decisions(pm, degree, cams), base)):
                skipped += 1
                continue
            fd = (loss(pp) - loss(pm)) / (2 * h)
            assert abs(fd - grads[row, g]) <= 1e-6 * gmax + 1e-5 * abs(grads[row, g]), (row, g, fd, grads[row, g])
            checked += 1
    assert checked > 0.95 * (checked + skipped)


@pytest.mark.parametrize("degree,shift,bg", [(3, 0.9, (0.0, 0.0, 0.0)), (3, 1.3, (0.3, 0.6, 0.1)),
                                             (0, 1.0, (0.0, 0.0, 0.0))])
def test_backward_matches_torch_autograd(degree, shift, bg):
    p, cams = tiny_scene(n=64, degree=degree, size=32, log_s_shift=shift, n_cams=2)
    rng = np.random.default_rng(12)
    wimg = rng.standard_normal((len(cams), 3, 32, 32))
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    L = sum((render_dense(pt, degree, c, bg) * torch.tensor(wimg[v])).sum() for v, c in enumerate(cams))
    L.backward()
    ref = pt.grad.numpy()
    # the forward of the dense route equals the oracle image
    for v, c in enumerate(cams):
        np.testing.assert_allclose(render_dense(pt.detach(), degree, c, bg).numpy(),
                                   O.render(p, degree, c, bg=bg)["image"], atol=1e-12)
    grads, _, _ = O.render_backward(p, degree, cams, wimg, bg=bg)
    scale = np.abs(ref).max()
    np.testing.assert_allclose(grads, ref, atol=1e-9 * scale, rtol=1e-9)


def test_backward_frozen_rows_untouched_and_active_unchanged():
    p, cams = tiny_scene(n=64, degree=3, size=32, log_s_shift=0.9)
    wimg = np.random.default_rng(13).standard_normal((2, 3, 32, 32))
    frozen = (np.arange(64) % 3 == 0).astype(np.uint8)
    init = np.full((p.shape[0], 64), 7.0)
    g_all, _, _ = O.render_backward(p, 3, cams, wimg)
    g_fz, _, _ = O.render_backward(p, 3, cams, wimg, frozen=frozen, grads_init=init)
    assert (g_fz[:, frozen == 1] == 7.0).all()
    np.testing.assert_array_equal(g_fz[:, frozen == 0], g_all[:, frozen == 0])


# ---------------------------------------------------------------------------
# Adam (Section 3.2.4 optimizer restricted to non-frozen Gaussians)
# ---------------------------------------------------------------------------

def test_l1_loss_and_psnr_hand_values():
    """Eq. 3 with lambda_SSIM = 0: L = mean |C - C*|, dL/dC = sign(C - C*) /
    count with sign(0) = 0; the PSNR clamps the rendered image only."""
    C = np.array([0.5, 1.2, -0.1, 0.3]).reshape(1, 1, 2, 2)
    T = np.array([0.5, 1.1, 0.0, 0.6]).reshape(1, 1, 2, 2)
    loss, dL, mse = O.l1_loss(C, T)
    assert loss == pytest.approx((0.0 + 0.1 + 0.1 + 0.3) / 4, abs=1e-15)
    np.testing.assert_array_equal(dL.reshape(-1), [0.0, 0.25, -0.25, -0.25])
    # clamp(C) = (0.5, 1.0, 0.0, 0.3): errors (0, -0.1, 0, -0.3); a clamped target would give 0 at index 1
    assert mse == pytest.approx((0.01 + 0.09) / 4, abs=1e-15)
    assert O.psnr(mse) == pytest.approx(10.0 * math.log10(40.0), abs=1e-12)
    assert O.psnr(0.01) == pytest.approx(20.0, abs=1e-12)
    # the count is every value of every view and channel
    C2 = np.zeros((2, 3, 4, 5))
    T2 = np.zeros_like(C2)
    C2[1, 2, 3, 4] = 0.6
    loss2, dL2, mse2 = O.l1_loss(C2, T2)
    assert loss2 == pytest.approx(0.6 / 120, abs=1e-15)
    assert dL2[1, 2, 3, 4] == pytest.approx(1.0 / 120, abs=1e-15)
    assert np.count_nonzero(dL2) == 1
    assert mse2 == pytest.approx(0.36 / 120, abs=1e-15)


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(14)
    R, n = 14, 50
    p0 = rng.standard_normal((R, n))
    lrs = np.linspace(1e-3, 2e-2, R)
    pt = [torch.tensor(p0[r].copy(), requires_grad=True) for r in range(R)]
    opt = torch.optim.Adam([{"params": [pt[r]], "lr": float(lrs[r])} for r in range(R)],
                           betas=(0.9, 0.999), eps=1e-15)
    p, m, v = p0.copy(), np.zeros((R, n)), np.zeros((R, n))
    for step in range(1, 6):
        g = rng.standard_normal((R, n))
        for r in range(R):
            pt[r].grad = torch.tensor(g[r].copy())
        opt.step()
        p, m, v = O.adam_masked(p, g, m, v, lrs, 0.9, 0.999, 1e-15, step)
        np.testing.assert_allclose(p, np.stack([x.detach().numpy() for x in pt]), rtol=1e-12, atol=1e-14)


def test_adam_first_step_closed_form_and_frozen():
    rng = np.random.default_rng(15)
    R, n = 59, 40
    p0, g = rng.standard_normal((R, n)), rng.standard_normal((R, n))
    lrs = np.full(R, 0.01)
    p1, m1, v1 = O.adam_masked(p0, g, np.zeros((R, n)), np.zeros((R, n)), lrs, 0.9, 0.999, 1e-15, 1)
    np.testing.assert_allclose(p1, p0 - 0.01 * g / (np.abs(g) + 1e-15), rtol=1e-12)
    frozen = np.ones(n, np.uint8)
    m0, v0 = rng.random((R, n)), rng.random((R, n))
    p2, m2, v2 = O.adam_masked(p0, g, m0, v0, lrs, 0.9, 0.999, 1e-15, 3, frozen)
    assert np.array_equal(p2, p0) and np.array_equal(m2, m0) and np.array_equal(v2, v0)


# ---------------------------------------------------------------------------
# Scores and freezing (eqs. 4-6) and the host schedule (eqs. 5, 7; Section 3.2.3)
# ---------------------------------------------------------------------------

def test_freeze_rule_hand_cases():
    sx = np.array([1e-5, 1e-5, 5e-5, 2e-5, 3e-5, np.finfo(np.float32).max], np.float32)
    sr = np.array([1e-5, 2e-4, 1e-5, 9e-5, 1e-5, 0.0], np.float32)
    old = np.array([0, 1, 0, 0, 0, 0], np.uint8)
    # eq. 4 strict: 3e-5 is not < 3e-5; eq. 6: both groups must pass
    assert list(O.freeze_update(old, sx, sr, 3e-5, 1e-4, 0)) == [1, 1, 0, 1, 0, 0]
    assert list(O.freeze_update(old, sx, sr, 3e-5, 1e-4, 2)) == [1, 0, 0, 1, 0, 0]
    assert list(O.freeze_update(old, sx, sr, 3e-5, 1e-4, 1)) == [0] * 6
    prop = np.array([0, 0, 1, 0, 0, 0], np.uint8)
    assert list(O.freeze_update(old, sx, sr, 3e-5, 1e-4, 0, prop)) == [1, 1, 1, 1, 0, 0]


def test_partition_order_hand_case_and_stable_sort():
    f = np.array([1, 0, 0, 1, 1, 0, 1], np.uint8)
    src, na = O.partition_order(f)
    assert na == 3 and list(src) == [1, 2, 5, 0, 3, 4, 6]
    # a stable sort by the 0/1 key is the same ordering
    rng = np.random.default_rng(4)
    for n in (0, 1, 63, 64, 65, 1000):
        f = (rng.random(n) < 0.6).astype(np.uint8)
        src, na = O.partition_order(f)
        assert np.array_equal(src, np.argsort(f, kind="stable")) and na == int((f == 0).sum())
    x = np.arange(14).reshape(2, 7)
    src, _ = O.partition_order(np.array([1, 0, 0, 1, 1, 0, 1]))
    assert O.apply_partition(x, src)[1].tolist() == [8, 9, 12, 7, 10, 11, 13]


def test_ema_hand_cases():
    big = np.finfo(np.float32).max
    ema = np.array([big, 2.0, 2.0, 2.0])
    g = np.array([0.5, 1.0, 1.0, 1.0])
    vis = np.array([1, 1, 0, 1])
    fz = np.array([0, 0, 0, 1])
    out = O.ema_update(ema, g, vis, fz, 0.9)
    np.testing.assert_allclose(out, [0.5, 1.9, 2.0, 2.0])


def test_scores_definition():
    g = np.zeros((59, 2))
    g[0:3, 0] = [3, 4, 0]
    g[11:14, 0] = [0, 0, 2]
    g[10, 1] = -0.5
    g[3:6, 1] = [1, 2, 2]
    gx, gr, go, gs = O.scores(g)
    assert list(gx) == [5, 0] and list(gr) == [2, 0] and list(go) == [0, 0.5] and list(gs) == [0, 3]


def test_threshold_schedule_hand_values():
    e0, K = 3e-5, 2000
    assert O.freeze_threshold(0, K, e0) == pytest.approx(1.5e-5)
    assert O.freeze_threshold(1000, K, e0) == pytest.approx(3.75e-5)
    assert O.freeze_threshold(2000, K, e0) == pytest.approx(4.5e-5)
    assert O.freeze_threshold(1500, K, e0, k_stop=1000) == pytest.approx(3.75e-5)
    assert O.freeze_threshold(1000, K, e0, linear=True) == pytest.approx(3e-5)


def test_early_stop_hand_sequences():
    assert not O.early_stop([20.0, 25.0])
    assert not O.early_stop([20.0, 25.0, 25.1])          # earlier gain 5 dB
    assert O.early_stop([20.0, 25.0, 25.1, 25.15])        # gains 0.1, 0.05
    assert not O.early_stop([25.0, 25.1, 25.5])           # latest gain 0.4


def test_plateau_lr_hand_sequence():
    s = O.PlateauLR(factor=0.75, patience=1, eps=1.0)
    seq = [20.0, 20.5, 20.8, 22.0, 22.3, 22.4, 22.5, 22.6]
    scales = [s.step(x) for x in seq]
    assert scales == [1, 1, 0.75, 0.75, 0.75, 0.5625, 0.5625, 0.421875]


def test_sampled_pixels_equal_full_render():
    p, cams = tiny_scene(n=500, degree=3, size=48, log_s_shift=0.8)
    r = O.render(p, 3, cams[0], bg=(0.2, 0.1, 0.4))
    pix = np.array([[x, y] for y in range(0, 48, 5) for x in range(0, 48, 3)])
    out, T, mv = O.render_pixels(p, 3, cams[0], pix, bg=(0.2, 0.1, 0.4))
    assert np.array_equal(out, r["image"][:, pix[:, 1], pix[:, 0]].T)
    assert np.array_equal(T, r["T_final"][pix[:, 1], pix[:, 0]])
    # the brute walk also sees Gaussians outside the pixel's tile, so its
    # decision margin can only be smaller
    assert (mv <= r["m_value"][pix[:, 1], pix[:, 0]]).all()


# ---------------------------------------------------------------------------
# Densification, pruning, opacity reset (Section 3.1, Section 4.1)
# ---------------------------------------------------------------------------

def test_screen_gradient_equals_principal_point_derivative():
    """dL/du of a lone Gaussian equals dL/dcx (u = fx x/z + cx, and cx enters
    nowhere else), likewise dL/dv and cy: pins the screen-space part of the
    per-view 2-D gradient that densification uses."""
    import dataclasses
    cam = S.config_cameras("c1")[0]
    p = _single([0.1, 0.15, -0.2], [math.log(0.07), math.log(0.05), math.log(0.06)],
                q=(0.9, 0.2, -0.3, 0.1), logit=0.4)
    w = np.random.default_rng(2).standard_normal((1, 3, cam.height, cam.width))

    def L(c):
        return (O.render(p, 0, c)["image"] * w[0]).sum()

    _, g2, vis = O.render_backward(p, 0, [cam], w)
    assert vis[0, 0] == 1
    h = 1e-5
    for k, name in ((0, "cx"), (1, "cy")):
        cp = dataclasses.replace(cam, **{name: getattr(cam, name) + h})
        cm = dataclasses.replace(cam, **{name: getattr(cam, name) - h})
        fd = (L(cp) - L(cm)) / (2 * h)
        assert g2[0, k, 0] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_densify_stats_hand_values():
    g2 = np.zeros((2, 9, 3))
    g2[0, 0], g2[0, 1] = [0.3, 0.0, 1.0], [0.4, 2.0, 1.0]
    g2[1, 0], g2[1, 1] = [0.6, 0.0, 0.0], [0.8, 0.0, 0.0]
    vis = np.array([[1, 1, 1], [1, 0, 0]])
    grads = np.zeros((14, 3))
    grads[11:14, 0] = [2.0, 3.0, 6.0]                # |.| = 7
    grads[11:14, 1] = [0.0, 0.0, 1.0]
    acc = O.densify_stats(np.zeros((4, 3)), g2, vis, grads, np.array([0, 0, 1]), width=2, height=2)
    # W/2 = H/2 = 1: norms 0.5 (view 0) + 1.0 (view 1) for G0, 2.0 for G1; G2 frozen
    np.testing.assert_allclose(acc[0], [1.5, 2.0, 0.0])
    np.testing.assert_allclose(acc[1], [2, 1, 0])
    np.testing.assert_allclose(acc[2], [7.0, 1.0, 0.0])
    np.testing.assert_allclose(acc[3], [1, 1, 0])
    acc2 = O.densify_stats(acc, g2, vis, grads, None, width=4, height=2)
    np.testing.assert_allclose(acc2[0], [1.5 + math.hypot(0.6, 0.4) + math.hypot(1.2, 0.8), 2.0 + 2.0,
                                         math.hypot(2.0, 1.0)])


def _dens_case():
    """Seven Gaussians, one per rule: 0 below threshold, 1 clone, 2 split,
    3 selected but pruned, 4 frozen, 5 selected by the colour criterion only,
    6 never visible."""
    n = 7
    P = np.zeros((14, n))
    P[0:3] = np.arange(3 * n, dtype=float).reshape(3, n) * 0.1
    P[3:6] = math.log(0.01)
    P[3:6, 2] = [math.log(0.2), math.log(0.3), math.log(0.4)]       # big: split
    P[6] = 1.0
    P[10] = 1.0
    P[10, 3] = -6.0                                                   # o = 0.0025 < 0.005
    P[11:14] = np.arange(3 * n).reshape(3, n)
    st = np.zeros((4, n), np.float32)
    st[0] = [1e-4, 6e-4, 9e-4, 8e-4, 7e-4, 1e-5, 0.0]
    st[1] = [2, 2, 3, 2, 1, 1, 0]
    st[2] = [0, 0, 0, 0, 0, 5e-6, 9.0]
    st[3] = [1, 1, 1, 1, 1, 1, 0]
    fz = np.array([0, 0, 0, 0, 1, 0, 0], np.uint8)
    M = np.full((14, n), 0.5)
    V = np.full((14, n), 0.25)
    E = np.arange(4 * n, dtype=float).reshape(4, n)
    noise = np.zeros((6, n))
    noise[0:3, 2] = [1.0, 0.0, 0.0]
    noise[3:6, 2] = [0.0, -2.0, 0.5]
    return P, M, V, E, fz, st, noise


def test_densify_prune_hand_case():
    P, M, V, E, fz, st, noise = _dens_case()
    thr, split_ls, prune_lg = 2e-4, math.log(0.01 * 10.0), math.log(0.005 / 0.995)
    for use_rgb in (False, True):
        nP, nM, nV, nE, nF, cnt = O.densify_prune(P, M, V, E, fz, st, noise, thr, 1e-6, use_rgb,
                                                  split_ls, prune_lg, math.log(1.6))
        kept = [0, 1, 4, 5, 6]
        clones = [1, 5] if use_rgb else [1]
        assert cnt == (len(kept) + len(clones) + 2, len(kept), len(clones), 1)
        np.testing.assert_array_equal(nP[:, :len(kept)], P[:, kept])
        np.testing.assert_array_equal(nP[:, len(kept):len(kept) + len(clones)], P[:, clones])
        c0, c1 = nP[:, -2], nP[:, -1]
        s = np.array([0.2, 0.3, 0.4])
        # identity rotation: offsets are scale * noise
        np.testing.assert_allclose(c0[0:3], P[0:3, 2] + s * [1.0, 0.0, 0.0], rtol=1e-14)
        np.testing.assert_allclose(c1[0:3], P[0:3, 2] + s * [0.0, -2.0, 0.5], rtol=1e-14)
        np.testing.assert_allclose(c0[3:6], np.log(s / 1.6), rtol=1e-14)
        np.testing.assert_array_equal(c0[6:], P[6:, 2])
        nk = len(kept)
        np.testing.assert_array_equal(nM[:, :nk], M[:, kept])
        assert (nM[:, nk:] == 0).all() and (nV[:, nk:] == 0).all()
        np.testing.assert_array_equal(nE[:, :nk], E[:, kept])
        assert (nE[:, nk:] == O.FLT_MAX).all()
        np.testing.assert_array_equal(nF, [0, 0, 1, 0, 0] + [0] * (len(clones) + 2))


def test_split_children_rotation_closed_form():
    th = 0.7
    q = (math.cos(th / 2), 0.0, 0.0, math.sin(th / 2))                # rotation about z by th
    P = _single([1.0, 2.0, 3.0], [math.log(0.5), math.log(0.2), math.log(0.1)], q=q)
    st = np.array([[1.0], [1.0], [0.0], [1.0]], np.float32)
    noise = np.array([[1.0], [0.0], [0.0], [0.0], [1.0], [2.0]])
    nP, *_, cnt = O.densify_prune(P, np.zeros_like(P), np.zeros_like(P), None, None, st, noise, 0.5, 1.0,
                                  False, math.log(0.1), -10.0, math.log(1.6))
    assert cnt == (2, 0, 0, 1)
    np.testing.assert_allclose(nP[0:3, 0], [1 + 0.5 * math.cos(th), 2 + 0.5 * math.sin(th), 3.0], atol=1e-14)
    np.testing.assert_allclose(nP[0:3, 1], [1 - 0.2 * math.sin(th), 2 + 0.2 * math.cos(th), 3.2], atol=1e-14)


def test_opacity_reset_hand_values():
    P = np.zeros((14, 4))
    P[10] = [-6.0, -3.0, 2.0, 5.0]
    M = np.ones((14, 4))
    V = np.ones((14, 4))
    cap = math.log(0.01 / 0.99)                                       # -4.595
    nP, nM, nV = O.opacity_reset(P, M, V, np.array([0, 0, 0, 1]), cap)
    np.testing.assert_allclose(nP[10], [-6.0, float(np.float32(cap)), float(np.float32(cap)), 5.0])
    np.testing.assert_array_equal(nM[10], [0, 0, 0, 1])
    np.testing.assert_array_equal(nV[10], [0, 0, 0, 1])
    assert (nM[:10] == 1).all() and (nP[:10] == 0).all()


# ---------------------------------------------------------------------------
# Learned freeze proposer (project extension)
# ---------------------------------------------------------------------------

def _mlp_case(n=300, seed=0):
    rng = np.random.default_rng(seed)
    wf = np.zeros(O.MLP_COUNT)
    o = O.MLP_OFF
    wf[o["W1"]:o["b1"]] = rng.standard_normal(2048) / np.sqrt(32)
    wf[o["b1"]:o["W2"]] = 0.1 * rng.standard_normal(64)
    wf[o["W2"]:o["b2"]] = rng.standard_normal(4096) / 8.0
    wf[o["b2"]:o["w3"]] = 0.1 * rng.standard_normal(64)
    wf[o["w3"]:o["b3"]] = rng.standard_normal(64) / 8.0
    wf[o["b3"]] = 0.3
    wf = wf.astype(np.float32).astype(np.float64)
    x = O.bf16_round(rng.standard_normal((n, 32)))
    return x, wf


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(1)
    v = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-20, 20, 5000),
                        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 0.0, 2.0 ** -130]]).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(O.bf16_round(v), ref)
    assert O.bf16_round(np.float32(1.0 + 2.0 ** -8)) == 1.0            # tie to even
    assert O.bf16_round(np.float32(1.0 + 3 * 2.0 ** -8)) == 1.0 + 2.0 ** -6


def _torch_mlp(x, wf):
    """The same network written with torch float64 ops and torch's bf16
    casts, the roundings passed straight through in the derivative."""
    def rnd(t):
        return t + (t.to(torch.float32).to(torch.bfloat16).to(torch.float64) - t).detach()
    o = O.MLP_OFF
    w = torch.tensor(wf, dtype=torch.float64, requires_grad=True)
    W1 = w[o["W1"]:o["b1"]].view(64, 32)
    W2 = w[o["W2"]:o["b2"]].view(64, 64)
    h1 = rnd(torch.relu(torch.tensor(x) @ rnd(W1).T + w[o["b1"]:o["W2"]]))
    h2 = torch.relu(h1 @ rnd(W2).T + w[o["b2"]:o["w3"]])
    z = h2 @ w[o["w3"]:o["b3"]] + w[o["b3"]]
    return z, w


def test_mlp_forward_backward_match_torch():
    x, wf = _mlp_case()
    z, h1, h2 = O.mlp_forward(x, wf)
    zt, w = _torch_mlp(x, wf)
    np.testing.assert_allclose(z, zt.detach().numpy(), rtol=1e-12, atol=1e-12)
    dz = np.random.default_rng(3).standard_normal(x.shape[0])
    (zt * torch.tensor(dz)).sum().backward()
    np.testing.assert_allclose(O.mlp_backward(x, wf, dz), w.grad.numpy(), rtol=1e-10, atol=1e-12)
    assert (h1 > 0).mean() > 0.2 and (h2 > 0).mean() > 0.2


def test_mlp_backward_finite_differences_on_unrounded_parameters():
    # b2, w3 and b3 enter without rounding: central differences apply
    x, wf = _mlp_case(n=50)
    dz = np.random.default_rng(4).standard_normal(50)
    g = O.mlp_backward(x, wf, dz)
    o = O.MLP_OFF
    for k in [o["b2"] + 3, o["b2"] + 40, o["w3"] + 5, o["w3"] + 63, o["b3"]]:
        h = 1e-6
        wp, wm = wf.copy(), wf.copy()
        wp[k] += h
        wm[k] -= h
        fd = ((O.mlp_forward(x, wp)[0] - O.mlp_forward(x, wm)[0]) @ dz) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-7, abs=1e-9)


def test_bce_closed_forms():
    loss, dz = O.bce(np.array([0.0, 0.0]), np.array([1, 0]))
    assert loss == pytest.approx(math.log(2.0))
    np.testing.assert_allclose(dz, [-0.25, 0.25])
    loss, dz = O.bce(np.array([50.0, -50.0]), np.array([1, 0]))
    assert loss == pytest.approx(math.exp(-50.0), rel=1e-6)


def test_propose_veto_and_labels_hand_cases():
    thr = math.log(0.9 / 0.1)
    z = np.array([3.0, 3.0, 3.0, 1.0, 2.2])
    sx = np.array([1e-6, 9e-5, 1e-6, 1e-6, 1e-6])
    sr = np.array([1e-6, 1e-6, 3e-4, 1e-6, 1e-6])
    # veto at 3 x (3e-5, 1e-4)
    np.testing.assert_array_equal(O.propose(z, sx, sr, thr, 9e-5, 3e-4), [1, 0, 0, 0, 1])
    np.testing.assert_array_equal(O.proposer_labels([0, 1, 0, 1], [0, 0, 1, 1]), [0, 1, 1, 1])


def test_traj_features_hand_case():
    n = 3
    ring = np.zeros((8, 4, n))
    for e in range(8):
        ring[e] = 10.0 ** (-(e + 1))                   # entry e holds 10^-(e+1)
    mean, std = np.zeros(32), np.ones(32)
    x = O.traj_features(ring, 5, mean, std)
    # feature 4j + q reads entry (5 - j) mod 8
    for j in range(8):
        e = (5 - j) % 8
        np.testing.assert_allclose(x[:, 4 * j:4 * j + 4], O.bf16_round(np.full((n, 4), -(e + 1.0))), rtol=0)
    x2 = O.traj_features(ring, 5, np.full(32, -4.0), np.full(32, 2.0))
    assert (x2[:, 0] == -1.0).all()                   # (log10(1e-6) + 4) / 2
    assert O.traj_features(np.zeros((8, 4, 1)), 0, mean, std)[0, 0] == O.bf16_round(-12.0)
