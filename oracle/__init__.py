"""FP64 CPU oracle of the GSta training path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  The GPU library never loads it and shares no code with
it.  The rasterizer (projection, binning, compositing, backward) lives in
``gsta_oracle.cpp`` (plain double-precision C++); the element-wise steps
(loss, Adam, gradient-norm scores, freezing, threshold schedule, early stop,
plateau learning rate) are written here in numpy float64.

Paper: "GSta: Efficient Training Scheme with Siestaed Gaussians for Monocular
3D Scene Reconstruction" (arXiv 2504.06716).  Each function names the
section or equation it follows.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gsta_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
NREC = 40
_lib = None


def build(force: bool = True) -> str:
    """Compile the C++ oracle (g++, FP64, no floating-point contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC",
               "-o", _LIB, _SRC]
        subprocess.run(cmd, check=True)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        L.oracle_project.argtypes = [P, i64, i64, i32, P, i32, i32, P]
        L.oracle_bin.argtypes = [P, i64, i64, i32, P, i32, i32, P, P, P, P]
        L.oracle_bin.restype = i64
        L.oracle_render.argtypes = [P, i64, i64, i32, P, i32, i32, P, i32] + [P] * 8
        L.oracle_render_backward.argtypes = [P, i64, i64, i32, P, i32, i32, i32, P, P, P, P, P, P]
        L.oracle_sh_basis.argtypes = [i32, P, i64, P, P]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_opacity_activation.argtypes = [ctypes.c_int]
        L.oracle_set_sh_mask.argtypes = [P, i64, ctypes.c_double, P]
        L.oracle_render_pixels.argtypes = [P, i64, i64, i32, P, P, P, i64, P, P, P]
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_threads(n: int) -> None:
    """Threads of the C++ oracle's parallel loops from now on."""
    lib().oracle_set_threads(int(n))


class opacity_activation:
    """Context in which the rasterizer reads row 10 as the opacity itself,
    opacity = |x| (act 1, the finetune stage of Section 4.1), instead of
    sigmoid(x) (act 0)."""

    def __init__(self, act: int):
        self.act = int(act)

    def __enter__(self):
        lib().oracle_set_opacity_activation(self.act)
        return self

    def __exit__(self, *exc):
        lib().oracle_set_opacity_activation(0)
        return False


class sh_mask:
    """Context in which the rasterizer gates SH bands 1..3 of every Gaussian
    with the hard masks of Section 3.3: M_l = 1 if sigmoid(logit_l) exceeds
    `threshold`, else 0, multiplying each coefficient of band l (band 0 is
    never masked).  render_backward inside the context also writes the
    straight-through gradient dL/dlogit = dL/dM sigmoid'(logit) into
    ``self.grad`` ([3, n]; frozen columns keep zero)."""

    def __init__(self, logits, threshold):
        self.logits = np.ascontiguousarray(logits, dtype=np.float64)
        assert self.logits.ndim == 2 and self.logits.shape[0] == 3
        self.threshold = float(threshold)
        self.grad = np.zeros_like(self.logits)

    def __enter__(self):
        n = self.logits.shape[1]
        lib().oracle_set_sh_mask(_ptr(self.logits), n, self.threshold,
                                 _ptr(self.grad))
        return self

    def __exit__(self, *exc):
        lib().oracle_set_sh_mask(None, 0, 0.0, None)
        return False


def sh_band_gates(logits, threshold):
    """Hard band gates M [3, n] (Section 3.3): 1 where sigmoid(logit) >
    threshold, decided as the rasterizer does, float32 logit > float32
    ln(t / (1 - t))."""
    xt = np.float32(math.log(threshold / (1.0 - threshold)))
    return (np.asarray(logits, np.float64).astype(np.float32) > xt).astype(np.float64)


def sh_mask_reg(logits, lam):
    """Sparsity term on the band masks, lam times the mean of sigmoid(logit)
    over every Gaussian and band, and its gradient with respect to the
    logits."""
    x = np.asarray(logits, np.float64)
    sg = 1.0 / (1.0 + np.exp(-x))
    return lam * sg.mean(), lam * sg * (1.0 - sg) / x.size


def opacity_to_absolute(params, m, v):
    """The switch to the absolute activation when the finetune starts:
    row 10 <- sigmoid(row 10) (every opacity unchanged) and the moments of
    row 10 restart from zero."""
    P = np.array(params, np.float64)
    M = np.array(m, np.float64)
    V = np.array(v, np.float64)
    P[10] = 1.0 / (1.0 + np.exp(-P[10]))
    M[10] = 0.0
    V[10] = 0.0
    return P, M, V


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _as_f64(params: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(params, dtype=np.float64)


def cam_vec(cam) -> np.ndarray:
    """Camera as the 22 doubles the C oracle reads."""
    v = np.zeros(22, dtype=np.float64)
    v[0], v[1] = cam.width, cam.height
    v[2:6] = [cam.fx, cam.fy, cam.cx, cam.cy]
    v[6:18] = np.concatenate([np.asarray(cam.R, np.float64), np.asarray(cam.t, np.float64)[:, None]],
                             axis=1).reshape(-1)
    v[18:21] = cam.campos
    v[21] = cam.near
    return v


def n_rows(degree: int) -> int:
    return 11 + 3 * (degree + 1) ** 2


# ---------------------------------------------------------------------------
# Rasterizer (Section 3.1, eqs. 1-2; Section 3.2.4)
# ---------------------------------------------------------------------------

def project(params, degree, cam, tile=16):
    """Per-Gaussian projected records (see oracle_project for the layout)."""
    P = _as_f64(params)
    n = P.shape[1]
    rec = np.zeros((n, NREC), dtype=np.float64)
    lib().oracle_project(_ptr(P), n, n, degree, _ptr(cam_vec(cam)), tile, tile, _ptr(rec))
    return rec


def bin_tiles(params, degree, cam, tile=16):
    """Per-tile depth-ordered id lists: (counts [T], ids [I], depth order)."""
    P = _as_f64(params)
    n = P.shape[1]
    cv = cam_vec(cam)
    ntiles = ((cam.width + tile - 1) // tile) * ((cam.height + tile - 1) // tile)
    counts = np.zeros(ntiles, dtype=np.int64)
    nvis = np.zeros(1, dtype=np.int64)
    order = np.zeros(n, dtype=np.int64)
    total = lib().oracle_bin(_ptr(P), n, n, degree, _ptr(cv), tile, tile, _ptr(counts), None,
                             _ptr(order), _ptr(nvis))
    ids = np.zeros(max(total, 1), dtype=np.int64)
    lib().oracle_bin(_ptr(P), n, n, degree, _ptr(cv), tile, tile, _ptr(counts), _ptr(ids), None, None)
    return counts, ids[:total], order[: int(nvis[0])]


def render(params, degree, cam, tile=16, bg=(0.0, 0.0, 0.0), brute=False):
    """Forward render of one view (eq. 2) with per-pixel decision margins."""
    P = _as_f64(params)
    n = P.shape[1]
    H, W = cam.height, cam.width
    out = dict(
        image=np.zeros((3, H, W)), T_final=np.zeros((H, W)),
        last=np.zeros((H, W), np.int64), n_members=np.zeros((H, W), np.int64),
        m_value=np.zeros((H, W)), m_grad=np.zeros((H, W)), ztie=np.zeros((H, W)),
        hash=np.zeros((H, W), np.uint64))
    bgv = np.asarray(bg, dtype=np.float64)
    lib().oracle_render(_ptr(P), n, n, degree, _ptr(cam_vec(cam)), tile, tile, _ptr(bgv), int(brute),
                        _ptr(out["image"]), _ptr(out["T_final"]), _ptr(out["last"]),
                        _ptr(out["n_members"]), _ptr(out["m_value"]), _ptr(out["m_grad"]),
                        _ptr(out["ztie"]), _ptr(out["hash"]))
    return out


def render_pixels(params, degree, cam, pix, bg=(0.0, 0.0, 0.0)):
    """Brute-force colour, T_final and decision margin of sampled pixels
    pix [m, 2] = (px, py) of one view."""
    P = _as_f64(params)
    n = P.shape[1]
    px = np.ascontiguousarray(pix, dtype=np.int64)
    m = px.shape[0]
    out, T, mv = np.zeros((m, 3)), np.zeros(m), np.zeros(m)
    bgv = np.asarray(bg, dtype=np.float64)
    lib().oracle_render_pixels(_ptr(P), n, n, degree, _ptr(cam_vec(cam)), _ptr(bgv), _ptr(px), m, _ptr(out),
                               _ptr(T), _ptr(mv))
    return out, T, mv


def render_backward(params, degree, cams, dL_dimage, frozen=None, tile=16, bg=(0.0, 0.0, 0.0),
                    grads_init=None):
    """Parameter gradients summed over views (Section 3.2.4).

    Frozen columns keep ``grads_init`` (zeros by default).  Returns
    (grads [R, n], grad2d [V, 9, n], visible [V, n]).
    """
    P = _as_f64(params)
    R, n = P.shape
    V = len(cams)
    cv = np.concatenate([cam_vec(c) for c in cams])
    dL = np.ascontiguousarray(dL_dimage, dtype=np.float64)
    grads = np.zeros((R, n)) if grads_init is None else np.array(grads_init, dtype=np.float64)
    g2 = np.zeros((V, 9, n))
    vis = np.zeros((V, n), np.uint8)
    fz = None if frozen is None else np.ascontiguousarray(frozen, dtype=np.uint8)
    bgv = np.asarray(bg, dtype=np.float64)
    lib().oracle_render_backward(_ptr(P), n, n, degree, _ptr(cv), V, tile, tile, _ptr(bgv), _ptr(dL),
                                 None if fz is None else _ptr(fz), _ptr(grads), _ptr(g2), _ptr(vis))
    return grads, g2, vis


def sh_basis(degree, dirs, with_grad=False):
    d = np.ascontiguousarray(dirs, dtype=np.float64)
    m = d.shape[0]
    K = (degree + 1) ** 2
    out = np.zeros((m, K))
    g = np.zeros((m, K, 3)) if with_grad else None
    lib().oracle_sh_basis(degree, _ptr(d), m, _ptr(out), None if g is None else _ptr(g))
    return (out, g) if with_grad else out


# ---------------------------------------------------------------------------
# Loss (eq. 3, L1 part) and PSNR
# ---------------------------------------------------------------------------

def l1_loss(image, target):
    """L = mean |C - C*| (eq. 3 with lambda_SSIM = 0); dL/dC = sign(C - C*) / count.

    PSNR = 10 log10(1 / MSE) with C clamped to [0, 1].
    """
    C = np.asarray(image, np.float64)
    Ct = np.asarray(target, np.float64)
    d = C - Ct
    count = d.size
    loss = np.abs(d).sum() / count
    dL = np.sign(d) / count
    mse = ((np.clip(C, 0.0, 1.0) - Ct) ** 2).sum() / count
    return loss, dL, mse


def psnr(mse):
    return 10.0 * np.log10(1.0 / mse)


# ---------------------------------------------------------------------------
# D-SSIM term of eq. 3 (lambda_SSIM = 0.2) and the loss of eq. 3.  SSIM is
# the structural similarity of Wang et al. (2004) with the window that 3D
# Gaussian splatting uses: an 11 x 11 Gaussian of standard deviation 1.5,
# normalised, applied per channel as a zero-padded 'same' 2-D filter;
# C1 = 0.01^2, C2 = 0.03^2.  L_D-SSIM = 1 - mean of the SSIM map over every
# view, channel and pixel.
# ---------------------------------------------------------------------------

SSIM_C1, SSIM_C2 = 0.01 ** 2, 0.03 ** 2
SSIM_RADIUS, SSIM_SIGMA = 5, 1.5


def ssim_window_1d():
    """The 11 taps exp(-(i - 5)^2 / (2 * 1.5^2)), normalised to sum 1."""
    i = np.arange(2 * SSIM_RADIUS + 1, dtype=np.float64) - SSIM_RADIUS
    g = np.exp(-(i * i) / (2.0 * SSIM_SIGMA * SSIM_SIGMA))
    return g / g.sum()


def filter2d_same(img, w1):
    """out(y, x) = sum over a, b of w(a) w(b) img(y + a - r, x + b - r), with
    img taken as zero outside the image: the 2-D window is the outer product
    of the 1-D taps, written here as a plain sum over its 121 offsets.  img
    is [..., H, W]."""
    img = np.asarray(img, np.float64)
    r = (len(w1) - 1) // 2
    H, W = img.shape[-2], img.shape[-1]
    pad = np.zeros(img.shape[:-2] + (H + 2 * r, W + 2 * r))
    pad[..., r:r + H, r:r + W] = img
    out = np.zeros_like(img)
    for a in range(2 * r + 1):
        for b in range(2 * r + 1):
            out += w1[a] * w1[b] * pad[..., a:a + H, b:b + W]
    return out


def ssim_map(x, y):
    """SSIM map of images x, y ([..., H, W], per channel): with mu = G*x,
    sigma_x^2 = G*(x^2) - mu_x^2, sigma_xy = G*(x y) - mu_x mu_y,
    S = (2 mu_x mu_y + C1)(2 sigma_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(sigma_x^2 + sigma_y^2 + C2))."""
    w = ssim_window_1d()
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    mx, my = filter2d_same(x, w), filter2d_same(y, w)
    sxx = filter2d_same(x * x, w) - mx * mx
    syy = filter2d_same(y * y, w) - my * my
    sxy = filter2d_same(x * y, w) - mx * my
    return ((2 * mx * my + SSIM_C1) * (2 * sxy + SSIM_C2)) / ((mx * mx + my * my + SSIM_C1) * (sxx + syy + SSIM_C2))


def dssim_loss(image, target):
    """L_D-SSIM = 1 - mean SSIM over every value of image [V, 3, H, W], and its
    gradient with respect to the image.  With m = G*x, s = G*(x^2), c =
    G*(x y) the map S depends on x only through (m, s, c) at each pixel, so
    dL/dx = G*(g_m) + 2 x G*(g_s) + y G*(g_c) with g_q = dL/dS * dS/dq:
    dS/dm = S (2 mu_y / A - 2 mu_y / B - 2 mu_x / C + 2 mu_x / D),
    dS/ds = -S / D, dS/dc = 2 S / B (A, B, C, D the four factors of S), and
    the filter is its own adjoint (symmetric taps, zero padding)."""
    w = ssim_window_1d()
    x = np.asarray(image, np.float64)
    y = np.asarray(target, np.float64)
    mx, my = filter2d_same(x, w), filter2d_same(y, w)
    sxx = filter2d_same(x * x, w) - mx * mx
    syy = filter2d_same(y * y, w) - my * my
    sxy = filter2d_same(x * y, w) - mx * my
    A = 2 * mx * my + SSIM_C1
    B = 2 * sxy + SSIM_C2
    C = mx * mx + my * my + SSIM_C1
    D = sxx + syy + SSIM_C2
    S = (A * B) / (C * D)
    count = S.size
    loss = 1.0 - S.sum() / count
    dS = -1.0 / count
    gm = dS * S * (2 * my / A - 2 * my / B - 2 * mx / C + 2 * mx / D)
    gs = dS * (-S / D)
    gc = dS * (2 * S / B)
    grad = filter2d_same(gm, w) + 2 * x * filter2d_same(gs, w) + y * filter2d_same(gc, w)
    return loss, grad, S.sum()


def total_loss(image, target, lam=0.2):
    """Eq. 3: L = (1 - lambda) L1 + lambda L_D-SSIM, and dL/dimage."""
    l1, g1, _ = l1_loss(image, target)
    ld, gd, _ = dssim_loss(image, target)
    return (1 - lam) * l1 + lam * ld, (1 - lam) * g1 + lam * gd


# ---------------------------------------------------------------------------
# Masked Adam (Section 3.2.4: frozen Gaussians are not updated)
# ---------------------------------------------------------------------------

def adam_masked(p, g, m, v, lr_rows, beta1, beta2, eps, step, frozen=None):
    """One Adam step (Kingma & Ba, bias-corrected, global step ``step``)
    on an [R, n] block; columns with frozen != 0 are left untouched."""
    p = np.array(p, np.float64)
    g = np.asarray(g, np.float64)
    m = np.array(m, np.float64)
    v = np.array(v, np.float64)
    lr = np.asarray(lr_rows, np.float64)[:, None]
    act = np.ones(p.shape[1], bool) if frozen is None else (np.asarray(frozen) == 0)
    m_new = beta1 * m + (1.0 - beta1) * g
    v_new = beta2 * v + (1.0 - beta2) * g * g
    mhat = m_new / (1.0 - beta1 ** step)
    vhat = v_new / (1.0 - beta2 ** step)
    p_new = p - lr * mhat / (np.sqrt(vhat) + eps)
    p[:, act] = p_new[:, act]
    m[:, act] = m_new[:, act]
    v[:, act] = v_new[:, act]
    return p, m, v


# ---------------------------------------------------------------------------
# Gradient-norm scores and freezing (Section 3.2.1, eqs. 4-6)
# ---------------------------------------------------------------------------

def scores(grads):
    """(g_xyz, g_rgb, g_op, g_sc): |dL/dmu|, |dL/df_dc|, |dL/dlogit|, |dL/dlog_s|."""
    g = np.asarray(grads, np.float64)
    return (np.sqrt((g[0:3] ** 2).sum(0)), np.sqrt((g[11:14] ** 2).sum(0)),
            np.abs(g[10]), np.sqrt((g[3:6] ** 2).sum(0)))


FLT_MAX = float(np.finfo(np.float32).max)


def ema_update(ema, g, visible_any, frozen, beta):
    """Exponential moving average of a score, only for active Gaussians seen
    in at least one view; an entry at FLT_MAX (never seen) takes g directly."""
    ema = np.array(ema, np.float64)
    upd = np.asarray(visible_any, bool) & (np.asarray(frozen) == 0)
    first = upd & (ema >= FLT_MAX)
    rest = upd & ~(ema >= FLT_MAX)
    ema[first] = g[first]
    ema[rest] = beta * ema[rest] + (1.0 - beta) * g[rest]
    return ema


def freeze_update(frozen, s_xyz, s_rgb, eps_xyz, eps_rgb, mode, proposal=None):
    """Eq. 4 per parameter group (|grad| < eps, strict), eq. 6 (both groups),
    accumulated into the previous map (mode 0), reset (mode 1) or overwrite
    (mode 2).  Inputs are compared in float32, as the GPU receives them."""
    sx = np.asarray(s_xyz, np.float32)
    sr = np.asarray(s_rgb, np.float32)
    cond = (sx < np.float32(eps_xyz)) & (sr < np.float32(eps_rgb))
    if proposal is not None:
        cond = cond | (np.asarray(proposal) != 0)
    old = np.asarray(frozen) != 0
    if mode == 0:
        new = old | cond
    elif mode == 1:
        new = np.zeros_like(old)
    else:
        new = cond
    return new.astype(np.uint8)


# ---------------------------------------------------------------------------
# The ablation's naive freezing rules (Section 4.3, Table 3 rows "+mingrad"
# and "+random"): freeze the Gaussians with the lowest 25% gradients, or a
# random 25% of them, in place of the thresholds of eqs. 4-6.  The random
# draws come from Philox4x64-10 (Salmon et al., "Parallel random numbers: as
# easy as 1, 2, 3", SC 2011), written here from its published round
# function; the GPU implements the same generator on its own.
# ---------------------------------------------------------------------------

_PHILOX_M = (0xD2E7470EE14C6C93, 0xCA5A826395121157)
_PHILOX_W = (0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)
_U64 = (1 << 64) - 1


def philox4x64_10(counter, key):
    """Philox4x64 with 10 rounds: counter = 4 uint64, key = 2 uint64 ->
    4 uint64.  Each round multiplies words 0 and 2 by the two constants
    (128-bit products), mixes the high halves with words 1 and 3 and the key,
    and the key is bumped by the Weyl constants between rounds."""
    c = [int(x) & _U64 for x in counter]
    k = [int(x) & _U64 for x in key]
    for r in range(10):
        if r:
            k = [(k[0] + _PHILOX_W[0]) & _U64, (k[1] + _PHILOX_W[1]) & _U64]
        p0 = _PHILOX_M[0] * c[0]
        p1 = _PHILOX_M[1] * c[2]
        c = [(p1 >> 64) ^ c[1] ^ k[0], p1 & _U64, (p0 >> 64) ^ c[3] ^ k[1], p0 & _U64]
    return c


def random_threshold(fraction):
    """Integer threshold t with P(u32 < t) = fraction for a uniform u32:
    floor(fraction * 2^32), at most 2^32."""
    import math
    return min(int(math.floor(float(fraction) * 4294967296.0)), 1 << 32)


def freeze_random(n, fraction, seed, draw):
    """"+random": Gaussian i is proposed for freezing iff the top 32 bits of
    the first word of Philox4x64-10(counter = (i, draw, 0, 0), key = (seed,
    0)) are below floor(fraction * 2^32), so each Gaussian is drawn
    independently with probability `fraction` and every freeze update
    (draw) gets fresh draws."""
    t = random_threshold(fraction)
    return np.array([(philox4x64_10((i, draw, 0, 0), (seed, 0))[0] >> 32) < t for i in range(n)], np.uint8)


def freeze_mingrad(score, fraction):
    """"+mingrad": among the Gaussians with a finite average (s < FLT_MAX,
    i.e. seen at least once), the m = floor(fraction * count) with the
    smallest positional gradient-norm average, compared in float32, equal
    values taken in ascending index order."""
    import math
    s = np.asarray(score, np.float32)
    cand = [i for i in range(s.size) if s[i] < np.float32(FLT_MAX)]
    m = int(math.floor(float(fraction) * float(len(cand))))
    chosen = sorted(cand, key=lambda i: (float(s[i]), i))[:m]
    out = np.zeros(s.size, np.uint8)
    out[chosen] = 1
    return out


def apply_freeze(frozen, cond, mode):
    """The freeze map after an update whose condition is `cond`: mode 0 ORs
    it into the map (frozen Gaussians stay frozen), mode 1 resets the map,
    mode 2 replaces it."""
    old = np.asarray(frozen) != 0
    c = np.asarray(cond) != 0
    new = old | c if mode == 0 else (np.zeros_like(old) if mode == 1 else c)
    return new.astype(np.uint8)


def partition_order(frozen):
    """Column order that puts the Gaussians the optimizer still updates
    (Section 3.2.4: frozen ones are skipped) in front: the active columns in
    their order, then the frozen ones in theirs.  Returns (src, n_active)
    with new column i = old column src[i]; a layout choice, so the
    definition is just this ordering."""
    f = np.asarray(frozen) != 0
    active = [j for j in range(f.size) if not f[j]]
    frozen_cols = [j for j in range(f.size) if f[j]]
    return np.array(active + frozen_cols, dtype=np.int64), len(active)


def apply_partition(x, src):
    """Columns of x ([rows, n] or [n]) in the order src."""
    x = np.asarray(x)
    return x[..., src].copy()


# ---------------------------------------------------------------------------
# Host schedule (Section 3.2.1 eq. 5, Section 3.2.2 eq. 7, Section 3.2.3)
# ---------------------------------------------------------------------------

def freeze_threshold(k, K, eps0, k_stop=None, lam1=0.5, lam2=1.5, linear=False):
    """Threshold at iteration k.  The recursion of eq. 5 is read with the
    previous threshold replaced by the initial one and the factor bounded to
    [lam1, lam2] (the text fixes the range [0.5, 1.5] of the initial value):
    eps0 * clamp(lam1 + lam2 * k'/K, lam1, lam2), k' = min(k, k_stop).  The
    ``linear`` reading is eps0 * (lam1 + (lam2 - lam1) * k'/K)."""
    kk = k if k_stop is None else min(k, k_stop)
    if linear:
        f = lam1 + (lam2 - lam1) * kk / K
    else:
        f = min(max(lam1 + lam2 * kk / K, lam1), lam2)
    return eps0 * f


def early_stop(psnrs, eps=0.2):
    """Eq. 7: stop when the last two PSNR gains are both below eps."""
    if len(psnrs) < 3:
        return False
    d1 = psnrs[-1] - psnrs[-2]
    d0 = psnrs[-2] - psnrs[-3]
    return (d1 < eps) and (d0 < eps)


class PlateauLR:
    """Section 3.2.3: a plateau scheduler on the position learning rate.  An
    evaluation improves iff its PSNR exceeds the best so far by more than
    ``eps``; after more than ``patience`` evaluations in a row without
    improvement the scale is multiplied by ``factor``."""

    def __init__(self, factor=0.75, patience=1, eps=1.0):
        self.factor, self.patience, self.eps = factor, patience, eps
        self.scale = 1.0
        self.bad = 0
        self.best = None

    def step(self, psnr_value):
        if self.best is None or psnr_value > self.best + self.eps:
            self.best = psnr_value
            self.bad = 0
        else:
            self.bad += 1
        if self.bad > self.patience:
            self.scale *= self.factor
            self.bad = 0
        return self.scale


# ---------------------------------------------------------------------------
# Freeze-map lifecycle and the end of training (Algorithm 1; Section 3.2.2;
# Section 4.1 "GSta Details").  Written as the sets of iterations at which
# something happens, so that a reader can check them against the text:
#   * no freezing before the warm-up;
#   * the freezing window closes at min(window_end, early-stop iteration);
#     the map is then reset and every Gaussian trains for K_f more
#     iterations (the finetune), after which training ends;
#   * inside the window the map is updated every `every` iterations and
#     accumulates; at every multiple of `reset_every` past the warm-up it is
#     reset and not updated again for `wait` iterations.
# Early stop (eq. 7) is tested on the PSNRs of the evaluations made every
# `eval_every` iterations while the window is open.
# ---------------------------------------------------------------------------

ACT_NONE, ACT_UPDATE, ACT_RESET = 0, 1, 2


def freeze_reset_iters(warmup, reset_every, close):
    """Iterations before which the freeze map is reset: the multiples of
    reset_every past the warm-up and before the window closes, and the
    closing iteration itself (start of the finetune)."""
    resets = [r for r in range(reset_every, close, reset_every) if r > warmup]
    return resets + [close]


def freeze_update_iters(warmup, every, reset_every, wait, close):
    """Iterations before which the freeze map is updated: multiples of
    `every` in [warmup, close) that are not a reset and do not fall within
    `wait` iterations after a reset."""
    resets = freeze_reset_iters(warmup, reset_every, close)
    out = []
    for k in range(0, close, every):
        if k < warmup or k in resets:
            continue
        if any(r <= k < r + wait for r in resets):
            continue
        out.append(k)
    return out


def freeze_action(k, warmup, every, reset_every, wait, window_end, stop_iter=None):
    """What happens to the freeze map before iteration k: ACT_NONE,
    ACT_UPDATE or ACT_RESET."""
    close = window_end if stop_iter is None else min(window_end, stop_iter)
    if k in freeze_reset_iters(warmup, reset_every, close):
        return ACT_RESET
    if k in freeze_update_iters(warmup, every, reset_every, wait, close):
        return ACT_UPDATE
    return ACT_NONE


def training_end(total_iters, window_end, stop_iter, finetune_iters):
    """Number of training iterations.  When the freezing window closes
    (early stop, or the forced stop at window_end) before total_iters, the
    finetune of finetune_iters iterations follows and training ends; the
    loop of Algorithm 1 keeps running while finetune iterations remain, so
    the end may lie past total_iters.  A window that never closes before
    total_iters ends training at total_iters."""
    close = window_end if stop_iter is None else min(window_end, stop_iter)
    if close >= total_iters:
        return total_iters
    return close + finetune_iters


def densify_action(k, start, stop, every, reset_every, stop_iter=None):
    """(densify, opacity_reset) before iteration k (Section 4.1): densify
    and prune every `every` iterations in [start, min(stop, early stop));
    opacity reset every reset_every iterations in [reset_every,
    min(stop, early stop)]."""
    end = stop if stop_iter is None else min(stop, stop_iter)
    dens = k > 0 and start <= k < end and k % every == 0
    reset = reset_every <= k <= end and k % reset_every == 0
    return dens, reset


def simulate_lifecycle(total_iters, warmup, every, reset_every, wait, window_end, finetune_iters,
                       eval_every=None, psnr_at=None, es_eps=0.2, plateau=None):
    """Run the host side of Algorithm 1 for a whole training: per iteration
    the freeze action, evaluations every eval_every iterations while the
    window is open (psnr_at(k) gives the PSNR measured after k iterations),
    eq. 7 early stop and the plateau scale of the position learning rate.
    Returns dict(actions [end], stop_iter, end, psnrs, pos_scale [end] (the
    scale used by iteration k))."""
    psnrs = []
    stop_iter = None
    actions = []
    scales = []
    scale = 1.0
    k = 0
    while k < training_end(total_iters, window_end, stop_iter, finetune_iters):
        actions.append(freeze_action(k, warmup, every, reset_every, wait, window_end, stop_iter))
        scales.append(scale)
        k += 1
        close = window_end if stop_iter is None else min(window_end, stop_iter)
        if eval_every and k % eval_every == 0 and k < close and stop_iter is None:
            psnrs.append(float(psnr_at(k)))
            if plateau is not None:
                scale = plateau.step(psnrs[-1])
            if early_stop(psnrs, es_eps):
                stop_iter = k
    return dict(actions=actions, stop_iter=stop_iter, end=k, psnrs=psnrs, pos_scale=scales)


# ---------------------------------------------------------------------------
# Adaptive densification, pruning and opacity reset (Section 3.1: Gaussians
# are pruned and densified by gradient norm and opacity; Section 4.1: every
# 100 iterations, thresholds eps_den_xyz = 2e-4 and eps_den_rgb = 1e-6 scaled
# like the freezing thresholds, diffuse-colour gradients used on 20 % of the
# densification steps, opacity reset every 3K).  The clone / split / prune
# rules themselves are the 3DGS conventions the paper builds on: clone a
# selected Gaussian whose largest scale is small, otherwise replace it by two
# children drawn from it with scales divided by 1.6; prune opacity < 0.005.
# ---------------------------------------------------------------------------

def densify_stats(acc, grad2d, visible, grads, frozen, width, height):
    """Accumulate one step's densification statistics into acc [4, n]:
    row 0 += |(dL/du * W/2, dL/dv * H/2)| (the gradient with respect to the
    normalised device coordinates of the projected mean) and row 1 += 1 for
    every view in which the Gaussian is visible; row 2 += |dL/df_dc| and
    row 3 += 1 once per step if it is visible in any view.  Frozen Gaussians
    are left unchanged.  grad2d [V, 9, n] and visible [V, n] are the
    per-view outputs of render_backward, grads [R, n] its parameter
    gradient."""
    acc = np.array(acc, np.float64)
    g2 = np.asarray(grad2d, np.float64)
    vis = np.asarray(visible) != 0
    act = np.ones(acc.shape[1], bool) if frozen is None else (np.asarray(frozen) == 0)
    for v in range(g2.shape[0]):
        m = vis[v] & act
        nrm = np.sqrt((g2[v, 0] * (0.5 * width)) ** 2 + (g2[v, 1] * (0.5 * height)) ** 2)
        acc[0, m] += nrm[m]
        acc[1, m] += 1.0
    anyv = vis.any(0) & act
    gdc = np.sqrt((np.asarray(grads, np.float64)[11:14] ** 2).sum(0))
    acc[2, anyv] += gdc[anyv]
    acc[3, anyv] += 1.0
    return acc


def _quat_rot(q):
    """Rotation matrices [n, 3, 3] of quaternions q [4, n] = (w, x, y, z),
    normalised first."""
    q = np.asarray(q, np.float64)
    w, x, y, z = q / np.sqrt((q ** 2).sum(0))
    return np.stack([
        np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], 1)


def densify_decisions(stats, params, frozen, grad_threshold, rgb_threshold, use_rgb, split_log_scale,
                      prune_logit):
    """Per-Gaussian (clone, split, live) decisions, taken in float32 as the
    GPU takes them: mean screen gradient = row0 / row1 (0 where row1 = 0),
    mean colour gradient = row2 / row3; selected iff the mean screen gradient
    >= grad_threshold, or (use_rgb) the mean colour gradient >= rgb_threshold,
    and not frozen; split iff selected and max log-scale > split_log_scale,
    clone iff selected otherwise; live iff logit >= prune_logit."""
    st = np.asarray(stats, np.float32)
    P = np.asarray(params, np.float32)
    with np.errstate(divide="ignore", invalid="ignore"):
        mxy = np.where(st[1] > 0, st[0] / np.where(st[1] > 0, st[1], np.float32(1)), np.float32(0))
        mrgb = np.where(st[3] > 0, st[2] / np.where(st[3] > 0, st[3], np.float32(1)), np.float32(0))
    sel = mxy >= np.float32(grad_threshold)
    if use_rgb:
        sel |= mrgb >= np.float32(rgb_threshold)
    if frozen is not None:
        sel &= np.asarray(frozen) == 0
    big = P[3:6].max(0) > np.float32(split_log_scale)
    live = P[10] >= np.float32(prune_logit)
    return sel & ~big, sel & big, live


def densify_noise(n, seed, draw):
    """Standard normals for the split children (noise [6][n], rows 3c..3c+2
    for child c of column i), from Philox4x64-10 with counter (i, draw, c, 0)
    and key (seed, 1): its four words become uniforms u = (floor(w / 2^11) +
    0.5) / 2^53 in (0, 1), and the Box-Muller transform gives r = sqrt(-2 ln
    u0), (r cos 2 pi u1, r sin 2 pi u1) and sqrt(-2 ln u2) cos 2 pi u3."""
    out = np.zeros((6, n))
    for i in range(n):
        for c in range(2):
            w = philox4x64_10((i, draw, c, 0), (seed, 1))
            u = [((x >> 11) + 0.5) / 2.0 ** 53 for x in w]
            r0 = np.sqrt(-2.0 * np.log(u[0]))
            r1 = np.sqrt(-2.0 * np.log(u[2]))
            out[3 * c:3 * c + 3, i] = [r0 * np.cos(2 * np.pi * u[1]), r0 * np.sin(2 * np.pi * u[1]),
                                       r1 * np.cos(2 * np.pi * u[3])]
    return out


def densify_prune(params, m, v, ema, frozen, stats, noise, grad_threshold, rgb_threshold, use_rgb,
                  split_log_scale, prune_logit, child_log_scale_shift):
    """One densify-and-prune step.  Output columns, in this order: the
    surviving Gaussians (live and not split) in their order; a copy of every
    live clone-selected Gaussian; the first child of every live split-selected
    Gaussian, then the second children.  Child c of Gaussian i sits at
    mu_i + R(q_i) (exp(log_s_i) * noise[3c:3c+3, i]) with log-scales
    log_s_i - child_log_scale_shift and every other parameter copied; the
    split parent is removed.  New columns get zero Adam moments, EMAs at
    FLT_MAX (never seen) and are not frozen; survivors keep theirs.  A
    Gaussian that is split or not live leaves the set.
    Returns (params, m, v, ema, frozen, counts = (n_out, kept, clones, splits))."""
    P = np.asarray(params, np.float64)
    n = P.shape[1]
    fz = np.zeros(n, np.uint8) if frozen is None else np.asarray(frozen, np.uint8)
    E = np.full((4, n), FLT_MAX) if ema is None else np.asarray(ema, np.float64)
    clone, split, live = densify_decisions(stats, params, frozen, grad_threshold, rgb_threshold, use_rgb,
                                           split_log_scale, prune_logit)
    keep = live & ~split
    cl = np.flatnonzero(clone & live)
    sp = np.flatnonzero(split & live)
    kp = np.flatnonzero(keep)
    nz = np.asarray(noise, np.float64)
    Rm = _quat_rot(P[6:10, sp])
    s = np.exp(P[3:6, sp])
    children = []
    for c in range(2):
        ch = P[:, sp].copy()
        off = np.einsum("nij,jn->in", Rm, s * nz[3 * c:3 * c + 3, sp])
        ch[0:3] = P[0:3, sp] + off
        ch[3:6] = P[3:6, sp] - child_log_scale_shift
        children.append(ch)
    newP = np.concatenate([P[:, kp], P[:, cl]] + children, 1)
    n_new = len(cl) + 2 * len(sp)
    zeros = np.zeros((P.shape[0], n_new))
    newM = np.concatenate([np.asarray(m, np.float64)[:, kp], zeros], 1)
    newV = np.concatenate([np.asarray(v, np.float64)[:, kp], zeros], 1)
    newE = np.concatenate([E[:, kp], np.full((4, n_new), FLT_MAX)], 1)
    newF = np.concatenate([fz[kp], np.zeros(n_new, np.uint8)])
    counts = (newP.shape[1], len(kp), len(cl), len(sp))
    return newP, newM, newV, newE, newF, counts


def opacity_reset(params, m, v, frozen, logit_cap):
    """Opacity reset: every active Gaussian's opacity becomes min(o, o_cap),
    i.e. logit <- min(logit, logit_cap), and the Adam moments of the opacity
    row are zeroed.  Frozen Gaussians are left untouched."""
    P = np.array(params, np.float64)
    M = np.array(m, np.float64)
    V = np.array(v, np.float64)
    act = np.ones(P.shape[1], bool) if frozen is None else (np.asarray(frozen) == 0)
    P[10, act] = np.minimum(P[10, act], np.float32(logit_cap))
    M[10, act] = 0.0
    V[10, act] = 0.0
    return P, M, V


# ---------------------------------------------------------------------------
# Learned freeze proposer (a project extension; the paper has no such
# model, so its label and veto semantics are parity unpinned by the paper).
# An MLP 32 -> 64 -> 64 -> 1 (ReLU, ReLU, logit) reads the last 8 logged
# gradient-norm averages (xyz, rgb, opacity, scale) of a Gaussian as
# standardised log10 features and proposes freezing it; the freeze rule
# vetoes proposals whose averages are far above its thresholds.  The GPU
# runs the two hidden layers on bf16 matrix cores with float32
# accumulation: inputs, weights and the first hidden layer are rounded to
# bf16 there, so the oracle rounds the same quantities (round to nearest,
# ties to even) and computes everything else in float64.
# ---------------------------------------------------------------------------

MLP_IN, MLP_H = 32, 64
# flat float32 parameter layout: W1 [64][32], b1 [64], W2 [64][64], b2 [64], w3 [64], b3
MLP_OFF = {"W1": 0, "b1": 2048, "W2": 2112, "b2": 6208, "w3": 6272, "b3": 6336}
MLP_COUNT = 6337


def bf16_round(x):
    """Round float32 values to bfloat16 (nearest, ties to even); returned as
    float64 holding the bf16 value.  Inputs are first rounded to float32."""
    f = np.ascontiguousarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def mlp_unpack(wf):
    w = np.asarray(wf, np.float64)
    o = MLP_OFF
    return (w[o["W1"]:o["b1"]].reshape(64, 32), w[o["b1"]:o["W2"]], w[o["W2"]:o["b2"]].reshape(64, 64),
            w[o["b2"]:o["w3"]], w[o["w3"]:o["b3"]], w[o["b3"]])


def traj_features(ring, head, mean, std):
    """Features of every Gaussian: x[i][4j + q] = bf16((log10(r + 1e-12) - mean) / std)
    with r = ring[(head - j) mod 8][q][i] (j = 0 is the newest entry)."""
    R = np.asarray(ring, np.float64)
    n = R.shape[2]
    x = np.zeros((n, 32))
    for j in range(8):
        for q in range(4):
            f = 4 * j + q
            x[:, f] = (np.log10(R[(head - j) % 8, q] + 1e-12) - mean[f]) / std[f]
    return bf16_round(x)


def mlp_forward(x, wf):
    """Logits of the MLP for bf16 features x [n][32]; also returns the bf16
    first hidden layer and the float64 second one."""
    W1, b1, W2, b2, w3, b3 = mlp_unpack(wf)
    W1b, W2b = bf16_round(W1), bf16_round(W2)
    a1 = np.asarray(x, np.float64) @ W1b.T + b1
    h1 = bf16_round(np.maximum(a1, 0.0))
    a2 = h1 @ W2b.T + b2
    h2 = np.maximum(a2, 0.0)
    z = h2 @ w3 + b3
    return z, h1, h2


def mlp_backward(x, wf, dz):
    """Gradient of sum_i dz_i * z_i with respect to the flat parameters,
    through the same rounded activations (the bf16 roundings are treated
    as identity in the derivative, weights and hidden units alike)."""
    W1, b1, W2, b2, w3, b3 = mlp_unpack(wf)
    W2b = bf16_round(W2)
    z, h1, h2 = mlp_forward(x, wf)
    dz = np.asarray(dz, np.float64)
    g = np.zeros(MLP_COUNT)
    o = MLP_OFF
    g[o["b3"]] = dz.sum()
    g[o["w3"]:o["b3"]] = h2.T @ dz
    d2 = np.outer(dz, w3) * (h2 > 0)
    g[o["b2"]:o["w3"]] = d2.sum(0)
    g[o["W2"]:o["b2"]] = (d2.T @ h1).reshape(-1)
    d1 = (d2 @ W2b) * (h1 > 0)
    g[o["b1"]:o["W2"]] = d1.sum(0)
    g[o["W1"]:o["b1"]] = (d1.T @ np.asarray(x, np.float64)).reshape(-1)
    return g


def bce(z, y):
    """Mean binary cross-entropy of logits z against labels y and its
    derivative dL/dz = (sigmoid(z) - y) / n."""
    z = np.asarray(z, np.float64)
    y = np.asarray(y, np.float64)
    n = z.size
    loss = np.mean(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z))))
    return loss, (1.0 / (1.0 + np.exp(-z)) - y) / n


def propose(z, s_xyz, s_rgb, logit_threshold, veto_xyz, veto_rgb):
    """Accepted proposals: logit above the threshold (sigmoid(z) > tau) and
    not vetoed by the rule (both averages below c_v times its thresholds);
    float32 comparisons."""
    z32 = np.asarray(z, np.float32)
    return ((z32 > np.float32(logit_threshold)) & (np.asarray(s_xyz, np.float32) < np.float32(veto_xyz))
            & (np.asarray(s_rgb, np.float32) < np.float32(veto_rgb))).astype(np.uint8)


def proposer_labels(cond_next, cond_after):
    """Label of a Gaussian at a freeze update: the rule freezes it at one of
    the next two updates."""
    return ((np.asarray(cond_next) != 0) | (np.asarray(cond_after) != 0)).astype(np.uint8)
