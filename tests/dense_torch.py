"""Dense float64 torch forward of the renderer, used only to pin the oracle's
hand-written backward through torch autograd (an independent library route).

Every pixel composites every Gaussian in (float32 depth, gid) order; the
membership tests (3-sigma ellipse, alpha >= 1/255, transmittance floor) are
masks, so autograd differentiates exactly the same function with every
discrete decision held at its forward value.
"""
import math

import numpy as np
import torch


def _sh(deg, d):
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    pi = math.pi
    out = [torch.full_like(x, 0.5 / math.sqrt(pi))]
    if deg >= 1:
        c = math.sqrt(3 / (4 * pi))
        out += [c * y, c * z, c * x]
    if deg >= 2:
        a, b, c = math.sqrt(15 / (4 * pi)), math.sqrt(5 / (16 * pi)), math.sqrt(15 / (16 * pi))
        out += [a * x * y, a * y * z, b * (2 * z * z - x * x - y * y), a * x * z, c * (x * x - y * y)]
    if deg >= 3:
        a = math.sqrt(35 / (32 * pi))
        b = math.sqrt(105 / (4 * pi))
        c = math.sqrt(21 / (32 * pi))
        d7 = math.sqrt(7 / (16 * pi))
        e = math.sqrt(105 / (16 * pi))
        out += [a * y * (3 * x * x - y * y), b * x * y * z, c * y * (4 * z * z - x * x - y * y),
                d7 * z * (2 * z * z - 3 * x * x - 3 * y * y), c * x * (4 * z * z - x * x - y * y),
                e * z * (x * x - y * y), a * x * (x * x - 3 * y * y)]
    return torch.stack(out, 1)


def render_dense(params, deg, cam, bg=(0.0, 0.0, 0.0)):
    """params: float64 tensor [R, N] (may require grad).  Returns image [3, H, W]."""
    f64 = torch.float64
    R = torch.tensor(np.asarray(cam.R), dtype=f64)
    t = torch.tensor(np.asarray(cam.t), dtype=f64)
    cpos = torch.tensor(np.asarray(cam.campos), dtype=f64)
    fx, fy, cx, cy = cam.fx, cam.fy, cam.cx, cam.cy
    H, W = cam.height, cam.width
    N = params.shape[1]
    mu = params[0:3].T
    xc = mu @ R.T + t
    z = xc[:, 2]
    s = torch.exp(params[3:6].T)
    q = params[6:10].T
    qn = q / q.norm(dim=1, keepdim=True)
    w, x, y, zq = qn.unbind(1)
    Rq = torch.stack([
        torch.stack([1 - 2 * (y * y + zq * zq), 2 * (x * y - w * zq), 2 * (x * zq + w * y)], 1),
        torch.stack([2 * (x * y + w * zq), 1 - 2 * (x * x + zq * zq), 2 * (y * zq - w * x)], 1),
        torch.stack([2 * (x * zq - w * y), 2 * (y * zq + w * x), 1 - 2 * (x * x + y * y)], 1)], 1)
    M = Rq * s[:, None, :]
    Sigma = M @ M.transpose(1, 2)
    limx = 1.3 * 0.5 * W / fx
    limy = 1.3 * 0.5 * H / fy
    rx, ry = xc[:, 0] / z, xc[:, 1] / z
    rxc, ryc = rx.clamp(-limx, limx), ry.clamp(-limy, limy)
    zero = torch.zeros_like(z)
    J = torch.stack([torch.stack([fx / z, zero, -fx * rxc / z], 1),
                     torch.stack([zero, fy / z, -fy * ryc / z], 1)], 1)
    T = J @ R
    cov = T @ Sigma @ T.transpose(1, 2)
    a = cov[:, 0, 0] + 0.3
    b = cov[:, 0, 1]
    c = cov[:, 1, 1] + 0.3
    det = a * c - b * b
    ca, cb, cc = c / det, -b / det, a / det
    u = fx * rx + cx
    v = fy * ry + cy
    dvec = mu - cpos
    dn = dvec / dvec.norm(dim=1, keepdim=True)
    B = _sh(deg, dn)
    K = B.shape[1]
    f = params[11:].T.reshape(N, K, 3)
    raw = (f * B[:, :, None]).sum(1) + 0.5
    rgb = raw.clamp(min=0.0)
    o = torch.sigmoid(params[10])

    zd = z.detach().numpy()
    vis = (zd > cam.near) & (det.detach().numpy() > 0)
    ids = [i for i in range(N) if vis[i]]
    ids.sort(key=lambda i: (np.float32(zd[i]), i))
    idx = torch.tensor(ids, dtype=torch.long)
    py, px = torch.meshgrid(torch.arange(H, dtype=f64), torch.arange(W, dtype=f64), indexing="ij")
    px, py = px.reshape(-1, 1), py.reshape(-1, 1)
    dx = u[idx][None, :] - px
    dy = v[idx][None, :] - py
    power = -0.5 * (ca[idx] * dx * dx + cc[idx] * dy * dy) - cb[idx] * dx * dy
    oG = o[idx] * torch.exp(power)
    alpha = torch.minimum(oG, torch.tensor(0.99, dtype=f64))
    member = ((power >= -4.5) & (alpha >= 1.0 / 255.0)).to(f64).detach()
    am = alpha * member
    Tincl = torch.cumprod(1.0 - am, dim=1)
    keep = (Tincl >= 1e-4).to(f64).detach()
    Texcl = torch.cat([torch.ones_like(Tincl[:, :1]), Tincl[:, :-1]], 1)
    wgt = am * Texcl * keep
    C = wgt @ rgb[idx]
    Tfin = torch.prod(1.0 - am * keep, dim=1)
    img = C + Tfin[:, None] * torch.tensor(bg, dtype=f64)[None, :]
    return img.T.reshape(3, H, W)
