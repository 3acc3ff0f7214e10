"""Helpers for the GPU parity tests: run the HIP path through the C ABI and
bring results back as numpy arrays, plus the comparison rules (tolerances
and decision margins) used against the oracle."""
import numpy as np

# Decision margins: a pixel whose oracle walk made a membership or
# termination decision within this relative distance of its threshold, or a
# Gaussian whose tile rectangle edge lies within RECT_PX of a tile boundary,
# may legitimately differ between float32 and float64.
MARGIN_VALUE = 1e-5
MARGIN_RECT_PX = 1e-3
MARGIN_NEAR = 1e-5
IMAGE_ATOL = 1e-4
GRAD_REL = 1e-3

GROUPS = {"mean": slice(0, 3), "log_scale": slice(3, 6), "quat": slice(6, 10), "logit": slice(10, 11),
          "sh_dc": slice(11, 14), "sh_rest": slice(14, None)}


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


class GpuScene:
    """One parameter block + cameras rendered through libgsta."""

    def __init__(self, params, degree, cams, bg=(0.0, 0.0, 0.0), capacity=1 << 22, ctx=None, opacity_act=0,
                 sh_mask=None, sh_mask_threshold=0.0):
        import torch
        import paper_2504_06716_amd as G
        self.torch = torch
        self.degree = degree
        self.cams = cams
        self.V = len(cams)
        self.H, self.W = cams[0].height, cams[0].width
        self.n = params.shape[1]
        self.bg = bg
        self.ctx = ctx or G.Context(max(self.n, 1), self.V, self.H, self.W, capacity, n_slots=1)
        self.P = dev(params.astype(np.float32))
        self.carr = G.camera_array(cams)
        self.R = params.shape[0]
        self.opacity_act = opacity_act
        # SH-band mask logits [3, n] (same row stride as the contiguous block)
        self.M = None if sh_mask is None else dev(np.ascontiguousarray(sh_mask, np.float32))
        self.thr = sh_mask_threshold
        self.mask_grad = None

    def forward(self):
        t = self.torch
        img = t.empty((self.V, 3, self.H, self.W), dtype=t.float32, device="cuda")
        self.ctx.render_forward(self.P, self.degree, self.carr, self.bg, img, 0, opacity_act=self.opacity_act,
                                sh_mask=self.M, sh_mask_threshold=self.thr)
        t.cuda.synchronize()
        self.image = img
        return img.cpu().numpy()

    def state(self, field, dtype, shape):
        t = self.torch
        out = t.empty(shape, dtype=dtype, device="cuda")
        self.ctx.get_state(0, field, out)
        t.cuda.synchronize()
        return out.cpu().numpy()

    def backward(self, dL, frozen=None, ema=None, beta=0.9, sentinel=None):
        t = self.torch
        grad = t.full((self.R, self.n), float("nan") if sentinel is None else sentinel,
                      dtype=t.float32, device="cuda")
        g2 = t.zeros((self.V, 9, self.n), dtype=t.float32, device="cuda")
        fz = None if frozen is None else dev(frozen.astype(np.uint8))
        em = None if ema is None else dev(ema.astype(np.float32))
        mg = None if self.M is None else t.full((3, self.n), float("nan"), dtype=t.float32, device="cuda")
        self.ctx.render_backward(self.P, self.degree, self.carr, self.bg, 0, dev(dL.astype(np.float32)),
                                 fz, grad, g2, em, beta, opacity_act=self.opacity_act, sh_mask=self.M,
                                 sh_mask_threshold=self.thr, sh_mask_grad=mg)
        t.cuda.synchronize()
        self.mask_grad = None if mg is None else mg.cpu().numpy()
        return grad.cpu().numpy(), g2.cpu().numpy(), (None if em is None else em.cpu().numpy())


def compare_grads(g, ref, exclude_cols=None, rel=GRAD_REL):
    """Per parameter group: ||d||/||ref|| <= rel and elementwise
    |d| <= rel*|ref| + rel*max|ref| (excluded columns skip the elementwise test)."""
    report = {}
    for name, sl in GROUPS.items():
        a, b = g[sl], ref[sl]
        if b.size == 0:
            continue
        nb = np.linalg.norm(b)
        d = a - b
        report[name] = (np.linalg.norm(d) / max(nb, 1e-30))
        assert report[name] <= rel, (name, report[name])
        tol = rel * np.abs(b) + rel * np.abs(b).max()
        bad = np.abs(d) > tol
        if exclude_cols is not None:
            bad[:, exclude_cols] = False
        assert not bad.any(), (name, np.argwhere(bad)[:5], a[bad][:5], b[bad][:5])
    return report
