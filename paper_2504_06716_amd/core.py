"""Tensor-level wrappers of the libgsta entry points.

PyTorch provides device memory and the stream; every computation runs in
the HIP kernels behind the C ABI.  Tensors must be CUDA(HIP) float32 and
contiguous in the layouts documented in include/gsta.h.
"""
from __future__ import annotations

import contextlib
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import AdamSched, Camera, Limits, Params, check

MAX_VIEWS = 8


def n_rows(degree: int) -> int:
    return 11 + 3 * (degree + 1) ** 2


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _ptr(t) -> int | None:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    return t.data_ptr()


def _arr(t, shape, dtype, name):
    """Pointer of a contiguous device tensor of the given shape and dtype
    (None passes through)."""
    if t is None:
        return None
    if tuple(t.shape) != tuple(shape) or t.dtype != dtype:
        raise ValueError(f"{name}: expected {tuple(shape)} {dtype}, got {tuple(t.shape)} {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return _ptr(t)


def params_struct(block: torch.Tensor, degree: int, opacity_act: int = 0, sh_mask: torch.Tensor | None = None,
                  sh_mask_threshold: float = 0.0) -> Params:
    """[R, n] float32 device tensor (row stride = block.stride(0)); opacity_act
    1 selects the finetune stage's absolute opacity activation.  sh_mask: the
    [3, n] float32 SH-band mask logits (or, for a gradient block, where their
    gradient goes), with the block's row stride; sh_mask_threshold in (0, 1)."""
    if block.dtype != torch.float32 or block.dim() != 2:
        raise ValueError("parameter blocks are [R, n] float32")
    if block.shape[0] != n_rows(degree):
        raise ValueError(f"expected {n_rows(degree)} rows for SH degree {degree}, got {block.shape[0]}")
    n = block.shape[1]
    if n == 0:
        return Params(n=0, ld=1, sh_degree=degree, opacity_act=opacity_act, block=block.data_ptr() or None)
    if block.stride(1) != 1 or block.stride(0) < n:
        raise ValueError("parameter blocks need unit column stride and row stride >= n")
    ps = Params(n=n, ld=block.stride(0), sh_degree=degree, opacity_act=opacity_act, block=block.data_ptr())
    if sh_mask is not None:
        if (sh_mask.dtype != torch.float32 or sh_mask.dim() != 2 or tuple(sh_mask.shape) != (3, n)
                or sh_mask.stride(1) != 1 or sh_mask.stride(0) != block.stride(0) or sh_mask.device != block.device):
            raise ValueError("SH-band masks are [3, n] float32 with the parameter block's row stride")
        ps.sh_mask = sh_mask.data_ptr()
        ps.sh_mask_threshold = float(sh_mask_threshold)
    return ps


def camera_struct(cam) -> Camera:
    """From a synthetic.Camera-like object (width, height, fx, fy, cx, cy, R, t, campos, near)."""
    c = Camera()
    c.width, c.height = int(cam.width), int(cam.height)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    w2c = np.concatenate([np.asarray(cam.R, np.float64), np.asarray(cam.t, np.float64)[:, None]], 1)
    c.world_to_cam[:] = [float(x) for x in w2c.reshape(-1).astype(np.float32)]
    c.cam_pos[:] = [float(x) for x in np.asarray(cam.campos, np.float32)]
    c.near_z = float(cam.near)
    return c


def camera_array(cams) -> ctypes.Array:
    arr = (Camera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = camera_struct(c)
    return arr


def _f3(bg):
    return (ctypes.c_float * 3)(*[float(x) for x in bg])


class Graph:
    """A captured sequence of library calls (gsta_graph), replayed with launch()."""

    def __init__(self, L, handle):
        self.L, self.h = L, handle

    def launch(self, stream=None):
        st = self.L.gsta_graph_launch(self.h, _stream(stream))
        if st != _lib.GSTA_OK:
            raise _lib.GstaError(st, "gsta_graph_launch failed")

    def close(self):
        if getattr(self, "h", None):
            self.L.gsta_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context:
    """Owns a libgsta context (all scratch is allocated here, once)."""

    def __init__(self, max_gaussians, max_views=1, max_height=64, max_width=64,
                 instance_capacity=1 << 20, n_slots=1):
        self.L = _lib.load()
        self.segment = 64                     # GSTA_OPT_BWD_SEGMENT (the library default)
        self.limits = Limits(int(max_gaussians), int(max_views), int(max_height), int(max_width),
                             int(instance_capacity), 16, 16, int(n_slots))
        h = ctypes.c_void_p()
        st = self.L.gsta_create(ctypes.byref(self.limits), ctypes.byref(h))
        self.h = h
        if st != _lib.GSTA_OK:
            msg = self.L.gsta_last_error(h) if h else b"create failed"
            if h:
                self.L.gsta_destroy(h)
            self.h = None
            raise _lib.GstaError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "h", None):
            self.L.gsta_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, **kw):
        lim = Limits(*[kw.get(f, getattr(self.limits, f)) for f, _ in Limits._fields_])
        check(self.h, self.L.gsta_reserve(self.h, ctypes.byref(lim)))
        self.limits = lim

    def check(self, stream=None):
        """Synchronise; returns (status, max instances needed since the last check)."""
        mi = ctypes.c_int64(0)
        st = self.L.gsta_check(self.h, _stream(stream), ctypes.byref(mi))
        return st, mi.value

    def get_state(self, slot, field, out: torch.Tensor, stream=None):
        check(self.h, self.L.gsta_get_state(self.h, slot, field, out.data_ptr(),
                                             out.numel() * out.element_size(), _stream(stream)))
        return out

    def set_option(self, option: int, value: int):
        check(self.h, self.L.gsta_set_option(self.h, int(option), int(value)))
        if option == _lib.OPT_BWD_SEGMENT:
            self.segment = int(value)

    @contextlib.contextmanager
    def forward_only(self):
        """Renders inside this block are not followed by a backward: they
        write no compositing checkpoints (segment option 0), so they cannot
        use up the checkpoint pool; the option is restored afterwards."""
        saved = self.segment
        self.set_option(_lib.OPT_BWD_SEGMENT, 0)
        try:
            yield self
        finally:
            self.set_option(_lib.OPT_BWD_SEGMENT, saved)

    def capture(self, fn, stream=None) -> Graph:
        """Capture the library calls fn() issues on `stream` (a created
        stream, not the null stream; default: the current stream) into a
        graph.  fn must issue only library calls (no torch work)."""
        s = _stream(stream)
        check(self.h, self.L.gsta_graph_begin(self.h, s))
        try:
            fn()
        finally:
            out = ctypes.c_void_p()
            st = self.L.gsta_graph_end(self.h, s, ctypes.byref(out))
        check(self.h, st)
        return Graph(self.L, out)

    def autotune(self, params, degree, cams, bg, image, dL_dimage, grad, repeats=3, stream=None, frozen=None):
        """Time the result-neutral launch options on this workload (with the
        freeze map `frozen`, if given) and keep the fastest (gsta_autotune);
        returns the gsta_tuning fields."""
        ps, gs = params_struct(params, degree), params_struct(grad, degree)
        ca = cams if isinstance(cams, ctypes.Array) else camera_array(cams)
        shape = (len(ca), 3, ca[0].height, ca[0].width)
        t = _lib.Tuning()
        check(self.h, self.L.gsta_autotune(self.h, ctypes.byref(ps), ca, len(ca), _f3(bg),
                                            _arr(image, shape, torch.float32, "image"),
                                            _arr(dL_dimage, shape, torch.float32, "dL_dimage"), ctypes.byref(gs),
                                            _arr(frozen, (ps.n,), torch.uint8, "frozen"),
                                            int(repeats), ctypes.byref(t), _stream(stream)))
        self.segment = int(t.bwd_segment)
        return {f: getattr(t, f) for f, _ in _lib.Tuning._fields_}

    def set_waves(self, fwd: int | None = None, bwd: int | None = None):
        if fwd is not None:
            self.set_option(_lib.OPT_FWD_WAVES, fwd)
        if bwd is not None:
            self.set_option(_lib.OPT_BWD_WAVES, bwd)

    def set_profiling(self, phases=None, counters=False):
        """Enable event timing for the named phases (all if None; [] disables);
        `counters` also runs the compositing kernels' counting variants."""
        if phases is None:
            mask = (1 << len(_lib.PHASES)) - 1
        else:
            mask = 0
            for p in phases:
                mask |= 1 << _lib.PHASES.index(p)
        if counters:
            mask |= _lib.PROFILE_COUNTERS
        check(self.h, self.L.gsta_set_profiling(self.h, mask))

    def read_profile(self):
        """Per-phase {name: (total ms, launches)} and counters (fwd pairs, bwd pairs,
        fwd wave iterations, bwd wave iterations, bwd splat reductions, bwd pairs
        with gradient work) since the last read."""
        ms = (ctypes.c_double * len(_lib.PHASES))()
        ln = (ctypes.c_int64 * len(_lib.PHASES))()
        pr = (ctypes.c_int64 * 6)()
        check(self.h, self.L.gsta_read_profile(self.h, ms, ln, pr))
        return {name: (ms[i], ln[i]) for i, name in enumerate(_lib.PHASES)}, tuple(pr)

    # ---- hot path --------------------------------------------------------
    def render_forward(self, params, degree, cams, bg, image, slot=0, stream=None, opacity_act=0, sh_mask=None,
                       sh_mask_threshold=0.0):
        ps = params_struct(params, degree, opacity_act, sh_mask, sh_mask_threshold)
        ca = cams if isinstance(cams, ctypes.Array) else camera_array(cams)
        shape = (len(ca), 3, ca[0].height, ca[0].width)
        check(self.h, self.L.gsta_render_forward(self.h, ctypes.byref(ps), ca, len(ca), _f3(bg),
                                                  _arr(image, shape, torch.float32, "image"), slot,
                                                  _stream(stream)))

    def render_forward_l1(self, params, degree, cams, bg, target, image, dL_dimage, sums, slot=0, stream=None,
                          opacity_act=0, sh_mask=None, sh_mask_threshold=0.0):
        """render_forward with the L1 loss against `target` fused into the
        compositing: dL_dimage and sums as l1_loss gives them."""
        ps = params_struct(params, degree, opacity_act, sh_mask, sh_mask_threshold)
        ca = cams if isinstance(cams, ctypes.Array) else camera_array(cams)
        shape = (len(ca), 3, ca[0].height, ca[0].width)
        check(self.h, self.L.gsta_render_forward_l1(
            self.h, ctypes.byref(ps), ca, len(ca), _f3(bg), _arr(target, shape, torch.float32, "target"),
            _arr(image, shape, torch.float32, "image"), _arr(dL_dimage, shape, torch.float32, "dL_dimage"),
            _arr(sums, (2,), torch.float64, "sums"), slot, _stream(stream)))

    def render_backward(self, params, degree, cams, bg, slot, dL_dimage, frozen, grad,
                        grad2d=None, ema=None, ema_beta=0.9, dstats=None, stream=None, opacity_act=0,
                        sh_mask=None, sh_mask_threshold=0.0, sh_mask_grad=None):
        """sh_mask (the forward's band-mask logits) also writes dL/dlogit into
        sh_mask_grad ([3, n], the gradient block's row stride) when given."""
        ps = params_struct(params, degree, opacity_act, sh_mask, sh_mask_threshold)
        gs = params_struct(grad, degree, 0, sh_mask_grad)
        ca = cams if isinstance(cams, ctypes.Array) else camera_array(cams)
        V, n = len(ca), ps.n
        check(self.h, self.L.gsta_render_backward(
            self.h, ctypes.byref(ps), ca, V, _f3(bg), slot,
            _arr(dL_dimage, (V, 3, ca[0].height, ca[0].width), torch.float32, "dL_dimage"),
            _arr(frozen, (n,), torch.uint8, "frozen"), ctypes.byref(gs),
            _arr(grad2d, (V, 9, n), torch.float32, "grad2d"), _arr(ema, (4, n), torch.float32, "ema"),
            float(ema_beta), _arr(dstats, (4, n), torch.float32, "dstats"), _stream(stream)))

    def adam_rows(self, p, g, m, v, lr_rows, beta1, beta2, eps, step, frozen=None, stream=None):
        """Masked Adam over a [rows, n] float32 block (p, g, m, v alike), e.g.
        the SH-band mask logits."""
        rows, n = p.shape
        for x, nm in ((g, "grad"), (m, "m"), (v, "v")):
            if tuple(x.shape) != (rows, n) or x.stride() != p.stride() or x.dtype != torch.float32:
                raise ValueError(f"{nm} must match p in shape, strides and dtype")
        if p.stride(1) != 1:
            raise ValueError("p needs unit column stride")
        lr = (ctypes.c_float * rows)(*[float(x) for x in lr_rows])
        check(self.h, self.L.gsta_adam_rows(self.h, p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), n,
                                            p.stride(0), rows, lr, float(beta1), float(beta2), float(eps),
                                            int(step), _arr(frozen, (n,), torch.uint8, "frozen"),
                                            _stream(stream)))

    def sh_mask_reg(self, logits, threshold, lam, out, frozen=None, grad=None, stream=None):
        """Sparsity term of the SH-band masks: out (float64 [4]) <- [lam *
        mean sigmoid, open gates of bands 1..3]; grad += its gradient."""
        rows, n = logits.shape
        if rows != 3 or logits.dtype != torch.float32 or logits.stride(1) != 1:
            raise ValueError("logits are [3, n] float32 with unit column stride")
        if grad is not None and (grad.shape != logits.shape or grad.stride() != logits.stride()):
            raise ValueError("grad must match logits in shape and strides")
        check(self.h, self.L.gsta_sh_mask_reg(self.h, logits.data_ptr(), n, logits.stride(0), float(threshold),
                                              float(lam), _arr(frozen, (n,), torch.uint8, "frozen"),
                                              None if grad is None else grad.data_ptr(),
                                              _arr(out, (4,), torch.float64, "out"), _stream(stream)))

    def adam_masked(self, p, g, m, v, degree, lr_rows, beta1, beta2, eps, step, frozen=None, stream=None):
        R = n_rows(degree)
        lr = (ctypes.c_float * R)(*[float(x) for x in lr_rows])
        sp, sg, sm, sv = (params_struct(x, degree) for x in (p, g, m, v))
        check(self.h, self.L.gsta_adam_masked(self.h, ctypes.byref(sp), ctypes.byref(sg), ctypes.byref(sm),
                                               ctypes.byref(sv), lr, float(beta1), float(beta2), float(eps),
                                               int(step), _arr(frozen, (sp.n,), torch.uint8, "frozen"),
                                               _stream(stream)))

    def adam_masked_sched(self, p, g, m, v, degree, sched, frozen=None, stream=None):
        """Adam with scalars from a device gsta_adam_sched (uint8 tensor of its size)."""
        sp, sg, sm, sv = (params_struct(x, degree) for x in (p, g, m, v))
        check(self.h, self.L.gsta_adam_masked_sched(self.h, ctypes.byref(sp), ctypes.byref(sg), ctypes.byref(sm),
                                                     ctypes.byref(sv), _ptr(sched),
                                                     _arr(frozen, (sp.n,), torch.uint8, "frozen"),
                                                     _stream(stream)))

    def update_freeze_mask(self, score_xyz, score_rgb, eps_xyz, eps_rgb, mode, frozen,
                           proposal=None, n_frozen=None, stream=None):
        n = frozen.numel()
        check(self.h, self.L.gsta_update_freeze_mask(self.h, _arr(score_xyz, (n,), torch.float32, "score_xyz"),
                                                      _arr(score_rgb, (n,), torch.float32, "score_rgb"), n,
                                                      float(eps_xyz), float(eps_rgb), int(mode),
                                                      _arr(proposal, (n,), torch.uint8, "proposal"),
                                                      _arr(frozen, (n,), torch.uint8, "frozen"),
                                                      _arr(n_frozen, (1,), torch.int64, "n_frozen"),
                                                      _stream(stream)))

    def dssim_loss(self, image, target, lam, dL_dimage, ssim_sum, stream=None):
        """Eq. 3's D-SSIM term: dL_dimage (the L1 gradient on entry) becomes
        (1 - lam) dL_dimage + lam dL_D-SSIM/dimage; ssim_sum (device double
        [1]) receives the sum of the SSIM map."""
        sh = tuple(image.shape)
        if len(sh) != 4 or sh[1] != 3:
            raise ValueError("image: expected [views, 3, H, W]")
        check(self.h, self.L.gsta_dssim_loss(self.h, _arr(image, sh, torch.float32, "image"),
                                              _arr(target, sh, torch.float32, "target"), sh[0], sh[2], sh[3],
                                              float(lam), _arr(dL_dimage, sh, torch.float32, "dL_dimage"),
                                              _arr(ssim_sum, (1,), torch.float64, "ssim_sum"), _stream(stream)))

    def update_freeze_mask_rule(self, rule, score, fraction, seed, draw, mode, frozen, n_frozen=None,
                                stream=None):
        """The ablation's naive freezing rules: rule "mingrad" (the fraction of
        Gaussians with the smallest score) or "random" (Philox draws)."""
        r = {"mingrad": _lib.FREEZE_RULE_MINGRAD, "random": _lib.FREEZE_RULE_RANDOM}[rule]
        n = frozen.numel()
        check(self.h, self.L.gsta_update_freeze_mask_rule(
            self.h, r, _arr(score, (n,), torch.float32, "score"), n, float(fraction), int(seed), int(draw),
            int(mode), _arr(frozen, (n,), torch.uint8, "frozen"), _arr(n_frozen, (1,), torch.int64, "n_frozen"),
            _stream(stream)))

    def partition_frozen(self, frozen, arrays, tmp, n_active=None, stream=None):
        """Stable partition of the columns by the freeze map (active first),
        in place.  frozen: uint8 [n]; arrays: device tensors [rows, n] (unit
        column stride, any row stride) or [n], 1-, 2- or 4-byte elements;
        tmp: device tensor of at least max(rows * n * elem_bytes) bytes;
        n_active: device int64 [1] or None."""
        n = frozen.numel()
        descs = []
        for k, t in enumerate(arrays):
            if t.device.type != "cuda":
                raise ValueError(f"arrays[{k}] is not a device tensor")
            if t.dim() == 1:
                t2 = t.view(1, -1)
            elif t.dim() == 2:
                t2 = t
            else:
                raise ValueError(f"arrays[{k}]: expected [rows, n] or [n]")
            if t2.shape[1] != n:
                raise ValueError(f"arrays[{k}]: {t2.shape[1]} columns, frozen has {n}")
            if n > 0 and (t2.stride(1) != 1 or (t2.shape[0] > 1 and t2.stride(0) < n)):
                raise ValueError(f"arrays[{k}] needs unit column stride and row stride >= n")
            ld = t2.stride(0) if t2.shape[0] > 1 else max(n, 1)
            descs.append(_lib.Columns(t2.data_ptr() or None, t2.shape[0], ld, t2.element_size()))
        arr = (_lib.Columns * max(len(descs), 1))(*descs)
        check(self.h, self.L.gsta_partition_frozen(self.h, n, _arr(frozen, (n,), torch.uint8, "frozen"), arr,
                                                    len(descs), tmp.data_ptr() if tmp is not None else None,
                                                    0 if tmp is None else tmp.numel() * tmp.element_size(),
                                                    _arr(n_active, (1,), torch.int64, "n_active"),
                                                    _stream(stream)))

    def densify_prune(self, p, m, v, degree, ema, frozen, dstats, noise, cfg, p_out, m_out, v_out,
                      ema_out, frozen_out, counts, stream=None):
        """Densify-and-prune into the output blocks (p_out etc. are [R, capacity]
        views; ema_out / frozen_out flat buffers of at least 4*capacity /
        capacity elements).  counts: device int64 [4] = (n_out, kept, clones,
        splits).  cfg: _lib.DensifyCfg."""
        sp, sm, sv = (params_struct(x, degree) for x in (p, m, v))
        so, smo, svo = (params_struct(x, degree) for x in (p_out, m_out, v_out))
        n, cap = sp.n, so.n
        if ema_out is not None and (ema_out.dtype != torch.float32 or not ema_out.is_contiguous()
                                    or ema_out.numel() < 4 * cap):
            raise ValueError("ema_out: contiguous float32 with room for 4 * capacity values")
        if frozen_out is not None and (frozen_out.dtype != torch.uint8 or not frozen_out.is_contiguous()
                                       or frozen_out.numel() < cap):
            raise ValueError("frozen_out: contiguous uint8 with room for capacity values")
        check(self.h, self.L.gsta_densify_prune(
            self.h, ctypes.byref(sp), ctypes.byref(sm), ctypes.byref(sv),
            _arr(ema, (4, n), torch.float32, "ema"), _arr(frozen, (n,), torch.uint8, "frozen"),
            _arr(dstats, (4, n), torch.float32, "dstats"), _arr(noise, (6, n), torch.float32, "noise"),
            ctypes.byref(cfg), ctypes.byref(so), ctypes.byref(smo), ctypes.byref(svo),
            _ptr(ema_out), _ptr(frozen_out), _arr(counts, (4,), torch.int64, "counts"), _stream(stream)))

    def opacity_to_absolute(self, p, m, v, degree, stream=None):
        """Finetune switch to the absolute opacity activation: row 10 <-
        sigmoid(row 10), its Adam moments zeroed."""
        sp, sm, sv = (params_struct(x, degree) for x in (p, m, v))
        check(self.h, self.L.gsta_opacity_to_absolute(self.h, ctypes.byref(sp), ctypes.byref(sm), ctypes.byref(sv),
                                                       _stream(stream)))

    def opacity_reset(self, p, m, v, degree, frozen, logit_cap, stream=None):
        sp, sm, sv = (params_struct(x, degree) for x in (p, m, v))
        check(self.h, self.L.gsta_opacity_reset(self.h, ctypes.byref(sp), ctypes.byref(sm), ctypes.byref(sv),
                                                 _arr(frozen, (sp.n,), torch.uint8, "frozen"),
                                                 float(logit_cap), _stream(stream)))

    # ---- learned freeze proposer (bf16 arrays are torch.int16 / uint16 storage) ----
    def traj_push(self, ema, ring, slot, stream=None):
        n = ema.shape[1]
        check(self.h, self.L.gsta_traj_push(self.h, _arr(ema, (4, n), torch.float32, "ema"), n,
                                             _arr(ring, (8, 4, n), torch.int16, "ring"), int(slot), _stream(stream)))

    def mlp_feature_stats(self, ring, head, sums, stream=None):
        n = ring.shape[2]
        check(self.h, self.L.gsta_mlp_feature_stats(self.h, _arr(ring, (8, 4, n), torch.int16, "ring"), n, int(head),
                                                     _arr(sums, (64,), torch.float64, "sums"), _stream(stream)))

    def mlp_features(self, ring, head, mean, std, x, stream=None):
        n = ring.shape[2]
        check(self.h, self.L.gsta_mlp_features(self.h, _arr(ring, (8, 4, n), torch.int16, "ring"), n, int(head),
                                                _arr(mean, (32,), torch.float32, "mean"),
                                                _arr(std, (32,), torch.float32, "std"),
                                                _arr(x, (n, 32), torch.int16, "x"), _stream(stream)))

    def mlp_forward(self, w_bf16, w, x, logits, h1=None, h2=None, stream=None):
        n = x.shape[0]
        check(self.h, self.L.gsta_mlp_forward(self.h, _arr(w_bf16, (_lib.MLP_BF16,), torch.int16, "w_bf16"),
                                               _arr(w, (_lib.MLP_PARAMS,), torch.float32, "w"),
                                               _arr(x, (n, 32), torch.int16, "x"), n,
                                               _arr(logits, (n,), torch.float32, "logits"),
                                               _arr(h1, (n, 64), torch.int16, "h1"),
                                               _arr(h2, (n, 64), torch.float32, "h2"), _stream(stream)))

    def mlp_bce(self, logits, labels, dz, loss, stream=None):
        n = logits.shape[0]
        check(self.h, self.L.gsta_mlp_bce(self.h, _arr(logits, (n,), torch.float32, "logits"),
                                           _arr(labels, (n,), torch.uint8, "labels"), n,
                                           _arr(dz, (n,), torch.float32, "dz"),
                                           _arr(loss, (1,), torch.float64, "loss"), _stream(stream)))

    def mlp_backward(self, w_bf16, w, x, h1, h2, dz, grad, stream=None):
        n = x.shape[0]
        check(self.h, self.L.gsta_mlp_backward(self.h, _arr(w_bf16, (_lib.MLP_BF16,), torch.int16, "w_bf16"),
                                                _arr(w, (_lib.MLP_PARAMS,), torch.float32, "w"),
                                                _arr(x, (n, 32), torch.int16, "x"),
                                                _arr(h1, (n, 64), torch.int16, "h1"),
                                                _arr(h2, (n, 64), torch.float32, "h2"),
                                                _arr(dz, (n,), torch.float32, "dz"), n,
                                                _arr(grad, (_lib.MLP_PARAMS,), torch.float32, "grad"),
                                                _stream(stream)))

    def mlp_adam(self, w, grad, m, v, lr, beta1, beta2, eps, step, w_bf16, stream=None):
        P = (_lib.MLP_PARAMS,)
        check(self.h, self.L.gsta_mlp_adam(self.h, _arr(w, P, torch.float32, "w"), _arr(grad, P, torch.float32, "grad"),
                                            _arr(m, P, torch.float32, "m"), _arr(v, P, torch.float32, "v"),
                                            float(lr), float(beta1), float(beta2), float(eps), int(step),
                                            _arr(w_bf16, (_lib.MLP_BF16,), torch.int16, "w_bf16"),
                                            _stream(stream)))

    def mlp_sync_bf16(self, w, w_bf16, stream=None):
        check(self.h, self.L.gsta_mlp_sync_bf16(self.h, _arr(w, (_lib.MLP_PARAMS,), torch.float32, "w"),
                                                 _arr(w_bf16, (_lib.MLP_BF16,), torch.int16, "w_bf16"),
                                                 _stream(stream)))

    def mlp_propose(self, logits, score_xyz, score_rgb, logit_threshold, veto_xyz, veto_rgb, proposal, stream=None):
        n = logits.shape[0]
        check(self.h, self.L.gsta_mlp_propose(self.h, _arr(logits, (n,), torch.float32, "logits"),
                                               _arr(score_xyz, (n,), torch.float32, "score_xyz"),
                                               _arr(score_rgb, (n,), torch.float32, "score_rgb"), n,
                                               float(logit_threshold), float(veto_xyz), float(veto_rgb),
                                               _arr(proposal, (n,), torch.uint8, "proposal"), _stream(stream)))

    def l1_loss(self, image, target, dL_dimage, sums, stream=None):
        sh = tuple(image.shape)
        check(self.h, self.L.gsta_l1_loss(self.h, _arr(image, sh, torch.float32, "image"),
                                           _arr(target, sh, torch.float32, "target"), image.numel(),
                                           _arr(dL_dimage, sh, torch.float32, "dL_dimage"),
                                           _arr(sums, (2,), torch.float64, "sums"), _stream(stream)))


def adam_sched_tensor(step, beta1, beta2, eps, lr_rows, pos_lr_init, pos_lr_final, decay_iters,
                      pos_scale=1.0) -> torch.Tensor:
    """A device buffer holding a gsta_adam_sched."""
    s = AdamSched()
    s.step, s.decay_iters = int(step), int(decay_iters)
    s.beta1, s.beta2, s.eps = float(beta1), float(beta2), float(eps)
    s.pos_lr_init, s.pos_lr_final, s.pos_scale = float(pos_lr_init), float(pos_lr_final), float(pos_scale)
    for i, x in enumerate(lr_rows):
        s.lr[i] = float(x)
    raw = bytes(s)
    return torch.frombuffer(bytearray(raw), dtype=torch.uint8).cuda()


def set_adam_sched_field(buf: torch.Tensor, name: str, value):
    """Write one scalar field of a device gsta_adam_sched (stream-ordered copy)."""
    off = getattr(AdamSched, name).offset
    dtype = torch.int32 if name in ("step", "decay_iters") else torch.float32
    buf[off:off + 4].copy_(torch.tensor([value], dtype=dtype).view(torch.uint8))
