"""GSta training loop on top of libgsta (Algorithm 1).

Per iteration: (densify / prune / opacity reset) -> (freeze-map update or
reset) -> render_forward (+ fused L1 loss) -> render_backward (frozen skipped,
gradient-norm EMAs, densification statistics) -> adam_masked (frozen
skipped).  Everything per Gaussian or per pixel runs in the HIP library; this
module keeps only host scalars (schedule, learning rates) and the device
buffers PyTorch allocates.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib
from .core import Context, adam_sched_tensor, camera_array, n_rows, set_adam_sched_field
from .schedule import (NONE, RESET, UPDATE, DensifySchedule, FreezeSchedule, LearningRates, PlateauLR,
                       early_stop, scene_extent, training_end)

FLT_MAX = float(np.finfo(np.float32).max)


def _padded(R: int, n: int, fill: float = 0.0, dtype=torch.float32) -> torch.Tensor:
    """[R, n] view of an [R, ld] device block with ld a multiple of 64 (16-byte rows)."""
    ld = max(64, (n + 63) // 64 * 64)
    return torch.full((R, ld), fill, dtype=dtype, device="cuda")[:, :n]


@dataclass
class TrainConfig:
    iters: int
    freeze: bool = True
    schedule: FreezeSchedule | None = None
    lrs: LearningRates = field(default_factory=LearningRates)
    ema_beta: float = 0.9
    beta1: float = 0.9
    beta2: float = 0.999
    adam_eps: float = 1e-15
    bg: tuple = (0.0, 0.0, 0.0)
    eval_every: int | None = None        # K_PSNR; None: no periodic validation
    early_stop_eps: float | None = None  # eq. 7 threshold (dB); None: no early stop
    plateau: PlateauLR | None = None
    finetune_iters: int = 0              # K_f: iterations trained after the freezing window closes
    track_ema: bool = False              # keep gradient-norm EMAs even without freezing
    device_sched: bool = False           # Adam scalars from a device schedule (implied by graph)
    graph: bool = False                  # capture each view's iteration once in a HIP graph, then replay
    views_per_step: int = 1              # V_b views rendered per library call; the loss averages them
    batches: list | None = None          # fixed groups of views (then the view order lists group ids); needed
                                         # for graph capture with several views per step
    densify: DensifySchedule | None = None   # adaptive densification (the number of Gaussians changes)
    max_gaussians: int | None = None     # capacity of the parameter blocks (default: the initial count)
    traj_every: int = 0                  # push the gradient-norm averages to the 8-deep ring every k iterations
    proposer: object | None = None       # learned freeze proposer (proposer.Proposer), needs traj_every
    dataset: object | None = None        # proposer.ProposerDataset to record the rule's decisions into
    update_hook: object | None = None    # called as hook(trainer, k, eps_xyz, eps_rgb, accepted proposals or None)
                                         # after every freeze-map update (measurement, e.g. false-freeze counts)
    partition: bool = False              # after each freeze update, move the frozen columns behind the active ones
    fused_loss: bool = True              # L1 loss computed by the forward compositing (else a separate pass)
    lambda_ssim: float = 0.0             # eq. 3: L = (1 - lambda) L1 + lambda D-SSIM (the paper uses 0.2)
    abs_opacity_finetune: bool = False   # Section 4.1: opacity = |x| instead of sigmoid once the finetune starts
    sh_mask_finetune: bool = False       # Section 3.3: learn hard SH-band masks during the finetune (+small variant)
    sh_mask_threshold: float = 0.01      # gate: sigmoid(logit) > threshold
    sh_mask_init: float = 2.0            # initial logits (every gate open)
    sh_mask_lr: float = 0.01             # Adam learning rate of the logits
    sh_mask_lambda: float = 5e-4         # weight of the masks' sparsity term (mean sigmoid)


class Trainer:
    """One GSta (or plain, freeze=False) training run on a single GPU."""

    def __init__(self, params0: np.ndarray, degree: int, cams, targets: torch.Tensor, cfg: TrainConfig,
                 view_order: np.ndarray, ctx: Context | None = None, capacity: int | None = None,
                 val_views=None):
        self.degree = degree
        self.cfg = cfg
        self.R, self.n = params0.shape
        assert self.R == n_rows(degree)
        self.cams = cams
        self.H, self.W = cams[0].height, cams[0].width
        self.cam1 = [camera_array([c]) for c in cams]
        self.batch_cams = None if cfg.batches is None else [camera_array([cams[v] for v in b]) for b in cfg.batches]
        self.targets = targets
        self.order = view_order
        self.val_views = list(range(len(cams))) if val_views is None else list(val_views)
        self.cap = max(cfg.max_gaussians or self.n, self.n)
        self.ctx = ctx or Context(self.cap, min(8, len(cams)), self.H, self.W, capacity or (1 << 22), n_slots=1)
        if self.ctx.limits.max_gaussians < self.cap:
            raise ValueError("the context reserves fewer Gaussians than the trainer's capacity")
        # Parameter, moment, EMA and freeze-map storage sized for the capacity;
        # densification compacts one set into the other and swaps.
        nsets = 2 if cfg.densify is not None else 1
        self.sets = [dict(P=_padded(self.R, self.cap), M=_padded(self.R, self.cap), V=_padded(self.R, self.cap),
                          ema=torch.full((4 * self.cap,), FLT_MAX, device="cuda"),
                          frozen=torch.zeros(self.cap, dtype=torch.uint8, device="cuda")) for _ in range(nsets)]
        self.cur = 0
        self.G_full = _padded(self.R, self.cap)
        self.dstats_buf = torch.zeros(4 * self.cap, device="cuda") if cfg.densify is not None else None
        self._bind(self.n)
        self.P.copy_(torch.from_numpy(np.ascontiguousarray(params0, dtype=np.float32)).cuda())
        self.counts = torch.zeros(4, dtype=torch.int64, device="cuda")
        self.n_history: list[tuple[int, int]] = []
        if cfg.densify is not None:
            ds = cfg.densify
            self.extent = scene_extent([c.campos for c in cams])
            self.dens_rng = np.random.Generator(np.random.Philox(ds.seed))
        self.n_frozen = torch.zeros(1, dtype=torch.int64, device="cuda")
        if cfg.batches is not None:
            sizes = {len(b) for b in cfg.batches}
            if len(sizes) != 1 or min(sizes) < 1 or min(sizes) > self.ctx.limits.max_views:
                raise ValueError("batches must be non-empty groups of equal size within the context's views")
            cfg.views_per_step = sizes.pop()
        vb = cfg.views_per_step
        if vb > 1 and cfg.graph and cfg.batches is None:
            raise ValueError("graph capture with several views per step needs fixed batches (cfg.batches)")
        # each fixed batch's targets, contiguous, gathered once
        self.batch_targets = None if cfg.batches is None else [
            torch.index_select(targets, 0, torch.as_tensor(b, device="cuda")).contiguous() for b in cfg.batches]
        self.image = torch.empty((vb, 3, self.H, self.W), device="cuda")
        self.dL = torch.empty_like(self.image)
        self.tgt_batch = torch.empty_like(self.image) if vb > 1 else None
        self.sums = torch.zeros(2, dtype=torch.float64, device="cuda")
        self.ssim_sum = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.opacity_act = 0                 # 1 after the finetune's switch to the absolute activation
        # SH-band masks (logits, gradient, moments; [3, n] views of capacity-sized
        # storage), allocated and switched on when the finetune starts
        self.shm = None
        self.shm_step = 0
        self.shm_out = torch.zeros(4, dtype=torch.float64, device="cuda")
        if cfg.sh_mask_finetune and cfg.graph:
            raise ValueError("the SH-band masks' Adam takes a host step count: no graph capture with them")
        if cfg.sh_mask_finetune and not (0.0 < cfg.sh_mask_threshold < 1.0):
            raise ValueError("sh_mask_threshold must be in (0, 1)")
        self.step_count = 0
        self.k = 0
        self.psnrs: list[float] = []
        self.stop_iter: int | None = None
        self.pos_scale = 1.0
        self.scale_log: list[tuple[int, float]] = []     # (first iteration using it, position-LR scale)
        self.frozen_log: list[tuple[int, int]] = []
        self.frozen_counts = torch.zeros(1024, dtype=torch.int64, device="cuda")
        self.use_sched = cfg.device_sched or cfg.graph
        if self.use_sched:
            l = cfg.lrs
            self.sched = adam_sched_tensor(1, cfg.beta1, cfg.beta2, cfg.adam_eps, l.rows(0, degree),
                                           l.extent * l.pos_init, l.extent * l.pos_final, l.decay_iters)
        self.graphs: dict = {}                # view (or batch id) -> library graph (core.Graph)
        self.traj = None
        if cfg.traj_every:
            if cfg.densify is not None:
                raise ValueError("the trajectory ring does not follow densification")
            from .proposer import TrajectoryLog
            self.traj = TrajectoryLog(self.ctx, self.n, cfg.traj_every)
        elif cfg.proposer is not None or cfg.dataset is not None:
            raise ValueError("the proposer and its dataset need traj_every > 0")
        self.prop_buf = torch.zeros(self.n, dtype=torch.uint8, device="cuda") if cfg.proposer is not None else None
        if cfg.schedule is not None and cfg.schedule.rule not in ("gradient", "mingrad", "random"):
            raise ValueError(f"unknown freezing rule {cfg.schedule.rule!r}")
        if cfg.schedule is not None and cfg.schedule.rule != "gradient" and (cfg.proposer or cfg.dataset):
            raise ValueError("the learned proposer works with the gradient rule only")
        # Column permutation of the partitioned layout: column i holds the
        # Gaussian that started in column origin[i] (not tracked through
        # densification, which renumbers the set).
        self.origin = None
        self.n_active = torch.zeros(1, dtype=torch.int64, device="cuda")
        if cfg.partition:
            if not cfg.freeze:
                raise ValueError("partition needs freeze=True")
            if cfg.dataset is not None:
                raise ValueError("the proposer dataset records column positions; it cannot follow a partition")
            if cfg.densify is None:
                self.origin = torch.arange(self.n, dtype=torch.int32, device="cuda")

    def _bind(self, n: int):
        """Point the working views at the first n columns of the current set."""
        st = self.sets[self.cur]
        self.n = n
        self.P, self.M, self.Vm = st["P"][:, :n], st["M"][:, :n], st["V"][:, :n]
        self.ema = st["ema"][:4 * n].view(4, n)
        self.frozen = st["frozen"][:n]
        self.G = self.G_full[:, :n]
        self.dstats = None if self.dstats_buf is None else self.dstats_buf[:4 * n].view(4, n)

    # ------------------------------------------------------------------
    def _densify_step(self, k: int):
        """Densify / prune (compaction into the other set) and opacity reset
        before iteration k, from the statistics of the iterations since the
        previous densify step."""
        ds = self.cfg.densify
        if ds is None:
            return
        if ds.densify_now(k, self.stop_iter):
            if self.shm is not None:
                raise ValueError("densification after the SH-band masks started: the masks do not follow it")
            ex, er = ds.thresholds(k, ds.end(self.stop_iter))
            use_rgb = bool(self.dens_rng.random() < ds.rgb_prob)
            # the split children's normals are drawn in the kernel from Philox (seed, iteration, column)
            cfg = _lib.DensifyCfg(ex, er, int(use_rgb), ds.split_log_scale(self.extent), ds.prune_logit(),
                                  float(np.log(ds.split_div)), ds.seed, k)
            noise = None
            out = self.sets[1 - self.cur]
            frz = self.frozen if self.cfg.freeze else None
            ema = self.ema if (self.cfg.freeze or self.cfg.track_ema) else None
            self.ctx.densify_prune(self.P, self.M, self.Vm, self.degree, ema, frz, self.dstats, noise, cfg,
                                   out["P"], out["M"], out["V"], out["ema"], out["frozen"], self.counts)
            st, max_inst = self.ctx.check()          # synchronises; reads the device flags
            n_out = int(self.counts[0])
            if st != _lib.GSTA_OK:
                raise _lib.GstaError(st, f"densify at iteration {k}: {n_out} Gaussians for capacity {self.cap}"
                                     if st == _lib.GSTA_ERR_CAPACITY else "device flag raised")
            n_in = self.n
            self.cur = 1 - self.cur
            self._bind(n_out)
            self.dstats.zero_()
            self._drop_graphs()                       # pointers and sizes changed: capture again
            self.n_history.append((k, n_out))
            # keep the tile-instance capacity ahead of the growth
            need = int(max_inst * max(1.0, n_out / max(n_in, 1)) * 1.3) + 1024
            if need > self.ctx.limits.instance_capacity:
                self.ctx.reserve(instance_capacity=need)
        if ds.reset_now(k, self.stop_iter):
            frz = self.frozen if self.cfg.freeze else None
            self.ctx.opacity_reset(self.P, self.M, self.Vm, self.degree, frz, ds.reset_logit())

    def _freeze_step(self, k: int):
        s = self.cfg.schedule
        if not self.cfg.freeze or s is None:
            return
        act = s.action(k, self.stop_iter)
        if act == NONE:
            return
        if act == UPDATE and s.rule != "gradient":
            # the ablation's naive rules; `draw` = the iteration keeps every update's draws fresh
            self.ctx.update_freeze_mask_rule(s.rule, self.ema[0], s.rule_fraction(k), s.seed, k,
                                             0 if s.accumulate else 2, self.frozen, n_frozen=self.n_frozen)
            if self.cfg.partition:
                self._partition()
        elif act == UPDATE:
            ex, er = s.thresholds(k, s.window_close(self.stop_iter))
            prop = None
            if self.cfg.dataset is not None:
                self.cfg.dataset.record(self.traj, self.ema, ex, er)
            if self.cfg.proposer is not None:
                prop = self.cfg.proposer.propose(self.traj.ring, self.traj.head, self.ema, ex, er, self.prop_buf)
            if self.cfg.update_hook is not None:
                self.cfg.update_hook(self, k, ex, er, prop, before=True)
            self.ctx.update_freeze_mask(self.ema[0], self.ema[1], ex, er, 0, self.frozen, proposal=prop,
                                        n_frozen=self.n_frozen)
            if self.cfg.update_hook is not None:
                self.cfg.update_hook(self, k, ex, er, prop, before=False)
            if self.cfg.partition:
                self._partition()
        elif act == RESET:
            self.ctx.update_freeze_mask(None, None, 0.0, 0.0, 1, self.frozen, n_frozen=self.n_frozen)
            if self.cfg.partition:
                self.n_active.fill_(self.n)
        i = len(self.frozen_log)
        if i < self.frozen_counts.numel():
            self.frozen_counts[i:i + 1].copy_(self.n_frozen, non_blocking=True)
        self.frozen_log.append((k, act))
        self.check_flags(f"freeze-map change before iteration {k}")

    def check_flags(self, where: str):
        """Synchronise and raise if a kernel raised a device flag since the
        last check (tile instances or forward checkpoints beyond the reserved
        capacity, a non-finite gradient): the iterations since then trained
        on incomplete or wrong gradients."""
        st, need = self.ctx.check()
        if st != _lib.GSTA_OK:
            raise _lib.GstaError(st, f"device flag raised by the iterations up to the {where} "
                                     f"(instances needed: {need}, reserved: {self.ctx.limits.instance_capacity})")

    def _drop_graphs(self):
        """Forget the captured graphs (after the stream has finished them)."""
        if self.graphs:
            torch.cuda.current_stream().synchronize()
            self.graphs.clear()

    def _partition(self):
        """Permute every per-Gaussian array in place so that the active
        Gaussians form the prefix [0, n_active): the backward's per-Gaussian
        chain and Adam then skip whole waves of frozen columns.  The gradient
        block is dead between iterations and serves as the scratch buffer;
        pointers do not change, so captured graphs stay valid."""
        arrays = [self.P, self.M, self.Vm, self.ema]
        if self.dstats is not None:
            arrays.append(self.dstats)
        if self.traj is not None:
            arrays.append(self.traj.ring.view(32, self.n))
        if self.origin is not None:
            arrays.append(self.origin)
        self.ctx.partition_frozen(self.frozen, arrays, self.G_full, self.n_active)

    def in_original_order(self, x: torch.Tensor) -> torch.Tensor:
        """x ([rows, n] or [n], columns in the current layout) with its
        columns back in the initial order of the Gaussians."""
        if self.origin is None:
            if self.cfg.partition:
                raise ValueError("the column order is not tracked through densification")
            return x
        out = torch.empty_like(x)
        out[..., self.origin.long()] = x
        return out

    def freeze_history(self):
        """[(iteration, action, frozen count after it)] for every freeze-map change."""
        c = self.frozen_counts[: len(self.frozen_log)].cpu().tolist()
        return [(k, a, n) for (k, a), n in zip(self.frozen_log, c)]

    def _body(self, view, k: int):
        """Forward, loss, backward and optimizer step of one view or a batch
        of views (the part a HIP graph captures)."""
        cfg = self.cfg
        frz = self.frozen if cfg.freeze else None
        ema = self.ema if (cfg.freeze or cfg.track_ema) else None
        if isinstance(view, tuple):             # a fixed batch: ("batch", id)
            b = view[1]
            cam = self.batch_cams[b]
            tgt = self.batch_targets[b]
        elif isinstance(view, int):
            cam = self.cam1[view]
            tgt = self.targets[view:view + 1]
        else:
            cam = camera_array([self.cams[v] for v in view])
            idx = torch.as_tensor(view, device="cuda")
            torch.index_select(self.targets, 0, idx, out=self.tgt_batch)
            tgt = self.tgt_batch
        act = self.opacity_act
        mk = {} if self.shm is None else dict(sh_mask=self.shm["x"], sh_mask_threshold=cfg.sh_mask_threshold)
        if cfg.fused_loss:
            self.ctx.render_forward_l1(self.P, self.degree, cam, cfg.bg, tgt, self.image, self.dL, self.sums, 0,
                                       opacity_act=act, **mk)
        else:
            self.ctx.render_forward(self.P, self.degree, cam, cfg.bg, self.image, 0, opacity_act=act, **mk)
            self.ctx.l1_loss(self.image, tgt, self.dL, self.sums)
        if cfg.lambda_ssim > 0.0:
            self.ctx.dssim_loss(self.image, tgt, cfg.lambda_ssim, self.dL, self.ssim_sum)
        self.ctx.render_backward(self.P, self.degree, cam, cfg.bg, 0, self.dL, frz, self.G, None, ema,
                                 cfg.ema_beta, dstats=self.dstats, opacity_act=act,
                                 sh_mask_grad=None if self.shm is None else self.shm["g"], **mk)
        if self.shm is not None:
            # the masks' sparsity term adds its gradient; then their own Adam step
            self.shm_step += 1
            self.ctx.sh_mask_reg(self.shm["x"], cfg.sh_mask_threshold, cfg.sh_mask_lambda, self.shm_out,
                                 frozen=frz, grad=self.shm["g"])
            self.ctx.adam_rows(self.shm["x"], self.shm["g"], self.shm["m"], self.shm["v"], [cfg.sh_mask_lr] * 3,
                               cfg.beta1, cfg.beta2, cfg.adam_eps, self.shm_step, frz)
        if self.use_sched:
            self.ctx.adam_masked_sched(self.P, self.G, self.M, self.Vm, self.degree, self.sched, frz)
        else:
            lr = cfg.lrs.rows(k, self.degree, self.pos_scale)
            self.ctx.adam_masked(self.P, self.G, self.M, self.Vm, self.degree, lr, cfg.beta1, cfg.beta2,
                                 cfg.adam_eps, self.step_count, frz)

    def step(self):
        """One training iteration k = self.k."""
        k = self.k
        cfg = self.cfg
        self._densify_step(k)
        if cfg.abs_opacity_finetune and self.opacity_act == 0 and k >= self.window_close():
            # the finetune starts: opacity = |x| from now on, x = the current opacity
            self.ctx.opacity_to_absolute(self.P, self.M, self.Vm, self.degree)
            self.opacity_act = 1
            self._drop_graphs()                      # the captured calls carry the old activation
        if cfg.sh_mask_finetune and self.shm is None and k >= self.window_close():
            # the finetune starts: every Gaussian's three band masks, all open
            # (the parameter block's row stride, which the library requires of them)
            self.shm = {nm: _padded(3, self.cap)[:, :self.n] for nm in ("x", "g", "m", "v")}
            self.shm["x"].fill_(cfg.sh_mask_init)
        if self.traj is not None:
            self.traj.maybe_push(k, self.ema)
        self._freeze_step(k)
        vb = cfg.views_per_step
        if cfg.batches is not None:
            view = ("batch", int(self.order[k % len(self.order)]))
        elif vb == 1:
            view = int(self.order[k % len(self.order)])
        else:
            view = [int(self.order[(k * vb + i) % len(self.order)]) for i in range(vb)]
        self.step_count += 1
        if cfg.graph:
            g = self.graphs.get(view)
            if g is None:
                # captured by the library on a side stream (the null stream cannot be captured)
                side = torch.cuda.Stream()
                side.wait_stream(torch.cuda.current_stream())
                with torch.cuda.stream(side):
                    g = self.ctx.capture(lambda: self._body(view, k))
                torch.cuda.current_stream().wait_stream(side)
                self.graphs[view] = g
            g.launch()
        else:
            self._body(view, k)
        self.k += 1
        self._after_step()

    def _after_step(self):
        """Host bookkeeping after iteration k - 1: validation every K_PSNR
        iterations while the freezing window is open, which feeds eq. 7 and
        the plateau scheduler."""
        cfg = self.cfg
        if (cfg.eval_every and self.k % cfg.eval_every == 0 and self.stop_iter is None
                and self.k < self.window_close()):
            self._validate()

    def _validate(self):
        p = self.evaluate(self.val_views)
        self.check_flags(f"validation after iteration {self.k}")
        self.psnrs.append(p)
        if self.cfg.plateau is not None:
            scale = self.cfg.plateau.step(p)
            if scale != self.pos_scale:
                if self.use_sched:
                    set_adam_sched_field(self.sched, "pos_scale", scale)
                self.scale_log.append((self.k, scale))
            self.pos_scale = scale
        if self.cfg.early_stop_eps is not None and early_stop(self.psnrs, self.cfg.early_stop_eps):
            self.stop_iter = self.k

    def window_close(self) -> int:
        """Iteration at which the freezing window closes (the finetune starts):
        the schedule's window end (the forced stop; the run's length without
        a schedule) or the early-stop iteration, whichever comes first."""
        s = self.cfg.schedule
        end = s.window_end if s is not None else self.cfg.iters
        return end if self.stop_iter is None else min(end, self.stop_iter)

    def end_iter(self) -> int:
        """Length of the whole training as known now (Algorithm 1): the
        window close + K_f when the window closes before cfg.iters, else
        cfg.iters."""
        s = self.cfg.schedule
        end = s.window_end if s is not None else self.cfg.iters
        return training_end(self.cfg.iters, end, self.stop_iter, self.cfg.finetune_iters)

    @property
    def finished(self) -> bool:
        return self.k >= self.end_iter()

    def run(self, iters: int | None = None):
        """Train `iters` iterations, or (None) to the end of training."""
        if iters is None:
            while not self.finished:
                self.step()
        else:
            for _ in range(iters):
                self.step()

    # ------------------------------------------------------------------
    def render_views(self, views, out: torch.Tensor | None = None) -> torch.Tensor:
        """Render views (up to 8 per library call) into [len(views), 3, H, W]."""
        views = list(views)
        out = out if out is not None else torch.empty((len(views), 3, self.H, self.W), device="cuda")
        vmax = self.ctx.limits.max_views
        with self.ctx.forward_only():
            for b in range(0, len(views), vmax):
                vs = views[b:b + vmax]
                self.ctx.render_forward(self.P, self.degree, [self.cams[v] for v in vs], self.cfg.bg,
                                        out[b:b + len(vs)], 0, opacity_act=self.opacity_act,
                                        **({} if self.shm is None else dict(
                                            sh_mask=self.shm["x"], sh_mask_threshold=self.cfg.sh_mask_threshold)))
        return out

    def sh_mask_stats(self) -> dict | None:
        """The SH-band masks after the last step: the sparsity term, open
        gates per band, and the SH coefficients a stored model keeps
        (closed bands pruned) as a fraction of all of them."""
        if self.shm is None:
            return None
        o = self.shm_out.cpu().numpy()
        D = self.degree
        kept = 3 * self.n + sum(3 * (2 * l + 1) * o[l] for l in range(1, D + 1))
        total = 3 * self.n * (D + 1) ** 2
        return {"loss": float(o[0]), "open": [int(o[l]) for l in range(1, 4)], "n": self.n,
                "sh_coeff_kept": float(kept / total)}

    def evaluate(self, views=None) -> float:
        """Mean over views of the PSNR 10 log10(count / SSE), the squared
        error summed by gsta_l1_loss over the image clamped to [0, 1]."""
        views = self.val_views if views is None else list(views)
        img = self.render_views(views)
        sse = self.view_sse(img, views)
        count = 3 * self.H * self.W
        return float(np.mean([10.0 * np.log10(count / s) for s in sse]))

    def view_sse(self, img: torch.Tensor, views) -> list[float]:
        """Per view, the squared error of the clamped image against its
        target, summed by the library's loss kernel (one readback)."""
        views = list(views)
        sums = torch.zeros((len(views), 2), dtype=torch.float64, device="cuda")
        scratch = torch.empty((1, 3, self.H, self.W), device="cuda")
        for i, v in enumerate(views):
            self.ctx.l1_loss(img[i:i + 1], self.targets[v:v + 1], scratch, sums[i])
        return sums[:, 1].cpu().tolist()

    def loss(self) -> float:
        """Eq. 3 loss of the last iteration (synchronises)."""
        count = self.image.numel()
        l1 = float(self.sums[0]) / count
        lam = self.cfg.lambda_ssim
        return l1 if lam == 0.0 else (1.0 - lam) * l1 + lam * (1.0 - float(self.ssim_sum[0]) / count)

    def frozen_fraction(self) -> float:
        return float(self.frozen.float().mean()) if self.cfg.freeze else 0.0


def render_targets(ctx: Context, params: np.ndarray, degree: int, cams, bg=(0.0, 0.0, 0.0)) -> torch.Tensor:
    """Render training targets for every camera through the library."""
    R, n = params.shape
    P = _padded(R, n)
    P.copy_(torch.from_numpy(np.ascontiguousarray(params, dtype=np.float32)).cuda())
    H, W = cams[0].height, cams[0].width
    out = torch.empty((len(cams), 3, H, W), device="cuda")
    vmax = ctx.limits.max_views
    with ctx.forward_only():
        for b in range(0, len(cams), vmax):
            cs = cams[b:b + vmax]
            ctx.render_forward(P, degree, cs, bg, out[b:b + len(cs)], 0)
    return out


def required_capacity(ctx: Context, params: np.ndarray, degree: int, cams) -> int:
    """Largest per-call instance count over the cameras (renders them once)."""
    render_targets(ctx, params, degree, cams)
    st, need = ctx.check()
    if st not in (_lib.GSTA_OK, _lib.GSTA_ERR_CAPACITY):
        raise _lib.GstaError(st, "check failed")
    return need
