"""Learned freeze proposer (a project extension; the paper has no such
model).

An MLP 32 -> 64 -> 64 -> 1 reads, per Gaussian, the last 8 logged values of
its 4 gradient-norm averages (xyz, rgb, opacity, scale) as standardised
log10 features and proposes it for the freeze map.  The rule of Section
3.2.1 keeps the last word: a proposal is vetoed when either average is at
least c_v times the rule's current threshold, and accepted proposals are
OR-ed into the map at the rule's own update.  Training labels come from the
rule itself: a Gaussian is labelled 1 at a freeze update if the rule freezes
it at one of the next two updates, so an accepted proposal freezes a
Gaussian up to two updates earlier than the rule would.

Every per-Gaussian step (ring push, features, statistics, forward on bf16
matrix cores, BCE, weight gradients, Adam, propose/veto) runs in libgsta;
this module holds the device buffers and host scalars.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import _lib
from .core import Context

TAU = 0.9            # propose iff sigmoid(z) > TAU
VETO = 3.0           # c_v = lambda2 / lambda1 of the threshold schedule


def init_weights(seed: int = 3) -> np.ndarray:
    """He-normal hidden layers and a small output layer, from a seeded
    Philox stream; biases zero."""
    rng = np.random.Generator(np.random.Philox(seed))
    w = np.zeros(_lib.MLP_PARAMS, np.float32)
    w[0:2048] = rng.standard_normal(2048) * math.sqrt(2.0 / 32)
    w[2112:6208] = rng.standard_normal(4096) * math.sqrt(2.0 / 64)
    w[6272:6336] = rng.standard_normal(64) * math.sqrt(1.0 / 64)
    return w


class Proposer:
    """Weights, optimizer state and standardisation of the proposer."""

    def __init__(self, ctx: Context, seed: int = 3):
        self.ctx = ctx
        self.w = torch.from_numpy(init_weights(seed)).cuda()
        self.wb = torch.zeros(_lib.MLP_BF16, dtype=torch.int16, device="cuda")
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.grad = torch.zeros_like(self.w)
        self.step = 0
        self.mean = torch.zeros(32, device="cuda")
        self.std = torch.ones(32, device="cuda")
        ctx.mlp_sync_bf16(self.w, self.wb)

    # ---- standardisation over a set of ring snapshots -------------------
    def fit_standardisation(self, snapshots):
        """snapshots: [(ring [8][4][n] int16 tensor, head)]."""
        sums = torch.zeros(64, dtype=torch.float64, device="cuda")
        count = 0
        for ring, head in snapshots:
            self.ctx.mlp_feature_stats(ring, head, sums)
            count += ring.shape[2]
        s = sums.cpu().numpy()
        mean = s[:32] / count
        var = np.maximum(s[32:] / count - mean ** 2, 1e-12)
        self.mean = torch.from_numpy(mean.astype(np.float32)).cuda()
        self.std = torch.from_numpy(np.sqrt(var).astype(np.float32)).cuda()

    def features(self, ring, head, out=None):
        n = ring.shape[2]
        out = out if out is not None else torch.empty((n, 32), dtype=torch.int16, device="cuda")
        self.ctx.mlp_features(ring, head, self.mean, self.std, out)
        return out

    def logits(self, x, out=None):
        out = out if out is not None else torch.empty(x.shape[0], device="cuda")
        self.ctx.mlp_forward(self.wb, self.w, x, out)
        return out

    # ---- training ---------------------------------------------------------
    def fit(self, x, labels, epochs: int = 300, lr: float = 3e-3, log_every: int = 50):
        """Full-batch Adam on the mean BCE; returns [(epoch, loss)]."""
        n = x.shape[0]
        z = torch.empty(n, device="cuda")
        h1 = torch.empty((n, 64), dtype=torch.int16, device="cuda")
        h2 = torch.empty((n, 64), device="cuda")
        dz = torch.empty(n, device="cuda")
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        hist = []
        for e in range(epochs):
            self.ctx.mlp_forward(self.wb, self.w, x, z, h1, h2)
            self.ctx.mlp_bce(z, labels, dz, loss)
            self.ctx.mlp_backward(self.wb, self.w, x, h1, h2, dz, self.grad)
            self.step += 1
            self.ctx.mlp_adam(self.w, self.grad, self.m, self.v, lr, 0.9, 0.999, 1e-8, self.step, self.wb)
            if e % log_every == 0 or e == epochs - 1:
                hist.append((e, float(loss.cpu())))
        return hist

    # ---- inference at a freeze update --------------------------------------
    def propose(self, ring, head, ema, eps_xyz, eps_rgb, out, tau: float = TAU, veto: float = VETO):
        """Accepted proposals (uint8 [n]) for the rule's thresholds eps."""
        x = self.features(ring, head)
        z = self.logits(x)
        self.ctx.mlp_propose(z, ema[0], ema[1], math.log(tau / (1.0 - tau)), veto * eps_xyz, veto * eps_rgb, out)
        return out


class TrajectoryLog:
    """The 8-deep bf16 ring of gradient-norm averages of a training run,
    pushed every `every` iterations."""

    def __init__(self, ctx: Context, n: int, every: int):
        self.ctx = ctx
        self.every = every
        self.ring = torch.zeros((8, 4, n), dtype=torch.int16, device="cuda")
        self.head = 7
        self.pushes = 0

    def maybe_push(self, k: int, ema):
        if k % self.every == 0:
            self.head = (self.head + 1) % 8
            self.ctx.traj_push(ema, self.ring, self.head)
            self.pushes += 1


class ProposerDataset:
    """Training data logged from a rule-only run: at each freeze update u a
    snapshot of the ring and the rule's condition; labels[u] = condition at
    update u+1 OR at u+2 (built on the device with the freeze kernel)."""

    def __init__(self, ctx: Context, n: int):
        self.ctx = ctx
        self.n = n
        self.snaps: list[tuple[torch.Tensor, int]] = []
        self.labels: list[torch.Tensor] = []

    def record(self, log: TrajectoryLog, ema, eps_xyz, eps_rgb):
        for back in (1, 2):
            if len(self.labels) >= back:
                self.ctx.update_freeze_mask(ema[0], ema[1], eps_xyz, eps_rgb, 0, self.labels[-back])
        self.snaps.append((log.ring.clone(), log.head))
        self.labels.append(torch.zeros(self.n, dtype=torch.uint8, device="cuda"))

    def complete(self):
        """Snapshots whose two following updates were seen."""
        k = max(len(self.snaps) - 2, 0)
        return self.snaps[:k], self.labels[:k]

    def build(self, proposer: Proposer):
        snaps, labels = self.complete()
        if not snaps:
            raise ValueError("no complete training samples: fewer than 3 freeze updates were logged")
        proposer.fit_standardisation(snaps)
        x = torch.empty((len(snaps) * self.n, 32), dtype=torch.int16, device="cuda")
        for u, (ring, head) in enumerate(snaps):
            proposer.features(ring, head, x[u * self.n:(u + 1) * self.n])
        y = torch.cat(labels)
        return x, y
