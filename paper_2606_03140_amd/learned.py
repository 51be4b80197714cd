"""Learned starting charges for the SCC loop, trained and run on the GPU.

Per-atom radial descriptors (16 Gaussians x 2 neighbour species, 5 A
cutoff) feed one 32-64-64-1 SiLU network per central species; the
prediction, shifted to zero net charge, starts the SCC iteration in place of
zero charges (the plain loop stays the fallback; the number of iterations
each start takes measures the guess).  Training runs the FP32 forward,
loss, backward and Adam kernels of libgdm; inference runs the BF16 forward.
Only orchestration lives here.
"""
from __future__ import annotations

import numpy as np
import torch

from ._lib import Context, System

N_PARAMS = 6337          # per species: 64*32 + 64 + 64*64 + 64 + 64 + 1
DESCRIPTOR_CUTOFF = 5.0
_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def pack(nets) -> np.ndarray:
    """[2, 6337] float32 from per-species dicts of W1 [64,32], b1, W2 [64,64], b2, W3 [1,64], b3."""
    return np.stack([np.concatenate([np.asarray(n[k], dtype=np.float64).reshape(-1) for k in _ORDER])
                     for n in nets]).astype(np.float32)


def unpack(flat: np.ndarray):
    shapes = {"W1": (64, 32), "b1": (64,), "W2": (64, 64), "b2": (64,), "W3": (1, 64), "b3": (1,)}
    nets = []
    for s in range(2):
        off, net = 0, {}
        for k in _ORDER:
            size = int(np.prod(shapes[k]))
            net[k] = np.asarray(flat[s, off:off + size], dtype=np.float64).reshape(shapes[k])
            off += size
        nets.append(net)
    return nets


class ChargeModel:
    """Both species networks, their feature normalisation and Adam state on the device."""

    def __init__(self, ctx: Context, nets):
        self.ctx = ctx
        dev = ctx.dev
        self.params = torch.tensor(pack(nets), device=dev).contiguous()
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.norm = torch.zeros(2, 64, dtype=torch.float32, device=dev)
        self.t = 0
        self._stats3 = torch.zeros(3, dtype=torch.float64, device=dev)
        self._partial = None

    # -------------------------------------------------------------- features
    def descriptors(self, system: System, graph=None):
        g = graph if graph is not None else self.ctx.build_graph_cutoff(system, DESCRIPTOR_CUTOFF)
        return self.ctx.descriptors(system, g)

    def fit_norm(self, feats_list, species):
        stats = torch.zeros(192, dtype=torch.float64, device=self.ctx.dev)
        for f in feats_list:
            self.ctx.feature_sums(f, species, stats)
        self.ctx.feature_norm(stats, self.norm)

    # ------------------------------------------------------------- training
    def forward(self, feats, species, bf16: bool, y=None):
        y = y if y is not None else torch.empty(feats.shape[0], dtype=torch.float32, device=self.ctx.dev)
        self.ctx.mlp_forward(species, feats, self.params, self.norm, bf16, y)
        return y

    def loss_and_grad(self, feats, species, q_ref, y=None):
        """FP32 forward + loss + backward for one configuration; grad in self.grad.
        Returns the device stats3 (mean y, mean residual, loss)."""
        n = feats.shape[0]
        y = self.forward(feats, species, False, y)
        self.ctx.mlp_loss(y, q_ref, self._stats3)
        nb = (n + 63) // 64
        if self._partial is None or self._partial.numel() < nb * 2 * N_PARAMS:
            self._partial = torch.empty(nb * 2 * N_PARAMS, dtype=torch.float32, device=self.ctx.dev)
        self.ctx.mlp_backward(species, feats, self.params, self.norm, y, q_ref, self._stats3, self._partial,
                              self.grad)
        return self._stats3

    def step(self, lr: float = 1e-3):
        self.t += 1
        self.ctx.adam_step(self.params, self.grad, self.m, self.v, self.t, lr=lr)

    def train(self, feats_list, species, labels, epochs: int, lr: float = 1e-3, seed: int = 0, log=None):
        """Adam over configurations in a seeded shuffled order each epoch;
        returns the mean training loss of every epoch."""
        rng = np.random.default_rng(seed)
        y = torch.empty(feats_list[0].shape[0], dtype=torch.float32, device=self.ctx.dev)
        losses = torch.zeros(len(feats_list), dtype=torch.float64, device=self.ctx.dev)
        history = []
        for ep in range(epochs):
            for k, j in enumerate(rng.permutation(len(feats_list))):
                st = self.loss_and_grad(feats_list[j], species, labels[j], y)
                losses[k] = st[2]
                self.step(lr)
            history.append(float(losses.mean()))
            if log is not None:
                log(ep, history[-1])
        return history

    # ------------------------------------------------------------ inference
    def predict(self, feats, species, bf16: bool = True):
        """Neutral FP64 starting charges from the BF16 (or FP32) forward."""
        y = self.forward(feats, species, bf16)
        q = torch.empty(feats.shape[0], dtype=torch.float64, device=self.ctx.dev)
        self.ctx.mlp_charges(y, q)
        return q


__all__ = ["ChargeModel", "pack", "unpack", "N_PARAMS", "DESCRIPTOR_CUTOFF"]
