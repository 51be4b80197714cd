"""Per-atom descriptors and the per-species charge MLP (oracle, FP64).

The learned starting guess for the self-consistent charges predicts each
atom's net Mulliken electron charge from its environment (the charge vector
n of SI section D); the plain SCC loop stays the fallback.  Definitions:

* descriptor G[I, s*16 + k] = sum over atoms J != I of species s with
  r_IJ < 5 A of exp(-(r - c_k)^2 / (2 * 0.3^2)) * (cos(pi r / 5) + 1) / 2,
  c_k = 0.8 + k * 3.2/15, k = 0..15 (minimum image);
* features standardised by per-species training mean and std;
* one network per central species: 32 -> 64 -> 64 -> 1 with SiLU,
  y = W3 silu(W2 silu(W1 x + b1) + b2) + b3;
* prediction q = y - mean(y) over the atoms of a configuration (neutrality);
* loss = mean over atoms of (q - q_ref)^2; Adam (1e-3, 0.9, 0.999, 1e-8).

Pins: gradients vs central finite differences for every parameter class;
a two-atom descriptor by hand (tests/test_oracle_learned.py).
"""
from __future__ import annotations

import math

import numpy as np

N_RADIAL = 16
R_CUT = 5.0
WIDTH = 0.3
CENTRES = 0.8 + np.arange(N_RADIAL) * (3.2 / 15.0)


def descriptors(pos: np.ndarray, species: np.ndarray, L: float) -> np.ndarray:
    """[N, 32] radial symmetry functions split by neighbour species (brute force)."""
    n = pos.shape[0]
    inv_L = 1.0 / L
    out = np.zeros((n, 2 * N_RADIAL))
    for i in range(n):
        d = pos - pos[i]
        d = d - L * np.rint(d * inv_L)
        r = np.sqrt((d * d).sum(axis=1))
        m = (r < R_CUT) & (np.arange(n) != i)
        rr = r[m]
        fc = 0.5 * (np.cos(np.pi * rr / R_CUT) + 1.0)
        g = np.exp(-((rr[:, None] - CENTRES[None, :]) ** 2) / (2 * WIDTH * WIDTH)) * fc[:, None]
        sp = species[m]
        for s in (0, 1):
            out[i, s * N_RADIAL:(s + 1) * N_RADIAL] = g[sp == s].sum(axis=0)
    return out


def silu(x):
    return x / (1.0 + np.exp(-x))


def dsilu(x):
    s = 1.0 / (1.0 + np.exp(-x))
    return s * (1.0 + x * (1.0 - s))


def standardise_stats(feats, species):
    """Per-species mean and std of the features (std floored at 1e-6)."""
    stats = []
    for s in (0, 1):
        f = feats[species == s]
        stats.append((f.mean(axis=0), np.maximum(f.std(axis=0), 1e-6)))
    return stats


def forward(nets, stats, feats, species):
    """Raw outputs y [N] and the cache for backprop."""
    y = np.zeros(feats.shape[0])
    cache = []
    for s in (0, 1):
        idx = np.nonzero(species == s)[0]
        mu, sd = stats[s]
        x = (feats[idx] - mu) / sd
        net = nets[s]
        z1 = x @ net["W1"].T + net["b1"]
        a1 = silu(z1)
        z2 = a1 @ net["W2"].T + net["b2"]
        a2 = silu(z2)
        y[idx] = a2 @ net["W3"][0] + net["b3"][0]
        cache.append((idx, x, z1, a1, z2, a2))
    return y, cache


def predict(nets, stats, feats, species):
    y, _ = forward(nets, stats, feats, species)
    return y - y.mean()


def loss_and_grads(nets, stats, feats, species, q_ref):
    """MSE of the neutral prediction and gradients for every parameter."""
    y, cache = forward(nets, stats, feats, species)
    n = y.shape[0]
    q = y - y.mean()
    r = q - q_ref
    loss = float(np.mean(r * r))
    # dL/dy_i = 2/N (r_i - mean(r))
    gy = 2.0 / n * (r - r.mean())
    grads = []
    for s in (0, 1):
        idx, x, z1, a1, z2, a2 = cache[s]
        net = nets[s]
        g = gy[idx]
        gW3 = (g[:, None] * a2).sum(axis=0)[None, :]
        gb3 = np.array([g.sum()])
        d2 = (g[:, None] * net["W3"][0][None, :]) * dsilu(z2)
        gW2 = d2.T @ a1
        gb2 = d2.sum(axis=0)
        d1 = (d2 @ net["W2"]) * dsilu(z1)
        gW1 = d1.T @ x
        gb1 = d1.sum(axis=0)
        grads.append({"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2, "W3": gW3, "b3": gb3})
    return loss, grads


class Adam:
    def __init__(self, nets, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [{k: np.zeros_like(v) for k, v in n.items()} for n in nets]
        self.v = [{k: np.zeros_like(v) for k, v in n.items()} for n in nets]
        self.t = 0

    def step(self, nets, grads):
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        for s in (0, 1):
            for k in nets[s]:
                g = grads[s][k]
                self.m[s][k] = self.b1 * self.m[s][k] + (1 - self.b1) * g
                self.v[s][k] = self.b2 * self.v[s][k] + (1 - self.b2) * g * g
                mh = self.m[s][k] / c1
                vh = self.v[s][k] / c2
                nets[s][k] = nets[s][k] - self.lr * mh / (np.sqrt(vh) + self.eps)
