"""Learned first guess of the inversion: training-set construction and training driver.

The training pairs are conserved states with the primitive states they came from:
cells of simulation snapshots (primitives as evolved, conserved vectors recomputed from
them on the device) plus synthetic states spanning wider density, magnetisation and
Lorentz-factor ranges at the same metrics.  Features, targets, normalisation, forward,
backward and the Adam update all run in libgrmhd.so; PyTorch holds the buffers and draws
the batch indices.
"""
from __future__ import annotations

import math

import numpy as np

from . import grmhd

SIZES = (8, 64, 64, 64, 2)


def init_params(seed=7, device="cuda"):
    """seeded initial master parameters in the library layout (W1 b1 W2 b2 W3 b3 W4 b4)"""
    import torch

    rng = np.random.default_rng(seed)
    parts = []
    for a, b in zip(SIZES[:-1], SIZES[1:]):
        parts.append(rng.normal(0.0, 1.0 / math.sqrt(a), (a, b)).ravel())
        parts.append(np.zeros(b))
    flat = np.concatenate(parts).astype(np.float32)
    return torch.from_numpy(flat).to(device)


def synthetic_states(geom, n, seed=11, gam=4.0 / 3.0):
    """primitive states with log-normal density (sigma 3), u/rho log-uniform in
    [1e-3, 10], Lorentz factor log-uniform in [1, 20], plasma beta log-uniform in
    [1e-2, 1e3] and isotropic directions, at the metrics of n random columns of geom
    [15][m] (device).  Returns device tensors P[5][n], B[3][n], geom[15][n]."""
    import torch

    rng = np.random.default_rng(seed)
    m = geom.shape[1]
    pick = torch.from_numpy(rng.integers(0, m, n)).to(geom.device)
    G = geom[:, pick].contiguous()
    g = G.cpu().numpy()
    g11, g13, g22, g33 = g[3], g[4], g[5], g[6]

    def norm_dir():
        v = rng.normal(size=(3, n))
        q = g11 * v[0] ** 2 + 2 * g13 * v[0] * v[2] + g22 * v[1] ** 2 + g33 * v[2] ** 2
        return v / np.sqrt(q)

    rho = np.exp(rng.normal(0.0, 3.0, n))
    u = rho * 10.0 ** rng.uniform(-3.0, 1.0, n)
    lorentz = 10.0 ** rng.uniform(0.0, math.log10(20.0), n)
    ut = norm_dir() * np.sqrt(lorentz ** 2 - 1.0)
    beta = 10.0 ** rng.uniform(-2.0, 3.0, n)
    B = norm_dir() * np.sqrt(2.0 * (gam - 1.0) * u / beta)
    P = np.vstack([rho, u, ut])
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(geom.device)
    return t(P), t(B), G


def pairs(P, B, geom, gam):
    """(X, Y) raw features/targets of states on the device, non-finite rows dropped"""
    U = grmhd.prim2cons_batch(P, B, geom, gam)
    X, Y, ok = grmhd.mlp_dataset(U, P, geom, gam)
    keep = ok.bool()
    return X[keep].contiguous(), Y[keep].contiguous()


def build_dataset(chunks, gam=4.0 / 3.0):
    """chunks: list of (P, B, geom) device tensors.  Returns normalised X, Y and the
    norm vector (feature means, stds, target means, stds) as 20 floats."""
    import torch

    xs, ys = [], []
    for P, B, G in chunks:
        X, Y = pairs(P, B, G, gam)
        xs.append(X)
        ys.append(Y)
    X = torch.cat(xs).contiguous()
    Y = torch.cat(ys).contiguous()
    xm, xsd = grmhd.mlp_normalize(X)
    ym, ysd = grmhd.mlp_normalize(Y)
    norm = torch.cat([xm, xsd, ym, ysd]).contiguous()
    return X, Y, norm


def train(X, Y, steps=2000, batch=4096, lr=1e-3, seed=7, log_every=0):
    """Adam with a cosine learning-rate schedule over `steps` batches; returns the
    trainer and the sampled losses"""
    import torch

    trainer = grmhd.MLPTrainer(init_params(seed, X.device), batch=batch)
    n = X.shape[0]
    # every step's batch rows drawn up front on the host (seeded), one upload
    rows = np.random.default_rng(seed).integers(0, n, size=(steps, batch), dtype=np.int32)
    rows = torch.from_numpy(rows).to(X.device)
    losses = []
    for s in range(steps):
        idx = rows[s]
        rate = 0.5 * lr * (1.0 + math.cos(math.pi * s / steps))
        trainer.step(X, Y, idx, rate)
        if log_every and (s % log_every == 0 or s == steps - 1):
            losses.append((s, float(trainer.loss.item())))
    return trainer, losses
