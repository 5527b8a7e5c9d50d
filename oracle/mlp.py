"""Oracle of the learned inversion guess: a small MLP written with plain numpy.

TEST INFRASTRUCTURE ONLY (imported by tests and the CPU-baseline leg of the benchmark,
never by the product path).  Shares no code with the HIP kernels.

The network maps eight normalised features of a conserved state to two normalised
targets from which the Newton inversion of Sec. 2.6 starts:
    features  log D, asinh(tau/D), log1p(S^2/D^2), log1p(B^2/D), log1p((S.B)^2/D^3),
              lapse, adiabatic index, sqrt(det gamma_ij)
    targets   log Gamma, log(W/D) with W = (rho + u + p) Gamma^2
with D = alpha rho u^t, S_i = alpha T^t_i, tau = -(Q.n) - D (Q.n = (Q_t - beta^i Q_i)/alpha),
S^2 = gamma^ij S_i S_j, B^i the lapse-scaled field (alpha B^i).  Layers 8 -> 64 -> 64 ->
64 -> 2 with tanh on the hidden layers; mean-squared-error loss; Adam.  "bf16" mode
rounds weights and layer inputs to bfloat16 (round to nearest even) and accumulates in
float32, as the MFMA kernels do.
"""
from __future__ import annotations

import numpy as np

SIZES = (8, 64, 64, 64, 2)


def bf16(x):
    """round float32/64 values to bfloat16 (nearest even), returned as float32"""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    out = r.astype(np.uint32).view(np.float32)
    return np.where(np.isnan(a), a, out)


def features(U, gcov, gcon, gdet, alpha, gam):
    """raw (unnormalised) features of conserved states U[9][n] with metric arrays
    gcov[4][4][n], gcon[4][4][n], gdet[n], alpha[n]"""
    ig = 1.0 / gdet
    D = alpha * U[0] * ig
    Qt = alpha * U[1] * ig - D
    Q = alpha * U[2:5] * ig
    Bc = alpha * U[5:8] * ig
    beta = alpha ** 2 * gcon[0, 1:]
    Qdotn = (Qt - np.einsum("in,in->n", beta, Q)) / alpha
    gamcon = gcon[1:, 1:] + np.einsum("in,jn->ijn", beta, beta) / alpha ** 2
    S2 = np.einsum("ijn,in,jn->n", gamcon, Q, Q)
    B2 = np.einsum("ijn,in,jn->n", gcov[1:, 1:], Bc, Bc)
    SB = np.einsum("in,in->n", Q, Bc)
    tau = -Qdotn - D
    sqrt_gamma = gdet / alpha
    return np.stack([np.log(D), np.arcsinh(tau / D), np.log1p(S2 / D ** 2), np.log1p(B2 / D),
                     np.log1p(SB ** 2 / D ** 3), alpha, np.full_like(D, gam), sqrt_gamma])


def targets(P, gcov, gam):
    """raw targets log Gamma, log(W/D) of primitive states P[5][n]"""
    ut = P[2:5]
    qsq = np.einsum("ijn,in,jn->n", gcov[1:, 1:], ut, ut)
    G = np.sqrt(1.0 + qsq)
    W = (P[0] + gam * P[1]) * G * G
    D = P[0] * G
    return np.stack([np.log(G), np.log(W / D)])


def init_params(seed=7):
    rng = np.random.default_rng(seed)
    params = []
    for a, b in zip(SIZES[:-1], SIZES[1:]):
        params.append(rng.normal(0.0, 1.0 / np.sqrt(a), (a, b)))
        params.append(np.zeros(b))
    return params


def forward(params, x, mode="f64"):
    """x[n][8] -> (y[n][2], cache).  mode 'f64' or 'bf16'."""
    acts = [x]
    pre = []
    h = x
    nl = len(params) // 2
    for l in range(nl):
        W, b = params[2 * l], params[2 * l + 1]
        if mode == "bf16":
            z = bf16(h).astype(np.float32) @ bf16(W).astype(np.float32) + b.astype(np.float32)
        else:
            z = h @ W + b
        pre.append(z)
        h = np.tanh(z) if l < nl - 1 else z
        acts.append(h)
    return h, (acts, pre)


def loss_and_grads(params, x, y, mode="f64"):
    """mean-squared error over batch and outputs, and its gradients"""
    out, (acts, pre) = forward(params, x, mode)
    n = x.shape[0]
    diff = out - y
    loss = float(np.mean(diff ** 2))
    g = 2.0 * diff / diff.size
    grads = [None] * len(params)
    nl = len(params) // 2
    for l in range(nl - 1, -1, -1):
        W = params[2 * l]
        h = acts[l]
        if mode == "bf16":
            # every product of the network takes bfloat16 operands (FP32 sums): the
            # backward signal g is rounded like the activations and weights
            gb = bf16(g).astype(np.float32)
            grads[2 * l] = bf16(h).astype(np.float32).T @ gb
            grads[2 * l + 1] = g.sum(axis=0)
            gh = gb @ bf16(W).astype(np.float32).T
        else:
            grads[2 * l] = h.T @ g
            grads[2 * l + 1] = g.sum(axis=0)
            gh = g @ W.T
        if l > 0:
            g = gh * (1.0 - acts[l] ** 2)
    return loss, grads


def adam_step(params, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """one Adam update in place; state = (t, m list, v list)"""
    t, m, v = state
    t += 1
    for i, (p, g) in enumerate(zip(params, grads)):
        m[i] = b1 * m[i] + (1 - b1) * g
        v[i] = b2 * v[i] + (1 - b2) * g * g
        mh = m[i] / (1 - b1 ** t)
        vh = v[i] / (1 - b2 ** t)
        p -= lr * mh / (np.sqrt(vh) + eps)
    return (t, m, v)
