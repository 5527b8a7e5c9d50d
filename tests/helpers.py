"""Shared test helpers: layout conversions and synthetic Minkowski states."""
from __future__ import annotations

import numpy as np


def pad_global(cfg, P, B1, B2, B3):
    """global interior arrays -> oracle padded arrays (ng below, ng+1 above)"""
    g = cfg["ng"]
    N1, N2, N3 = cfg["n"]
    shp = (N3 + 2 * g + 1, N2 + 2 * g + 1, N1 + 2 * g + 1)
    Pp = np.zeros((5,) + shp)
    Bp = np.zeros((3,) + shp)
    Pp[:, g:g + N3, g:g + N2, g:g + N1] = P
    Bp[0, g:g + N3, g:g + N2, g:g + N1 + 1] = B1
    Bp[1, g:g + N3, g:g + N2 + 1, g:g + N1] = B2
    Bp[2, g:g + N3 + 1, g:g + N2, g:g + N1] = B3
    return Pp, Bp


def unpad_global(cfg, Pp, Bp):
    g = cfg["ng"]
    N1, N2, N3 = cfg["n"]
    P = Pp[:, g:g + N3, g:g + N2, g:g + N1].copy()
    B1 = Bp[0, g:g + N3, g:g + N2, g:g + N1 + 1].copy()
    B2 = Bp[1, g:g + N3, g:g + N2 + 1, g:g + N1].copy()
    B3 = Bp[2, g:g + N3 + 1, g:g + N2, g:g + N1].copy()
    return P, B1, B2, B3


def mink_cfg(n, recon=1, riemann=1, ng=3, L=None, **kw):
    L = L if L is not None else tuple(float(x) / n[0] for x in n)
    cfg = dict(coords=0, n=tuple(n), block=tuple(n), ng=ng, recon=recon, riemann=riemann,
               bc=(2, 2, 2, 2, 2, 2), gam=4.0 / 3.0, a=0.0, xlo=(0.0, 0.0, 0.0), xhi=tuple(L),
               courant=0.8, rho_fl_c=0.0, rho_fl_p=0.0, u_fl_c=0.0, u_fl_p=0.0,
               bsq_rho_max=1e300, bsq_u_max=1e300, gamma_max=1e150, tol=1e-12, maxit=50)
    cfg.update(kw)
    return cfg


def random_periodic_state(n, seed=1, amp=0.1, bamp=0.3, vamp=0.3, dx=None):
    """smooth random periodic state with a divergence-free face field built from a
    random edge vector potential (discrete curl with the grid spacing dx, default cubic
    cells of size 1/n[0] as in mink_cfg, so div B = 0 to round-off)."""
    rng = np.random.default_rng(seed)
    N1, N2, N3 = n
    k, j, i = np.meshgrid(np.arange(N3), np.arange(N2), np.arange(N1), indexing="ij")
    x, y, z = (i + 0.5) / N1, (j + 0.5) / N2, (k + 0.5) / N3

    def smooth(scale):
        a = rng.normal(size=4)
        return scale * (a[0] * np.sin(2 * np.pi * (x + a[1])) * np.cos(2 * np.pi * (y + a[2]))
                        + 0.5 * np.sin(2 * np.pi * (z + a[3]) + 2 * np.pi * x))

    P = np.empty((5, N3, N2, N1))
    P[0] = 1.0 + amp * smooth(1.0)
    P[1] = 1.0 + amp * smooth(1.0)
    for c in range(3):
        P[2 + c] = vamp * smooth(1.0)
    # edge potentials A1(i, j-1/2, k-1/2), A2(i-1/2, j, k-1/2), A3(i-1/2, j-1/2, k), periodic
    A = [bamp * smooth(1.0) / (2 * np.pi) for _ in range(3)]
    dx = dx if dx is not None else (1.0 / N1, 1.0 / N1, 1.0 / N1)
    roll = np.roll
    # face fields on the periodic interior (upper boundary faces equal lower ones)
    b1 = (roll(A[2], -1, axis=1) - A[2]) / dx[1] - (roll(A[1], -1, axis=0) - A[1]) / dx[2]
    b2 = (roll(A[0], -1, axis=0) - A[0]) / dx[2] - (roll(A[2], -1, axis=2) - A[2]) / dx[0]
    b3 = (roll(A[1], -1, axis=2) - A[1]) / dx[0] - (roll(A[0], -1, axis=1) - A[0]) / dx[1]
    B1 = np.concatenate([b1, b1[:, :, :1]], axis=2)
    B2 = np.concatenate([b2, b2[:, :1, :]], axis=1)
    B3 = np.concatenate([b3, b3[:1, :, :]], axis=0)
    return P, B1 + 0.5, B2 + 0.3, B3 - 0.2
