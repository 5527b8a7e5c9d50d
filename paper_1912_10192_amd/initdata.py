"""Seeded synthetic initial data shared by the oracle tests and the GPU path.

This module only builds INPUTS: a Fishbone-Moncrief torus in a Kerr-Schild
log-spherical grid, a single-loop poloidal field from a corner vector potential, a
floor atmosphere and a counter-based random perturbation.  It holds none of the
update's arithmetic (no fluxes, no inversion, no time stepping).

Output layout ("global interior" arrays, x1 fastest):
    P  [5][N3][N2][N1]      rho, u_g, utilde^1, utilde^2, utilde^3 at cell centres
    B1 [N3][N2][N1+1]       sqrt(-g) B^1 on x1 faces (index i = face at x1_i)
    B2 [N3][N2+1][N1]       sqrt(-g) B^2 on x2 faces
    B3 [N3+1][N2][N1]       sqrt(-g) B^3 on x3 faces (zero for this field)
"""
from __future__ import annotations

import math

import numpy as np

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x):
    """SplitMix64 output function (Steele, Lea & Flood 2014) on uint64 arrays."""
    z = (np.asarray(x, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15)) & _M64
    z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _M64
    z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _M64
    return z ^ (z >> np.uint64(31))


def uniform01(seed: int, index) -> np.ndarray:
    """Counter-based U[0,1): top 53 bits of splitmix64(seed XOR index) / 2^53."""
    with np.errstate(over="ignore"):
        z = splitmix64(np.uint64(seed) ^ np.asarray(index, dtype=np.uint64))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


# --------------------------------------------------------------------------- torus

def fm_ell(a: float, rmax: float) -> float:
    """u^t u_phi of the prograde circular equatorial geodesic at rmax (Bardeen, Press &
    Teukolsky 1972 energy and angular momentum, Boyer-Lindquist inverse metric)."""
    r = rmax
    sr = math.sqrt(r)
    den = r ** 0.75 * math.sqrt(r ** 1.5 - 3.0 * sr + 2.0 * a)
    u_t = -(r ** 1.5 - 2.0 * sr + a) / den
    u_phi = (r * r - 2.0 * a * sr + a * a) / den
    sig = r * r
    delta = r * r - 2.0 * r + a * a
    big_a = (r * r + a * a) ** 2 - a * a * delta
    gtt = -big_a / (sig * delta)
    gtp = -2.0 * a * r / (sig * delta)
    ut = gtt * u_t + gtp * u_phi
    return ut * u_phi


def fm_lnh(r, th, a, ell):
    """ln of the specific enthalpy of the constant-(u^t u_phi) torus, up to a constant:
    ln u^t - ell * Omega written in Boyer-Lindquist quantities."""
    r = np.asarray(r, dtype=float)
    s = np.sin(th)
    c = np.cos(th)
    sig = r * r + a * a * c * c
    delta = r * r - 2.0 * r + a * a
    big_a = (r * r + a * a) ** 2 - delta * a * a * s * s
    with np.errstate(divide="ignore", invalid="ignore"):
        d = np.sqrt(1.0 + 4.0 * ell * ell * sig * sig * delta / (big_a * big_a * s * s))
        return 0.5 * np.log((1.0 + d) / (sig * delta / big_a)) - 0.5 * d - 2.0 * a * ell * r / big_a


def fm_velocity(r, th, a, ell):
    """Boyer-Lindquist u^t, u^phi of the torus flow (equal to the Kerr-Schild ones, as u^r = 0)."""
    s = np.sin(th)
    c = np.cos(th)
    sig = r * r + a * a * c * c
    delta = r * r - 2.0 * r + a * a
    big_a = (r * r + a * a) ** 2 - delta * a * a * s * s
    usq = 0.5 * (np.sqrt(1.0 + 4.0 * ell * ell * sig * sig * delta / (big_a * big_a * s * s)) - 1.0)
    uz = np.sqrt(usq)                                     # ZAMO-frame u^(phi)
    gam = np.sqrt(1.0 + usq)
    ut = gam * np.sqrt(big_a / (sig * delta))
    uphi = 2.0 * a * r * gam / np.sqrt(big_a * sig * delta) + np.sqrt(sig / big_a) * uz / s
    return ut, uphi


class Torus:
    def __init__(self, a=0.9375, rin=6.0, rmax=12.0, gam=4.0 / 3.0, kappa=1e-3):
        self.a, self.rin, self.rmax, self.gam, self.kappa = a, rin, rmax, gam, kappa
        self.ell = fm_ell(a, rmax)
        self.lnh_in = float(fm_lnh(rin, 0.5 * math.pi, a, self.ell))
        self.rho_max = float(self._rho_raw(np.array(rmax), np.array(0.5 * math.pi))[0])

    def inside(self, r, th):
        lnh = fm_lnh(r, th, self.a, self.ell) - self.lnh_in
        return (np.asarray(r) >= self.rin) & np.isfinite(lnh) & (lnh > 0.0), lnh

    def _rho_raw(self, r, th):
        ins, lnh = self.inside(r, th)
        h = np.exp(np.where(ins, lnh, 0.0))
        g = self.gam
        base = np.maximum((h - 1.0) * (g - 1.0) / (self.kappa * g), 0.0)
        return np.where(ins, base ** (1.0 / (g - 1.0)), 0.0), ins

    def rho_u(self, r, th):
        """normalised density (max 1 at rmax on the equator) and internal energy"""
        rho, ins = self._rho_raw(r, th)
        u = self.kappa * rho ** self.gam / (self.gam - 1.0)
        return rho / self.rho_max, u / self.rho_max, ins


# --------------------------------------------------------- Kerr-Schild for b^2 only

def _ks_internal(r, th, a):
    """covariant internal metric (x1 = ln r) and the inverse entries needed for
    utilde -> u^mu; used here only to normalise the field strength."""
    s = np.sin(th)
    c = np.cos(th)
    sig = r * r + a * a * c * c
    q = 2.0 * r / sig
    z = np.zeros_like(r)
    g = np.empty(r.shape + (4, 4))
    g[...] = 0.0
    g[..., 0, 0] = -(1.0 - q)
    g[..., 0, 1] = g[..., 1, 0] = q * r
    g[..., 0, 3] = g[..., 3, 0] = -a * q * s * s
    g[..., 1, 1] = (1.0 + q) * r * r
    g[..., 1, 3] = g[..., 3, 1] = -a * s * s * (1.0 + q) * r
    g[..., 2, 2] = sig
    g[..., 3, 3] = s * s * (sig + a * a * s * s * (1.0 + q))
    gtt_con = -(1.0 + q)
    gt1_con = 2.0 / sig
    gdet = r * sig * s
    return g, gtt_con, gt1_con + z, gdet


def _bsq(P, Bc, r, th, a):
    g, gtt, gt1, _ = _ks_internal(r, th, a)
    ut_ = P[2:5]
    qsq = np.einsum("i...,j...,...ij->...", ut_, ut_, g[..., 1:, 1:])
    gamma = np.sqrt(1.0 + qsq)
    alpha = 1.0 / np.sqrt(-gtt)
    beta1 = alpha * alpha * gt1
    ucon = np.stack([gamma / alpha, ut_[0] - gamma * beta1 / alpha, ut_[1], ut_[2]])
    ucov = np.einsum("...ij,j...->i...", g, ucon)
    bt = np.einsum("i...,i...->...", Bc, ucov[1:])
    bcon = np.stack([bt] + [(Bc[i] + bt * ucon[i + 1]) / ucon[0] for i in range(3)])
    bcov = np.einsum("...ij,j...->i...", g, bcon)
    return np.einsum("i...,i...->...", bcon, bcov)


# ------------------------------------------------------------------ public builder

def torus_state(n, a=0.9375, rin_grid=1.2, rout_grid=50.0, rin=6.0, rmax=12.0,
                gam=4.0 / 3.0, beta=100.0, amp=0.02, seed=20191221,
                rho_fl_c=1e-6, rho_fl_p=-1.5, u_fl_c=1e-9, u_fl_p=-10.0 / 3.0):
    """FM torus + single-loop field + atmosphere + seeded u_g perturbation on an
    n = (N1, N2, N3) grid covering ln r in [ln rin_grid, ln rout_grid], theta in [0, pi],
    phi in [0, 2 pi).  Returns (P, B1, B2, B3) global interior arrays."""
    N1, N2, N3 = n
    x1lo, x1hi = math.log(rin_grid), math.log(rout_grid)
    dx1 = (x1hi - x1lo) / N1
    dx2 = math.pi / N2
    tor = Torus(a, rin, rmax, gam)
    # cell centres
    x1c = x1lo + (np.arange(N1) + 0.5) * dx1
    x2c = (np.arange(N2) + 0.5) * dx2
    R, TH = np.meshgrid(np.exp(x1c), x2c)               # [N2][N1]
    rho_t, u_t, ins = tor.rho_u(R, TH)
    ut, uphi = fm_velocity(np.where(ins, R, 10.0), np.where(ins, TH, 0.5 * math.pi), a, tor.ell)
    sig = R * R + a * a * np.cos(TH) ** 2
    ut1 = np.where(ins, 2.0 * ut / (sig + 2.0 * R), 0.0)
    ut3 = np.where(ins, uphi, 0.0)
    rho_atm = rho_fl_c * R ** rho_fl_p
    u_atm = u_fl_c * R ** u_fl_p
    rho = np.where(ins, np.maximum(rho_t, rho_atm), rho_atm)
    uu = np.where(ins, np.maximum(u_t, u_atm), u_atm)
    P2d = np.stack([rho, uu, ut1, np.zeros_like(rho), ut3])          # [5][N2][N1]
    P = np.repeat(P2d[:, None, :, :], N3, axis=1).copy()           # [5][N3][N2][N1]
    # corner vector potential A_phi = max(rho/rho_max - 0.2, 0)
    x1f = x1lo + np.arange(N1 + 1) * dx1
    x2f = np.arange(N2 + 1) * dx2
    Rf, THf = np.meshgrid(np.exp(x1f), x2f)              # [N2+1][N1+1]
    rho_c, _, _ = tor.rho_u(Rf, THf)
    A = np.maximum(rho_c - 0.2, 0.0)
    b1 = (A[1:, :] - A[:-1, :]) / dx2                    # [N2][N1+1]
    b2 = -(A[:, 1:] - A[:, :-1]) / dx1                   # [N2+1][N1]
    # normalise: max p_g / max (b^2/2) = beta over the grid
    gdet_c = R * sig * np.sin(TH)
    Bc = np.stack([0.5 * (b1[:, 1:] + b1[:, :-1]) / gdet_c,
                   0.5 * (b2[1:, :] + b2[:-1, :]) / gdet_c, np.zeros_like(R)])
    bsq = _bsq(P2d, Bc, R, TH, a)
    pmax = float(np.max((gam - 1.0) * uu))
    bmax = float(np.max(0.5 * bsq))
    scale = math.sqrt(pmax / (beta * bmax)) if bmax > 0.0 else 0.0
    B1 = np.repeat((scale * b1)[None], N3, axis=0).copy()
    B2 = np.repeat((scale * b2)[None], N3, axis=0).copy()
    B3 = np.zeros((N3 + 1, N2, N1))
    # seeded multiplicative perturbation of u_g inside the torus, keyed by the global
    # cell index so that it does not depend on the block decomposition
    if amp != 0.0:
        kk, jj, ii = np.meshgrid(np.arange(N3), np.arange(N2), np.arange(N1), indexing="ij")
        gidx = ((kk.astype(np.uint64) * np.uint64(N2) + jj.astype(np.uint64)) * np.uint64(N1)
                + ii.astype(np.uint64))
        xi = uniform01(seed, gidx)
        insk = np.broadcast_to(ins[None], (N3, N2, N1))
        P[1] = np.where(insk, P[1] * (1.0 + amp * (2.0 * xi - 1.0)), P[1])
    return P, B1, B2, B3


# --------------------------------------------------------------------------- block grids

def coarsen_state(state, r):
    """a state on a grid coarser by r[d] in {0, 1} per dimension: cell values as the mean
    of the fine cells, face fields as the mean of the fine sub-faces (so a discretely
    divergence-free field stays divergence-free).  state = global interior arrays."""
    P, B1, B2, B3 = state
    s = [1 + x for x in r]

    def mean_cells(A):
        acc = 0.0
        for ok in range(s[2]):
            for oj in range(s[1]):
                for oi in range(s[0]):
                    acc = acc + A[..., ok::s[2], oj::s[1], oi::s[0]]
        return acc / (s[0] * s[1] * s[2])

    def mean_faces(A, d):
        acc = 0.0
        cnt = 0
        offs = [range(1) if x == d else range(s[x]) for x in range(3)]
        for ok in offs[2]:
            for oj in offs[1]:
                for oi in offs[0]:
                    acc = acc + A[ok::s[2], oj::s[1], oi::s[0]]
                    cnt += 1
        return acc / cnt

    return mean_cells(P), mean_faces(B1, 0), mean_faces(B2, 1), mean_faces(B3, 2)


def block_states(state, blocks, lmax):
    """per-block interior arrays of a block grid from a state at the finest level:
    block b at levels lev takes the state coarsened to its level (one factor of two per
    level below lmax, applied level by level)"""
    cache = {tuple(lmax): state}

    def at(lev):
        lev = tuple(lev)
        if lev not in cache:
            d = max(range(3), key=lambda x: lmax[x] - lev[x])
            up = list(lev)
            r = [0, 0, 0]
            for x in range(3):
                if lev[x] < lmax[x] and lmax[x] - lev[x] == lmax[d] - lev[d]:
                    up[x] += 1
                    r[x] = 1
            cache[lev] = coarsen_state(at(up), r)
        return cache[lev]

    out = []
    for b in blocks:
        P, B1, B2, B3 = at(b.get("lev", (0, 0, 0)))
        o, n = b["org"], b["n"]
        out.append((P[:, o[2]:o[2] + n[2], o[1]:o[1] + n[1], o[0]:o[0] + n[0]].copy(),
                    B1[o[2]:o[2] + n[2], o[1]:o[1] + n[1], o[0]:o[0] + n[0] + 1].copy(),
                    B2[o[2]:o[2] + n[2], o[1]:o[1] + n[1] + 1, o[0]:o[0] + n[0]].copy(),
                    B3[o[2]:o[2] + n[2] + 1, o[1]:o[1] + n[1], o[0]:o[0] + n[0]].copy()))
    return out
