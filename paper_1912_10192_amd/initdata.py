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


# ------------------------------------------------------------------ off-centre explosion

EXPLOSION_INIT = dict(a=0.9375, gam=4.0 / 3.0, centre=(3.0, 0.0, 10.0), r_s=2.0,
                      rho_in=1e-4, p_in=3e-5, rho_out=1e-6, p_out=3e-8, width=0.25,
                      magnetised=False, beta_max=10.0)


def explosion_state(n, xlo, xhi, a=0.9375, gam=4.0 / 3.0, centre=(3.0, 0.0, 10.0), r_s=2.0,
                    rho_in=1e-4, p_in=3e-5, rho_out=1e-6, p_out=3e-8, width=0.25,
                    magnetised=False, beta_max=10.0):
    """The off-centre spherical explosion of the paper's validation (Sec. 7.3) on a
    log-spherical Kerr-Schild grid n over [xlo, xhi]: gas at rest (utilde = 0) with
    rho = rho_in, p = p_in inside a sphere of radius r_s about `centre` (flat spherical
    embedding x = r sin th cos ph, ...), falling exponentially to the ambient rho_out,
    p_out over `width` outside it; optionally threaded by the field of the vector
    potential A_phi = max(r_s - d, 0) (d the distance from the centre) taken at cell
    corners, scaled so that max p_g / max (b^2/2) = beta_max.  Returns (P, B1, B2, B3)."""
    N1, N2, N3 = n
    dx = [(xhi[d] - xlo[d]) / n[d] for d in range(3)]

    def dist(x1, x2, x3):
        r = np.exp(x1)
        X = r * np.sin(x2) * np.cos(x3) - centre[0]
        Y = r * np.sin(x2) * np.sin(x3) - centre[1]
        Z = r * np.cos(x2) - centre[2]
        return np.sqrt(X * X + Y * Y + Z * Z)

    c = [xlo[d] + (np.arange(n[d]) + 0.5) * dx[d] for d in range(3)]
    X3, X2, X1 = np.meshgrid(c[2], c[1], c[0], indexing="ij")     # [N3][N2][N1]
    dd = dist(X1, X2, X3)
    s = np.exp(-np.maximum(dd - r_s, 0.0) / width)
    P = np.zeros((5, N3, N2, N1))
    P[0] = rho_out + (rho_in - rho_out) * s
    P[1] = (p_out + (p_in - p_out) * s) / (gam - 1.0)
    B1 = np.zeros((N3, N2, N1 + 1))
    B2 = np.zeros((N3, N2 + 1, N1))
    B3 = np.zeros((N3 + 1, N2, N1))
    if magnetised:
        # A_3 on the x3-directed edges (x1, x2 faces; x3 centres): B1 = d2 A3, B2 = -d1 A3
        f1 = xlo[0] + np.arange(N1 + 1) * dx[0]
        f2 = xlo[1] + np.arange(N2 + 1) * dx[1]
        E3, E2, E1 = np.meshgrid(c[2], f2, f1, indexing="ij")       # [N3][N2+1][N1+1]
        A = np.maximum(r_s - dist(E1, E2, E3), 0.0)
        b1 = (A[:, 1:, :] - A[:, :-1, :]) / dx[1]
        b2 = -(A[:, :, 1:] - A[:, :, :-1]) / dx[0]
        R, TH = np.exp(X1), X2
        sig = R * R + a * a * np.cos(TH) ** 2
        gdet = R * sig * np.sin(TH)
        Bc = np.stack([0.5 * (b1[..., 1:] + b1[..., :-1]) / gdet,
                       0.5 * (b2[:, 1:, :] + b2[:, :-1, :]) / gdet, np.zeros_like(R)])
        bsq = _bsq(P, Bc, R, TH, a)
        pmax = float(np.max((gam - 1.0) * P[1]))
        bmax = float(np.max(0.5 * bsq))
        scale = math.sqrt(pmax / (beta_max * bmax)) if bmax > 0.0 else 0.0
        B1 = scale * b1
        B2 = scale * b2
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


# --------------------------------------------------------------------- tilted thin disk

DISK_INIT = dict(a=0.9375, gam=4.0 / 3.0, tilt=math.pi / 4, h_r=0.03, r_in=6.0, r_out=200.0,
                 beta=10.0, amp=0.01, seed=20191221, rho_fl_c=1e-6, rho_fl_p=-1.5,
                 u_fl_c=1e-9, u_fl_p=-10.0 / 3.0)


def _smoothstep(x):
    x = np.clip(x, 0.0, 1.0)
    return x * x * (3.0 - 2.0 * x)


class Disk:
    """A thin disk in a frame tilted by `tilt` about the x axis of the hole's frame
    (flat spherical positions x = r sin(th) cos(ph), ...):
      rho = (R'/r_in)^(-3/2) exp(-z'^2 / (2 H^2)) T(R'),  H = h_r R',
    T a C1 taper from 0 to 1 over [r_in, 1.1 r_in] and back to 0 over [0.9 r_out, r_out],
    normalised to a midplane maximum of 1; p = rho h_r^2 / R'; Keplerian rotation
    v = R'^(-1/2) about z'; a toroidal field about z' from the vector potential
    A = A_R'(R', z') R'-hat, A_R' = sqrt(2 p_mid(R') / beta0) sqrt(pi) H erf(z' / (2H)),
    whose curl is the toroidal field sqrt(2 p / beta0) (in flat space)."""

    def __init__(self, a, gam, tilt, h_r, r_in, r_out, **_):
        self.a, self.gam, self.h_r, self.r_in, self.r_out = a, gam, h_r, r_in, r_out
        self.ct, self.st = math.cos(tilt), math.sin(tilt)
        R = np.linspace(r_in, r_out, 200001)
        self.norm = float(np.max(self._mid_raw(R)))

    def _taper(self, R):
        return (_smoothstep((R - self.r_in) / (0.1 * self.r_in))
                * _smoothstep((self.r_out - R) / (0.1 * self.r_out)))

    def _mid_raw(self, R):
        return (np.maximum(R, 1e-300) / self.r_in) ** -1.5 * self._taper(R)

    @staticmethod
    def _trig(th, ph):
        s, c = np.sin(th), np.cos(th)
        s = np.where((th == 0.0) | (th == math.pi), 0.0, s)     # exactly on the axis
        c = np.where(th == 0.0, 1.0, np.where(th == math.pi, -1.0, c))
        return s, c, np.sin(ph), np.cos(ph)

    def frame(self, r, th, ph):
        """hole-frame Cartesian position and disk-frame (x', y', z')"""
        s, c, sp, cp = self._trig(th, ph)
        x, y, z = r * s * cp, r * s * sp, r * c
        return (x, y, z), (x, self.ct * y + self.st * z, -self.st * y + self.ct * z)

    def rho_mid(self, R):
        return self._mid_raw(R) / self.norm

    def state(self, r, th, ph):
        """disk density, internal energy (gamma-law p = rho h_r^2 / R') and the hole-frame
        Cartesian Keplerian velocity at points"""
        (x, y, z), (xp, yp, zp) = self.frame(r, th, ph)
        R = np.sqrt(xp * xp + yp * yp)
        H = self.h_r * np.maximum(R, 1e-300)
        rho = self.rho_mid(R) * np.exp(-zp * zp / (2.0 * H * H))
        u = rho * self.h_r ** 2 / np.maximum(R, 1e-300) / (self.gam - 1.0)
        v = np.maximum(R, 1e-300) ** -0.5
        vxp, vyp = -v * yp / np.maximum(R, 1e-300), v * xp / np.maximum(R, 1e-300)
        # back to the hole's frame (z' has no velocity)
        vx, vy, vz = vxp, self.ct * vyp, self.st * vyp
        return rho, u, (vx, vy, vz)

    def potential(self, r, th, ph, beta0=1.0):
        """hole-frame Cartesian vector potential A = A_R' R'-hat"""
        (x, y, z), (xp, yp, zp) = self.frame(r, th, ph)
        R = np.sqrt(xp * xp + yp * yp)
        Rs = np.maximum(R, 1e-300)
        H = self.h_r * Rs
        pmid = self.rho_mid(R) * self.h_r ** 2 / Rs
        from scipy.special import erf
        AR = np.sqrt(2.0 * pmid / beta0) * math.sqrt(math.pi) * H * erf(zp / (2.0 * H))
        axp, ayp = AR * xp / Rs, AR * yp / Rs
        return axp, self.ct * ayp, self.st * ayp


def _edge_integrals(disk, cfg, b, lmax):
    """line integrals of the covariant vector potential along every edge of block b
    (internal coordinates x1 = ln r, x2 = theta, x3 = phi), each the sum of the midpoint
    values times length of the finest-level sub-edges it contains, so that a coarse
    edge's integral is the sum of its fine sub-edges'.  Returns I1 [n3+1][n2+1][n1],
    I2 [n3+1][n2][n1+1], I3 [n3][n2+1][n1+1]."""
    N = cfg["n"]
    lev, o, n = b["lev"], b["org"], b["n"]
    f = [1 << (lmax[d] - lev[d]) for d in range(3)]
    dxf = [(cfg["xhi"][d] - cfg["xlo"][d]) / N[d] for d in range(3)]

    def coords(axis):
        # finest-level sample coordinates: sub-edge midpoints along `axis`, nodes across;
        # broadcast shapes [x3][x2][x1]
        out = []
        for d in range(3):
            if d == axis:
                c = (o[d] * f[d] + np.arange(n[d] * f[d]) + 0.5) * dxf[d]
            else:
                c = (o[d] + np.arange(n[d] + 1)) * f[d] * dxf[d]
            shape = [1, 1, 1]
            shape[2 - d] = -1
            out.append((cfg["xlo"][d] + c).reshape(shape))
        return out

    res = []
    for axis in range(3):
        x1, x2, x3 = coords(axis)
        r = np.exp(x1)
        s, c, sp, cp = Disk._trig(x2, x3)
        Ax, Ay, Az = disk.potential(r, x2, x3)
        if axis == 0:     # d x / d ln r = position
            Ai = Ax * (r * s * cp) + Ay * (r * s * sp) + Az * (r * c)
        elif axis == 1:   # d x / d theta
            Ai = Ax * (r * c * cp) + Ay * (r * c * sp) - Az * (r * s)
        else:             # d x / d phi
            Ai = -Ax * (r * s * sp) + Ay * (r * s * cp)
        Ai = np.broadcast_to(Ai, (x3.size, x2.size, x1.size)) * dxf[axis]
        shape = list(Ai.shape)
        ax = 2 - axis
        shape[ax:ax + 1] = [n[axis], f[axis]]
        res.append(Ai.reshape(shape).sum(axis=ax + 1))
    return res


def _disk_block(args):
    """one block of disk_block_states before the field is scaled: (P, B1, B2, B3, max p_g,
    max b^2/2)"""
    cfg, b, lmax, p = args
    disk = Disk(**p)
    N = cfg["n"]
    lev, o, n = b["lev"], b["org"], b["n"]
    Nl = [N[d] >> (lmax[d] - lev[d]) for d in range(3)]
    dx = [(cfg["xhi"][d] - cfg["xlo"][d]) / Nl[d] for d in range(3)]
    x1 = (cfg["xlo"][0] + (o[0] + np.arange(n[0]) + 0.5) * dx[0])[None, None, :]
    x2 = (cfg["xlo"][1] + (o[1] + np.arange(n[1]) + 0.5) * dx[1])[None, :, None]
    x3 = (cfg["xlo"][2] + (o[2] + np.arange(n[2]) + 0.5) * dx[2])[:, None, None]
    shp = (n[2], n[1], n[0])
    r = np.exp(x1)
    rho_d, u_d, (vx, vy, vz) = disk.state(r, x2, x3)
    rho_a = p["rho_fl_c"] * r ** p["rho_fl_p"]
    u_a = p["u_fl_c"] * r ** p["u_fl_p"]
    ins = np.broadcast_to(rho_d > rho_a, shp)
    s, c, sp, cp = Disk._trig(x2, x3)
    vr = vx * s * cp + vy * s * sp + vz * c
    vth = vx * c * cp + vy * c * sp - vz * s
    vph = -vx * sp + vy * cp
    ut1 = np.where(ins, vr / r, 0.0)
    ut2 = np.where(ins, vth / r, 0.0)
    ut3 = np.where(ins, vph / np.maximum(r * s, 1e-300), 0.0)
    rho = np.where(ins, rho_d, rho_a)
    uu = np.where(ins, np.maximum(u_d, u_a), u_a)
    if p["amp"] != 0.0:
        kk, jj, ii = np.meshgrid(o[2] + np.arange(n[2]), o[1] + np.arange(n[1]),
                                 o[0] + np.arange(n[0]), indexing="ij")
        code = (lev[0] * 16 + lev[1]) * 16 + lev[2]
        gidx = (((np.uint64(code) * np.uint64(Nl[2]) + kk.astype(np.uint64)) * np.uint64(Nl[1])
                 + jj.astype(np.uint64)) * np.uint64(Nl[0]) + ii.astype(np.uint64))
        xi = uniform01(p["seed"], gidx)
        rho = np.where(ins, rho * (1.0 + p["amp"] * (2.0 * xi - 1.0)), rho)
    P = np.stack([rho, uu, ut1, ut2, ut3])
    I1, I2, I3 = _edge_integrals(disk, cfg, b, lmax)
    a12, a13, a23 = dx[0] * dx[1], dx[0] * dx[2], dx[1] * dx[2]
    B1 = (I3[:, 1:, :] - I3[:, :-1, :]) / a23 - (I2[1:, :, :] - I2[:-1, :, :]) / a23
    B2 = (I1[1:, :, :] - I1[:-1, :, :]) / a13 - (I3[:, :, 1:] - I3[:, :, :-1]) / a13
    B3 = (I2[:, :, 1:] - I2[:, :, :-1]) / a12 - (I1[:, 1:, :] - I1[:, :-1, :]) / a12
    # field strength of this block (cell-centred coordinate field, Kerr-Schild b^2)
    th = np.broadcast_to(x2[0], (n[1], n[0]))
    rr = np.broadcast_to(r[0], (n[1], n[0]))
    gdet = rr * (rr * rr + p["a"] ** 2 * np.cos(th) ** 2) * np.sin(th)
    Bc = np.stack([0.5 * (B1[..., 1:] + B1[..., :-1]), 0.5 * (B2[:, 1:] + B2[:, :-1]),
                   0.5 * (B3[1:] + B3[:-1])]) / gdet[None, None]
    bsq = np.stack([_bsq(P[:, k], Bc[:, k], rr, th, p["a"]) for k in range(n[2])])
    return P, B1, B2, B3, float(np.max((p["gam"] - 1.0) * uu)), float(np.max(0.5 * bsq))


def disk_block_states(cfg, blocks, init=None, procs=1):
    """per-block interior arrays of the tilted disk (prims at each block's cell centres,
    face fields from the edge integrals of the vector potential, scaled to max p_g /
    max(b^2/2) = beta over all blocks), with the atmosphere rho = rho_fl r^rho_fl_p,
    u_g = u_fl r^u_fl_p outside the disk and a seeded density perturbation rho (1 + amp
    (2 xi - 1)) in disk cells, xi keyed by the cell's index on its block's level grid
    and the level.  procs > 1 builds the blocks in that many worker processes (the
    result does not depend on it)."""
    p = dict(DISK_INIT, **(init or {}))
    lmax = [max(b["lev"][d] for b in blocks) for d in range(3)]
    work = [(cfg, b, lmax, p) for b in blocks]
    if procs > 1:
        import multiprocessing as mp

        with mp.get_context("spawn").Pool(procs) as pool:
            out = pool.map(_disk_block, work, chunksize=max(1, len(work) // (8 * procs)))
    else:
        out = [_disk_block(w) for w in work]
    pmax = max(o[4] for o in out)
    bmax = max(o[5] for o in out)
    scale = math.sqrt(pmax / (p["beta"] * bmax)) if bmax > 0.0 else 0.0
    return [(P, scale * B1, scale * B2, scale * B3) for P, B1, B2, B3, _, _ in out]
