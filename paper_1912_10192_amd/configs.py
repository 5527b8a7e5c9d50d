"""Workload definitions (plain data).

Each workload is a dict with the grid, scheme and floor parameters of one run:
    coords   0 Minkowski Cartesian, 1 Kerr-Schild log-spherical (x1 = ln r, x2 = theta, x3 = phi)
    n        effective cells (N1, N2, N3);  block (b1, b2, b3) cells per block
    ng       ghost layers (2 for PLM, 3 for PPM)
    recon    0 PLM with MC limiter, 1 PPM;  riemann 0 LLF, 1 HLLE
    bc       x1lo, x1hi, x2lo, x2hi, x3lo, x3hi: 0 outflow, 1 polar, 2 periodic
Floors follow rho >= rho_fl_c r^rho_fl_p, u >= u_fl_c r^u_fl_p, b^2/rho <= bsq_rho_max,
b^2/u <= bsq_u_max, Lorentz factor <= gamma_max.
"""
from __future__ import annotations

import math

KS_TORUS_BASE = dict(
    coords=1, a=0.9375, gam=4.0 / 3.0,
    xlo=(math.log(1.2), 0.0, 0.0), xhi=(math.log(50.0), math.pi, 2.0 * math.pi),
    bc=(0, 0, 1, 1, 2, 2), courant=0.8,
    rho_fl_c=1e-6, rho_fl_p=-1.5, u_fl_c=1e-9, u_fl_p=-10.0 / 3.0,
    bsq_rho_max=50.0, bsq_u_max=750.0, gamma_max=50.0, tol=1e-12, maxit=50,
)

# one 64x32x32 block, PLM-MC + LLF, 10 steps
TORUS_TINY = dict(KS_TORUS_BASE, name="torus-64x32x32-plm-llf", n=(64, 32, 32),
                  block=(64, 32, 32), ng=2, recon=0, riemann=0, steps=10)

# one GPU's share of a uniform grid: 256x128x128 in 128 blocks of 32^3, PPM + HLLE
TORUS_UNIFORM = dict(KS_TORUS_BASE, name="torus-256x128x128-b32-ppm-hlle", n=(256, 128, 128),
                     block=(32, 32, 32), ng=3, recon=1, riemann=1, steps=200)

TORUS_INIT = dict(a=0.9375, rin_grid=1.2, rout_grid=50.0, rin=6.0, rmax=12.0,
                  gam=4.0 / 3.0, beta=100.0, amp=0.02, seed=20191221,
                  rho_fl_c=1e-6, rho_fl_p=-1.5, u_fl_c=1e-9, u_fl_p=-10.0 / 3.0)


def scaled(cfg: dict, n, block=None, **kw) -> dict:
    """the same workload on another grid size"""
    out = dict(cfg, n=tuple(n), block=tuple(block if block is not None else n))
    out.update(kw)
    out["name"] = f"{cfg['name'].split('-')[0]}-{n[0]}x{n[1]}x{n[2]}"
    return out


def polar_smr_blocks(n, b1, lats=None):
    """Block layout of a log-spherical grid with coarser polar bands (paper Sec. 3.4,
    external mesh refinement toward the poles), for an effective grid n = (N1, N2, N3):
      equatorial band, theta rows [N2/4, 3 N2/4): full resolution (levels 1, 1, 2)
      mid-latitude bands, [N2/8, N2/4) and mirror: half resolution in every dimension
                                                    (levels 0, 0, 1)
      polar caps, [0, N2/8) and mirror: half resolution in r and theta, a quarter in
                                        phi (levels 0, 0, 0)
    Blocks span b1 effective cells in x1 in every band (so x1 block faces line up and a
    time level per x1 column applies to all bands); lats[i] is the time level of x1
    column i."""
    N1, N2, N3 = n
    nb1 = N1 // b1
    lats = list(lats) if lats is not None else [0] * nb1
    out = []

    def add(lev, org2, n2, nb3, n3):
        f1 = b1 >> (1 - lev[0])
        for k in range(nb3):
            for i in range(nb1):
                out.append(dict(org=(i * f1, org2, k * n3), n=(f1, n2, n3), lev=lev, lat=lats[i]))

    r = N2 // 16            # rows of a polar cap / mid band at their (half) theta level
    add((0, 0, 0), 0, r, 2, N3 // 8)                           # cap, theta < pi/8
    add((0, 0, 1), r, r, 4, N3 // 8)                           # mid band
    for j in range(2):                                         # equatorial band
        add((1, 1, 2), N2 // 4 + j * (N2 // 4), N2 // 4, 4, N3 // 4)
    add((0, 0, 1), N2 // 2 - 2 * r, r, 4, N3 // 8)             # mid band, southern
    add((0, 0, 0), N2 // 2 - r, r, 2, N3 // 8)                 # cap, southern
    return out


# Batched refinement + local time stepping: effective 512x256x256 with coarser polar
# bands (polar_smr_blocks, 64-cell x1 block columns) and 4 time levels by the inner
# radius of each x1 column (r < 2.4 -> 0, < 4.8 -> 1, < 9.6 -> 2, else 3)
TORUS_AMR_LAT = dict(KS_TORUS_BASE, name="torus-eff512x256x256-polar-smr-lat4", n=(512, 256, 256),
                     block=(64, 64, 64), ng=3, recon=1, riemann=1, cycles=25,
                     lat_edges=(2.4, 4.8, 9.6))
