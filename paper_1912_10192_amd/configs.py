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


def amr_lat_blocks(n, shapes=None, lat_edges=(2.4, 4.8, 9.6), xlo=None, xhi=None):
    """Block layout of the batched refinement + local time stepping workload (paper Sec.
    3.3, 3.4 external refinement toward the poles, 3.5) for an effective log-spherical
    grid n = (N1, N2, N3) at the finest level of each dimension (levels 1, 1, 2):
      equatorial band, theta rows [N2/4, 3 N2/4): full resolution; x1 [0, N1/4) in
          blocks shapes["eq_in"], x1 [N1/4, N1) in blocks shapes["eq_out"];
      mid-latitude bands [N2/8, N2/4) and mirror: half resolution in every dimension
          (levels 0, 0, 1), blocks shapes["mid"];
      polar caps [0, N2/8) and mirror: half resolution in r and theta and a quarter in
          phi (levels 0, 0, 0), blocks shapes["cap"].
    Every refinement jump is 2:1.  Default shapes (effective 512x256x256): 32x16x16
    (512 blocks) and 64x32x32 (192) in the equatorial band, 32x16x16 (128) in the mid
    bands, 16x8x8 (512) in the caps: 1344 blocks, 18,350,080 cells.  The time level of
    a block is set by the radius of its inner x1 face (level = number of lat_edges at or
    below it), then lowered where needed so that blocks that touch differ by at most one
    level."""
    import math

    N1, N2, N3 = n
    if shapes is None:
        shapes = dict(eq_in=(N1 // 16, N2 // 16, N3 // 16), eq_out=(N1 // 8, N2 // 8, N3 // 8),
                      mid=(N1 // 16, N2 // 16, N3 // 16), cap=(N1 // 32, N2 // 32, N3 // 32))
    xlo = xlo if xlo is not None else KS_TORUS_BASE["xlo"][0]
    xhi = xhi if xhi is not None else KS_TORUS_BASE["xhi"][0]
    out = []

    def tile(lev, ext, rows, x1r, shape):
        b1, b2, b3 = shape
        for k in range(0, ext[2], b3):
            for j in range(rows[0], rows[1], b2):
                for i in range(x1r[0], x1r[1], b1):
                    out.append(dict(org=(i, j, k), n=(b1, b2, b3), lev=lev, lat=0))

    # caps, mid bands and equator from the north pole down (levels' extents in cells)
    ext0 = (N1 // 2, N2 // 2, N3 // 4)
    ext1 = (N1 // 2, N2 // 2, N3 // 2)
    ext2 = (N1, N2, N3)
    tile((0, 0, 0), ext0, (0, N2 // 16), (0, N1 // 2), shapes["cap"])
    tile((0, 0, 1), ext1, (N2 // 16, N2 // 8), (0, N1 // 2), shapes["mid"])
    tile((1, 1, 2), ext2, (N2 // 4, 3 * N2 // 4), (0, N1 // 4), shapes["eq_in"])
    tile((1, 1, 2), ext2, (N2 // 4, 3 * N2 // 4), (N1 // 4, N1), shapes["eq_out"])
    tile((0, 0, 1), ext1, (3 * N2 // 8, 7 * N2 // 16), (0, N1 // 2), shapes["mid"])
    tile((0, 0, 0), ext0, (7 * N2 // 16, N2 // 2), (0, N1 // 2), shapes["cap"])
    # time levels by inner radius
    lmax = (1, 1, 2)
    dx1 = (xhi - xlo) / N1
    for b in out:
        i_eff = b["org"][0] << (lmax[0] - b["lev"][0])
        r = math.exp(xlo + i_eff * dx1)
        b["lat"] = sum(1 for e in lat_edges if r >= e)
    # boxes in effective cells; touching blocks (phi periodic) differ by at most one level
    import numpy as np
    lo = np.array([[b["org"][d] << (lmax[d] - b["lev"][d]) for d in range(3)] for b in out])
    hi = lo + np.array([[b["n"][d] << (lmax[d] - b["lev"][d]) for d in range(3)] for b in out])
    touch = np.ones((len(out), len(out)), dtype=bool)
    for d, Nd in enumerate(n):
        a0, a1 = lo[:, d][:, None], hi[:, d][:, None]
        b0, b1 = lo[:, d][None, :], hi[:, d][None, :]
        t = (a0 <= b1) & (b0 <= a1)
        if d == 2:
            t |= (a0 == 0) & (b1 == Nd) | (b0 == 0) & (a1 == Nd)
        touch &= t
    lat = np.array([b["lat"] for b in out])
    while True:
        lim = np.where(touch, lat[None, :] + 1, 1 << 30).min(axis=1)
        new = np.minimum(lat, lim)
        if np.array_equal(new, lat):
            break
        lat = new
    for b, l in zip(out, lat):
        b["lat"] = int(l)
    return out


# Batched refinement + local time stepping as specified: effective 512x256x256 in 1344
# blocks of 64x32x32, 32x16x16 and 16x8x8 (amr_lat_blocks), phi halved per level toward
# each pole (3 levels), 4 time levels by radius, 25 cycles
TORUS_AMR3 = dict(KS_TORUS_BASE, name="torus-eff512x256x256-amr-lat4-1344blocks", n=(512, 256, 256),
                  block=(64, 32, 32), ng=3, recon=1, riemann=1, cycles=25,
                  lat_edges=(2.4, 4.8, 9.6))
