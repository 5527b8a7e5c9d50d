"""Regridding: a new block layout filled from the state of an old one (paper Sec. 3.3:
blocks are refined and derefined during the run; new fine blocks are prolonged and new
coarse blocks restricted from the blocks they replace, the face field by a
divergence-free prolongation after Balsara 2001).

TEST INFRASTRUCTURE ONLY.  Shares no code with the HIP path.

Rules (readings stated in the design notes):
  * Both layouts cover the same domain with the same level-0 grid; the new one may add or
    drop a finest level (its effective grid cfg["n"] then doubles or halves: the property
    `N` here).  Every new block lies, in each dimension, at the level of each old block it
    overlaps, one level finer, or one coarser, and never finer in one dimension and
    coarser in another; where it is coarser, the old blocks' boundaries fall on its cell
    faces.
  * The old state is taken at the end of a cycle (every block at the same time), with
    every ghost value filled by the ghost rules of the old layout.
  * A new cell takes its value from the old block that covers it: a copy at the same
    level; for a coarser new cell, the sqrt(-g)-weighted mean of the primitives of the
    fine cells it covers; for a finer new cell, the parent's value plus, per refined
    dimension, +-1/4 of the minmod-limited slope (the neighbours at the parent's level,
    ghosts included).
  * A new face takes its value from the old block that covers the new cell whose lower
    face it is (the cell below, for the upper face of the new block):
      - same level: a copy;
      - coarser: the mean of the fine sub-faces on it;
      - finer, on a face of the parent cell: the parent face's value plus, per refined
        transverse dimension, +-1/4 of its minmod-limited slope along that dimension (the
        neighbouring parent faces in the face's plane);
      - finer, inside the parent cell: the face average of Balsara's divergence-free
        reconstruction of the parent cell.  In the cell (coordinates x_d from the centre,
        widths D_d), B^d is quadratic in x_d and linear in the other two coordinates,
        matches on its two faces the linear distributions above (face value plus slope
        times position), and the x_d^2 coefficient follows from div B = 0:
            c_dd = -(1/2) sum_{e != d} (S_{e+}^d - S_{e-}^d) / D_e,
        with S_{e+-}^d the slope along x_d of B^e on the cell's upper and lower e faces.
        The face in the middle of the cell (x_d = 0) at transverse offsets t_e then has
            B^d = (B^d_+ + B^d_-)/2 - c_dd D_d^2/4 + sum_e t_e (S_{d+}^e + S_{d-}^e)/2.
    Since the reconstruction is divergence-free and matches the prolonged faces on the
    parent's faces, every fine cell inherits div B = 0 from its parent.
  * Conserved option (Sec. 3.3 names both forms: primitives are fast and robust,
    conserved quantities conservative): where a new cell is restricted or prolonged, the
    conserved vector U = sqrt(-g)(rho u^t, T^t_t + rho u^t, T^t_i, kappa rho u^t) of each
    old cell (from its primitives and cell-centred field) is averaged (restriction: the
    plain mean, the coordinate volumes being equal) or prolonged (the densities
    U / sqrt(-g) with +-1/4 of their minmod slopes, moved by one common amount in all
    children so that their U, the densities times the child's sqrt(-g), sum to the
    parent's U), so that the totals over
    the new cells equal the old ones; the new cell's field is the mean of its new faces;
    the primitives follow from the inversion (started from the primitive form's value),
    then the floors, as after an update.
"""
from __future__ import annotations

import math

import numpy as np

import oracle
from oracle.amr import AmrGrid


def _minmod(a, b):
    if a > 0.0 and b > 0.0:
        return min(a, b)
    if a < 0.0 and b < 0.0:
        return max(a, b)
    return 0.0


def _covering(blocks, Lmax, lam, gcell):
    """index of the block containing the cell gcell (indices at levels lam)"""
    f = [gcell[d] << (Lmax[d] - lam[d]) for d in range(3)]
    for n, b in enumerate(blocks):
        s = [Lmax[d] - b["lev"][d] for d in range(3)]
        if all((b["org"][d] << s[d]) <= f[d] < ((b["org"][d] + b["n"][d]) << s[d]) for d in range(3)):
            return n
    raise ValueError(f"cell {gcell} at levels {lam} is not covered by the old layout")


def _relation(old_b, lam):
    r = [lam[d] - old_b["lev"][d] for d in range(3)]
    if max(abs(x) for x in r) > 1 or (max(r) > 0 and min(r) < 0):
        raise ValueError(f"new levels {lam} against old {old_b['lev']}: not a one-level change")
    return r


class Regrid:
    """the new layout's state from an old AmrGrid at the end of a cycle"""

    def __init__(self, old: AmrGrid, new_blocks, conserved=False):
        self.old = old
        self.conserved = conserved
        self.cfg = old.cfg
        self.g = old.g
        self.new = [dict(b, lev=tuple(int(x) for x in b.get("lev", (0, 0, 0)))) for b in new_blocks]
        lm = tuple(max(b["lev"][d] for b in self.new) for d in range(3))
        # cells are located at the finer of the two layouts' finest levels; the new layout
        # may add or drop a finest level (its effective grid doubles or halves)
        self.Lmax = tuple(max(lm[d], old.Lmax[d]) for d in range(3))
        self.Lnew = lm
        self.N = tuple((old.N[d] >> old.Lmax[d]) << lm[d] for d in range(3))
        # the old state at the cycle's end, every ghost filled from it
        for i in range(len(old.blocks)):
            old.Pold[i] = old.P[i].copy()
            old.Bold[i] = old.B[i].copy()
        self.pads = [old.patch(i, "pred", 0) for i in range(len(old.blocks))]

    # ------------------------------------------------------------------ helpers
    def _loc(self, ob, gidx):
        """padded local index tuple (k, j, i) in old block ob of global indices (x1, x2, x3)
        at ob's levels"""
        o = self.old.blocks[ob]["org"]
        g = self.g
        return (g + gidx[2] - o[2], g + gidx[1] - o[1], g + gidx[0] - o[0])

    def _dx(self, ob):
        return self.old.bdx[ob]

    # ------------------------------------------------------------------ cells
    def cell(self, lam, gc):
        ob = _covering(self.old.blocks, self.Lmax, lam, gc)
        r = _relation(self.old.blocks[ob], lam)
        VP = self.pads[ob][0]
        if max(r) == 0 and min(r) == 0:
            return VP[(slice(None),) + self._loc(ob, gc)].copy()
        if max(r) <= 0:
            # coarser: sqrt(-g)-weighted mean of the covered fine cells (k, j, i order)
            o = self.old.blocks[ob]["org"]
            W = self.old.gdet[ob]
            subs = [range(2) if r[d] < 0 else range(1) for d in range(3)]
            num = np.zeros(5)
            den = 0.0
            for ok in subs[2]:
                for oj in subs[1]:
                    for oi in subs[0]:
                        f = [(gc[d] << (-r[d])) + (oi, oj, ok)[d] for d in range(3)]
                        w = W[f[1] - o[1], f[0] - o[0]]
                        num = num + w * VP[(slice(None),) + self._loc(ob, f)]
                        den = den + w
            return num / den
        # finer: parent plus limited slopes
        pc = [gc[d] >> r[d] for d in range(3)]
        c0 = VP[(slice(None),) + self._loc(ob, pc)]
        val = c0.copy()
        for d in range(3):
            if not r[d]:
                continue
            e = [0, 0, 0]
            e[d] = 1
            cm = VP[(slice(None),) + self._loc(ob, [pc[x] - e[x] for x in range(3)])]
            cp = VP[(slice(None),) + self._loc(ob, [pc[x] + e[x] for x in range(3)])]
            t = 0.25 if gc[d] & 1 else -0.25
            for v in range(5):
                val[v] = val[v] + t * _minmod(c0[v] - cm[v], cp[v] - c0[v])
        return val

    # ------------------------------------------------------------------ conserved form
    def _x2(self, x2):
        """x2 of a ghost cell beyond the polar axis, mirrored (its geometry)"""
        lo, hi = self.cfg["xlo"][1], self.cfg["xhi"][1]
        if self.cfg["bc"][2] == oracle.BC_POLAR:
            if x2 < lo:
                return 2.0 * lo - x2
            if x2 > hi:
                return 2.0 * hi - x2
        return x2

    def _cons_old(self, ob, gidx):
        """U of the old cell gidx of block ob (padded state, ghosts included) and its
        sqrt(-g)"""
        VP, VB = self.pads[ob]
        loc = self._loc(ob, gidx)
        dx = self._dx(ob)
        x1 = self.cfg["xlo"][0] + (gidx[0] + 0.5) * dx[0]
        x2 = self._x2(self.cfg["xlo"][1] + (gidx[1] + 0.5) * dx[1])
        gcov, gcon, gdet, alpha, _ = oracle.geom_point(self.cfg, x1, x2)
        B = []
        for d in range(3):
            hi = list(loc)
            hi[2 - d] += 1
            B.append(0.5 * (VB[(d,) + loc] + VB[(d,) + tuple(hi)]) / gdet)
        U = oracle.prim_to_flux(VP[(slice(None),) + loc], B, gcov, gcon, gdet, alpha,
                                self.cfg["gam"], 0)
        return U, gdet

    def _gdet_new(self, lam, gc):
        c = self.cfg
        dx = [(c["xhi"][d] - c["xlo"][d]) / (self.N[d] >> (self.Lnew[d] - lam[d])) for d in range(2)]
        x1 = c["xlo"][0] + (gc[0] + 0.5) * dx[0]
        x2 = self._x2(c["xlo"][1] + (gc[1] + 0.5) * dx[1])
        return oracle.geom_point(c, x1, x2)[2]

    def _cons_cell(self, lam, gc, ob, r):
        """U of a restricted new cell (the mean of the covered cells' U: the coordinate
        volumes are equal) or of a prolonged one: the densities per unit sqrt(-g),
        q = U / sqrt(-g), of the parent plus +-1/4 of their minmod slopes per refined
        dimension, moved by one common amount in all children of the parent so that
        their U (q times the child's sqrt(-g)) sum to the parent's U times their number"""
        if max(r) <= 0:
            subs = [range(2) if r[d] < 0 else range(1) for d in range(3)]
            acc = np.zeros(9)
            cnt = 0
            for ok in subs[2]:
                for oj in subs[1]:
                    for oi in subs[0]:
                        f = [(gc[d] << (-r[d])) + (oi, oj, ok)[d] for d in range(3)]
                        acc = acc + self._cons_old(ob, f)[0]
                        cnt += 1
            return acc * (1.0 / cnt)
        pc = [gc[d] >> r[d] for d in range(3)]
        U0, g0 = self._cons_old(ob, pc)
        q0 = U0 / g0
        slope = np.zeros((3, 9))
        for d in range(3):
            if not r[d]:
                continue
            e = [0, 0, 0]
            e[d] = 1
            Um, gm = self._cons_old(ob, [pc[x] - e[x] for x in range(3)])
            Up, gp = self._cons_old(ob, [pc[x] + e[x] for x in range(3)])
            qm, qp = Um / gm, Up / gp
            for v in range(9):
                slope[d, v] = _minmod(q0[v] - qm[v], qp[v] - q0[v])

        def child(cell):
            q = q0.copy()
            for d in range(3):
                if r[d]:
                    q = q + (0.25 if cell[d] & 1 else -0.25) * slope[d]
            return self._gdet_new(lam, cell) * q

        # the children of the parent, k outermost, i innermost: their densities move by
        # one common amount dq so that they sum to the parent's U times their number
        subs = [range(2) if r[d] else range(1) for d in range(3)]
        acc = np.zeros(9)
        gsum = 0.0
        cnt = 0
        for ok in subs[2]:
            for oj in subs[1]:
                for oi in subs[0]:
                    cell = [(pc[d] << r[d]) + (oi, oj, ok)[d] for d in range(3)]
                    acc = acc + child(cell)
                    gsum = gsum + self._gdet_new(lam, cell)
                    cnt += 1
        dq = (cnt * U0 - acc) / gsum
        return child(list(gc)) + self._gdet_new(lam, list(gc)) * dq

    def _invert_new(self, lam, gc, U, Bnew, guess):
        """primitives of a new cell from its conserved vector and new faces: the inversion,
        then the floors (as after an update)"""
        c = self.cfg
        dx = [(c["xhi"][d] - c["xlo"][d]) / (self.N[d] >> (self.Lnew[d] - lam[d])) for d in range(3)]
        x1 = c["xlo"][0] + (gc[0] + 0.5) * dx[0]
        x2 = c["xlo"][1] + (gc[1] + 0.5) * dx[1]
        gcov, gcon, gdet, alpha, _ = oracle.geom_point(c, x1, x2)
        U = U.copy()
        B = [0.0, 0.0, 0.0]
        for d in range(3):
            U[5 + d] = 0.5 * (Bnew[d][0] + Bnew[d][1])
            B[d] = U[5 + d] / gdet
        P, tier, _ = oracle.cons2prim(U, gcov, gcon, gdet, alpha, c["gam"], guess, guess,
                                      c.get("tol", 1e-12), c.get("maxit", 50))
        r = math.exp(x1) if c["coords"] == 1 else 1.0
        rho_fl = c.get("rho_fl_c", 0.0) * r ** c.get("rho_fl_p", 0.0)
        u_fl = c.get("u_fl_c", 0.0) * r ** c.get("u_fl_p", 0.0)
        P, _ = oracle.floors(c.get("floor_frame", oracle.FLOOR_FIXED), P, B, gcov, gcon, gdet,
                             alpha, c["gam"], rho_fl, u_fl, c.get("bsq_rho_max", 1e300),
                             c.get("bsq_u_max", 1e300), c.get("gamma_max", 1e150),
                             c.get("tol", 1e-12), c.get("maxit", 50))
        return P, tier

    # ------------------------------------------------------------------ faces
    def _face_slope(self, ob, d, fidx, e):
        """minmod slope along x_e (per parent cell) of the B^d faces at old global face
        index fidx (normal index in d, cell indices in the others)"""
        VB = self.pads[ob][1]
        step = [0, 0, 0]
        step[e] = 1
        c = VB[(d,) + self._loc(ob, fidx)]
        m = VB[(d,) + self._loc(ob, [fidx[x] - step[x] for x in range(3)])]
        p = VB[(d,) + self._loc(ob, [fidx[x] + step[x] for x in range(3)])]
        return _minmod(c - m, p - c)

    def face(self, lam, d, gf, top):
        """B^d on the new face gf (normal index in d) of a new block; top: the face is the
        block's upper face in d (its owner is the cell below)"""
        gc = list(gf)
        if top:
            gc[d] -= 1
        ob = _covering(self.old.blocks, self.Lmax, lam, gc)
        r = _relation(self.old.blocks[ob], lam)
        VB = self.pads[ob][1]
        if max(r) == 0 and min(r) == 0:
            return VB[(d,) + self._loc(ob, gf)]
        if max(r) <= 0:
            subs = [range(1) if (x == d or r[x] == 0) else range(2) for x in range(3)]
            acc = 0.0
            cnt = 0
            for ok in subs[2]:
                for oj in subs[1]:
                    for oi in subs[0]:
                        f = [(gf[x] << (-r[x])) + (oi, oj, ok)[x] for x in range(3)]
                        acc = acc + VB[(d,) + self._loc(ob, f)]
                        cnt += 1
            return acc * (1.0 / cnt)
        # finer
        pc = [gf[x] >> r[x] for x in range(3)]               # parent cell (transverse)
        t = [0.0, 0.0, 0.0]
        for x in range(3):
            if x != d and r[x]:
                t[x] = 0.25 if gf[x] & 1 else -0.25
        tr = [x for x in range(3) if x != d]
        if r[d] == 0 or gf[d] % 2 == 0:
            F = list(pc)
            F[d] = gf[d] >> r[d]
            val = VB[(d,) + self._loc(ob, F)]
            for e in tr:
                if r[e]:
                    val = val + t[e] * self._face_slope(ob, d, F, e)
            return val
        # inside the parent cell C (normal index gf[d] >> 1): Balsara's reconstruction
        C = list(pc)
        lo = list(C)
        hi = list(C)
        hi[d] += 1
        bm, bp = VB[(d,) + self._loc(ob, lo)], VB[(d,) + self._loc(ob, hi)]
        dx = self._dx(ob)
        val = 0.5 * (bm + bp)
        for e in tr:
            # c_dd part from the B^e faces' slopes along x_d (slopes per parent cell:
            # S = slope / D_d, so D_d^2/8 (S_+ - S_-)/D_e = D_d/(8 D_e) (s_+ - s_-))
            em = list(C)
            ep = list(C)
            ep[e] += 1
            s_lo = self._face_slope(ob, e, em, d)
            s_hi = self._face_slope(ob, e, ep, d)
            val = val + dx[d] / (8.0 * dx[e]) * (s_hi - s_lo)
        for e in tr:
            if r[e]:
                val = val + t[e] * 0.5 * (self._face_slope(ob, d, lo, e) + self._face_slope(ob, d, hi, e))
        return val

    # ------------------------------------------------------------------ blocks
    def states(self):
        out = []
        self.tiers = [0] * 5
        for b in self.new:
            lam, o, n = b["lev"], b["org"], b["n"]
            Bs = []
            for d in range(3):
                shp = [n[x] + (1 if x == d else 0) for x in range(3)]
                A = np.zeros((shp[2], shp[1], shp[0]))
                for k in range(shp[2]):
                    for j in range(shp[1]):
                        for i in range(shp[0]):
                            loc = (i, j, k)
                            A[k, j, i] = self.face(lam, d, (o[0] + i, o[1] + j, o[2] + k),
                                                   loc[d] == n[d])
                Bs.append(A)
            P = np.zeros((5, n[2], n[1], n[0]))
            for k in range(n[2]):
                for j in range(n[1]):
                    for i in range(n[0]):
                        gc = (o[0] + i, o[1] + j, o[2] + k)
                        val = self.cell(lam, gc)
                        if self.conserved:
                            ob = _covering(self.old.blocks, self.Lmax, lam, gc)
                            r = _relation(self.old.blocks[ob], lam)
                            if max(r) != 0 or min(r) != 0:
                                U = self._cons_cell(lam, gc, ob, r)
                                Bn = [(Bs[0][k, j, i], Bs[0][k, j, i + 1]),
                                      (Bs[1][k, j, i], Bs[1][k, j + 1, i]),
                                      (Bs[2][k, j, i], Bs[2][k + 1, j, i])]
                                val, tier = self._invert_new(lam, gc, U, Bn, val)
                                self.tiers[tier] += 1
                        P[:, k, j, i] = val
            out.append((P, Bs[0], Bs[1], Bs[2]))
        return out


def regrid(old: AmrGrid, new_blocks, conserved=False):
    """per-block interior states of the new layout (P, B1, B2, B3 as AmrGrid.set_blocks
    takes them); conserved: restrict and prolong the conserved vector, then invert"""
    return Regrid(old, new_blocks, conserved).states()
