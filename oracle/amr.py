"""Static mesh refinement with local time stepping on a block grid, written plainly with
the oracle's stage.

TEST INFRASTRUCTURE ONLY.  Shares no code with the HIP path.

Blocks carry a refinement level per dimension (paper Sec. 3.3, and the per-direction
coarsening toward the poles of Sec. 3.4) and a time level (Sec. 3.5).  The effective
grid cfg["n"] is the grid at the finest level of each dimension; a block at level l in
dimension d has cells 2^(Lmax_d - l) times the effective spacing, and its origin is
counted in cells of its own level.  Rules, with the readings stated in the design notes:

  * Every block sees the whole domain at its own level (a "view"), built from every
    block's state as it stands at the viewing block's stage time (the time rules of
    local time stepping):
      - blocks at the viewing level are copied;
      - a block one level finer (in some dimensions, equal in the others) is restricted:
        cell primitives as the sqrt(-g)-weighted mean of the fine cells, face fields as
        the arithmetic mean of the fine sub-faces on the coarse face;
      - a block one level coarser is prolonged from the view at its own level (which
        includes its physical-boundary and neighbour values): child = parent +
        minmod(backward, forward difference) * (+-1/4) per refined dimension; a face
        field is prolonged the same way across its face from the coarse face that
        contains it, and a fine face that cuts a coarse cell in two takes the mean of
        the two prolonged values on the coarse faces bounding that cell;
      - the physical boundaries are then applied to the view at that level;
      - a face shared by several blocks takes the value of the viewing block if it owns
        one, else of a block at the viewing time level, then of the finest block, then of
        the block listed last (so that blocks of one time level, which evolve such a face
        side by side, read the same copy of it in every stage).
  * Time levels are independent of refinement levels and of the direction of a face
    (Sec. 3.5).  Every face and every edge shared by blocks has a dominant holder: the
    fastest holder, among those the finest, among those the lowest block index (holders
    of one time and refinement level compute the same values).  An edge counts as held by
    a block only where it lies on the block's own edge lattice (an edge of fine cells in
    the middle of a coarse face is not an edge of the coarse block).
  * Same time level: in each stage, after all fluxes and EMFs of the level are computed
    and before any update, the coarse block's fluxes on faces shared with finer blocks
    are replaced by the area mean of the fine fluxes, and every EMF of a block whose
    dominant holder is finer (at the same time level) by the dominant's EMF (the mean of
    its two sub-edges where it is finer along the edge).  After the update, the coarse
    copy of each shared face takes the mean of the fine faces.
  * Faster holder: at the end of the slower block's step (Sec. 3.5 flux correction, Sec.
    3.3 refluxing) its face fluxes on faces shared with the faster block are replaced by
    the faster side's time integral over its two steps (area-averaged where the faster
    side is finer; the coarse density itself where it is coarser), its EMFs on edges
    whose dominant holder is faster by the dominant's time integral, the faces of the
    slower block around those edges are corrected by constrained transport, shared faces
    take the faster copy (the mean of its sub-faces where it is finer; none where it is
    coarser), and every cell whose conserved state or faces changed is inverted again.
"""
from __future__ import annotations

import itertools

import numpy as np

import oracle
from oracle.lat import LatGrid

CONS_Q = (0, 1, 2, 3, 4, 5, 6, 7, 8)


def minmod(a, b):
    """0 unless both differences have one sign, else the one of smaller magnitude"""
    return np.where((a > 0) & (b > 0), np.minimum(a, b),
                    np.where((a < 0) & (b < 0), np.maximum(a, b), 0.0))


def _lev(b):
    return tuple(int(x) for x in b.get("lev", (0, 0, 0)))


class AmrGrid(LatGrid):
    def __init__(self, cfg: dict, blocks: list):
        self.cfg = dict(cfg)
        self.g = g = cfg["ng"]
        self.N = tuple(cfg["n"])
        self.blocks = [dict(b, lev=_lev(b)) for b in blocks]
        self.Lmax = tuple(max(b["lev"][d] for b in self.blocks) for d in range(3))
        self.dx = [(cfg["xhi"][d] - cfg["xlo"][d]) / self.N[d] for d in range(3)]
        self.L = max(b["lat"] for b in self.blocks) + 1
        self.vgrid = {}
        self.ctx, self.bdx, self.gdet = [], [], []
        for b in self.blocks:
            lam, o, n = b["lev"], b["org"], b["n"]
            Nl = self.nlev(lam)
            dxl = [(cfg["xhi"][d] - cfg["xlo"][d]) / Nl[d] for d in range(3)]
            bc = list(cfg["bc"])
            for d, (lo, hi) in enumerate(((0, 1), (2, 3), (4, 5))):
                assert 0 <= o[d] and o[d] + n[d] <= Nl[d], "block outside the grid"
                if o[d] != 0:
                    bc[lo] = oracle.BC_PERIODIC
                if o[d] + n[d] != Nl[d]:
                    bc[hi] = oracle.BC_PERIODIC
            xlo = tuple(cfg["xlo"][d] + o[d] * dxl[d] for d in range(3))
            xhi = tuple(cfg["xlo"][d] + (o[d] + n[d]) * dxl[d] for d in range(3))
            self.ctx.append(oracle.Grid(dict(cfg, n=tuple(n), xlo=xlo, xhi=xhi, bc=tuple(bc))))
            self.bdx.append(dxl)
            self.gdet.append(self._gdet_columns(b, dxl))
        self.P = [c.zeros()[0] for c in self.ctx]
        self.B = [c.zeros()[1] for c in self.ctx]
        self.Ps = [p.copy() for p in self.P]
        self.Bs = [b.copy() for b in self.B]
        self.Pold = [p.copy() for p in self.P]
        self.Bold = [b.copy() for b in self.B]
        self.reg_step = [dict() for _ in self.blocks]
        self.reg_pair = [dict() for _ in self.blocks]
        self.t = 0.0
        self.dt_min = 0.0
        self.steps = [0] * self.L
        self.trace = []
        self.links = self._refinement_faces()
        self.owner = self._owner_map()
        self._sync_tables()

    # ------------------------------------------------------------------ layout
    def nlev(self, lam):
        return tuple(self.N[d] >> (self.Lmax[d] - lam[d]) for d in range(3))

    def _gdet_columns(self, b, dxl):
        """sqrt(-g) at the block's interior cell centres, [n2][n1]"""
        n1, n2 = b["n"][0], b["n"][1]
        out = np.ones((n2, n1))
        if self.cfg["coords"] == 0:
            return out
        for j in range(n2):
            x2 = self.cfg["xlo"][1] + (b["org"][1] + j + 0.5) * dxl[1]
            for i in range(n1):
                x1 = self.cfg["xlo"][0] + (b["org"][0] + i + 0.5) * dxl[0]
                out[j, i] = oracle.geom_point(self.cfg, x1, x2)[2]
        return out

    def _refinement_faces(self):
        """(coarse block, fine block, d, side, lo, hi): the fine block is one level finer
        (in the dimensions of e, equal in the others) and touches the coarse block across
        its lower (side 0) or upper (side 1) d-face; lo/hi bound the shared patch in the
        coarse block's global cells of the two transverse dimensions."""
        out = []
        for c, bc in enumerate(self.blocks):
            Nc = self.nlev(bc["lev"])
            for f, bf in enumerate(self.blocks):
                e = tuple(bf["lev"][d] - bc["lev"][d] for d in range(3))
                if min(e) < 0 or max(e) > 1 or max(e) == 0:
                    continue
                lo_f = [bf["org"][d] >> e[d] for d in range(3)]
                hi_f = [(bf["org"][d] + bf["n"][d]) >> e[d] for d in range(3)]
                lo_c = list(bc["org"])
                hi_c = [bc["org"][d] + bc["n"][d] for d in range(3)]
                for d in range(3):
                    t = [x for x in range(3) if x != d]
                    if any(max(lo_f[x], lo_c[x]) >= min(hi_f[x], hi_c[x]) for x in t):
                        continue
                    per = self.cfg["bc"][2 * d] == oracle.BC_PERIODIC
                    below = hi_f[d] == lo_c[d] or (per and lo_c[d] == 0 and hi_f[d] == Nc[d])
                    above = hi_c[d] == lo_f[d] or (per and lo_f[d] == 0 and hi_c[d] == Nc[d])
                    lo = tuple(max(lo_f[x], lo_c[x]) for x in range(3))
                    hi = tuple(min(hi_f[x], hi_c[x]) for x in range(3))
                    for side, hit in ((0, below), (1, above)):
                        if hit and bc["lat"] == bf["lat"]:
                            out.append((c, f, d, side, e, lo, hi))
        return out

    def _owner_map(self):
        """block id of every cell of the effective grid"""
        N = self.N
        own = np.full((N[2], N[1], N[0]), -1, dtype=np.int64)
        for i, b in enumerate(self.blocks):
            s = [self.Lmax[d] - b["lev"][d] for d in range(3)]
            o, n = b["org"], b["n"]
            own[o[2] << s[2]:(o[2] + n[2]) << s[2], o[1] << s[1]:(o[1] + n[1]) << s[1],
                o[0] << s[0]:(o[0] + n[0]) << s[0]] = i
        return own

    def _owner(self, lam, idx):
        """the block holding cell idx (i, j, k) of the grid at levels lam; positions
        outside the grid wrap across periodic boundaries, else None (outflow, polar)"""
        N = self.nlev(lam)
        x = list(idx)
        for d in range(3):
            if 0 <= x[d] < N[d]:
                continue
            if self.cfg["bc"][2 * d] != oracle.BC_PERIODIC:
                return None
            x[d] %= N[d]
        s = [self.Lmax[d] - lam[d] for d in range(3)]
        h = int(self.owner[x[2] << s[2], x[1] << s[1], x[0] << s[0]])
        return h if h >= 0 else None

    def _local(self, D, lam, pos, kind, a=None):
        """padded local indices in block D of an element at positions pos (per dimension,
        in cells/nodes of levels lam): kind 'cell' index per dimension, 'face' normal
        dimension a (a node along a), 'edge' along a (a cell along a, nodes otherwise).
        Returns the list of D's elements covering it (several where D is finer, their
        values to be averaged), each as (K, J, I)."""
        g = self.g
        bD = self.blocks[D]
        ranges = []
        for d in range(3):
            diff = bD["lev"][d] - lam[d]
            node = (kind == "face" and d == a) or (kind == "edge" and d != a)
            if node:
                if diff >= 0:
                    vals = [pos[d] << diff]
                else:
                    assert pos[d] % 2 == 0, "a node off the coarser lattice"
                    vals = [pos[d] >> 1]
            else:
                vals = [(pos[d] << 1) + q for q in range(2)] if diff > 0 else [pos[d] >> (-diff)]
            Nd = self.nlev(bD["lev"])[d]
            per = self.cfg["bc"][2 * d] == oracle.BC_PERIODIC
            out = []
            for v in vals:
                hi = bD["org"][d] + bD["n"][d] + (1 if node else 0)
                cands = [v, v - Nd, v + Nd] if per else [v]
                got = [w for w in cands if bD["org"][d] <= w < hi]
                assert got, "element outside its holder"
                out.append(got[0] - bD["org"][d] + g)
            ranges.append(out)
        return [(k, j, i) for k in ranges[2] for j in ranges[1] for i in ranges[0]]

    def _dominant(self, hs):
        """fastest, then finest, then lowest index"""
        return min(hs, key=lambda h: (self.blocks[h]["lat"], -sum(self.blocks[h]["lev"]), h))

    def _sync_tables(self):
        """Per block: the faces of its boundary shared with a faster block (reflux and
        face copy); the edges of its boundary whose finest holder at its own time level is
        finer than it (EMF replaced in each stage), and those whose dominant holder is
        faster (time-integrated EMF replaced at the end of its step)."""
        g = self.g
        nb = len(self.blocks)
        self.reflux = [[] for _ in range(nb)]     # (d, side, face (K,J,I), D, D faces)
        self.sync_edges = [[] for _ in range(nb)]  # (a, edge (K,J,I), D, D edges)
        self.stage_edges = [[] for _ in range(nb)]
        for b, bb in enumerate(self.blocks):
            lam, o, n = bb["lev"], bb["org"], bb["n"]
            N = self.nlev(lam)
            polar = self.cfg["bc"][2] == oracle.BC_POLAR
            for d in range(3):
                t = [x for x in range(3) if x != d]
                for side in (0, 1):
                    p = o[d] + (n[d] if side else 0)
                    if d == 1 and polar and (p == 0 or p == N[1]):
                        continue                     # the polar axis carries no flux
                    for c1 in range(o[t[1]], o[t[1]] + n[t[1]]):
                        for c0 in range(o[t[0]], o[t[0]] + n[t[0]]):
                            cell = [0, 0, 0]
                            cell[d] = p if side else p - 1
                            cell[t[0]], cell[t[1]] = c0, c1
                            D = self._owner(lam, cell)
                            if D is None or self.blocks[D]["lat"] >= bb["lat"]:
                                continue
                            pos = list(cell)
                            pos[d] = p
                            mine = self._local(b, lam, pos, "face", d)[0]
                            self.reflux[b].append((d, side, mine, D,
                                                   self._local(D, lam, pos, "face", d)))
            for a in range(3):
                t = [x for x in range(3) if x != a]
                for x1 in range(o[t[1]], o[t[1]] + n[t[1]] + 1):
                    for x0 in range(o[t[0]], o[t[0]] + n[t[0]] + 1):
                        on0 = x0 in (o[t[0]], o[t[0]] + n[t[0]])
                        on1 = x1 in (o[t[1]], o[t[1]] + n[t[1]])
                        if not (on0 or on1):
                            continue
                        if polar and 1 in t and (x0 if t[0] == 1 else x1) in (0, N[1]):
                            continue                 # on the axis: E1 = E3 = 0
                        for ca in range(o[a], o[a] + n[a]):
                            hs = set()
                            for q0 in (x0 - 1, x0):
                                for q1 in (x1 - 1, x1):
                                    cell = [0, 0, 0]
                                    cell[a], cell[t[0]], cell[t[1]] = ca, q0, q1
                                    h = self._owner(lam, cell)
                                    if h is None:
                                        continue
                                    hl = self.blocks[h]["lev"]
                                    if any(hl[e] < lam[e] and (x0 if e == t[0] else x1) % 2
                                           for e in t):
                                        continue     # not on the holder's edge lattice
                                    hs.add(h)
                            if not hs:
                                continue
                            pos = [0, 0, 0]
                            pos[a], pos[t[0]], pos[t[1]] = ca, x0, x1
                            mine = self._local(b, lam, pos, "edge", a)[0]
                            # in each stage the holders at this time level agree on the
                            # finest one's value; at the end of the step the faster
                            # dominant's time integral replaces it
                            same = [h for h in hs if self.blocks[h]["lat"] == bb["lat"]]
                            D = self._dominant(same)
                            if D != b and self.blocks[D]["lev"] != lam:
                                self.stage_edges[b].append(
                                    (a, mine, D, self._local(D, lam, pos, "edge", a)))
                            D = self._dominant(hs)
                            if self.blocks[D]["lat"] < bb["lat"]:
                                self.sync_edges[b].append(
                                    (a, mine, D, self._local(D, lam, pos, "edge", a)))

    def _vg(self, lam):
        if lam not in self.vgrid:
            self.vgrid[lam] = oracle.Grid(dict(self.cfg, n=self.nlev(lam)))
        return self.vgrid[lam]

    # ------------------------------------------------------------------ state
    def set_blocks(self, states):
        """states[i] = (P[5][n3][n2][n1], B1[n3][n2][n1+1], B2[n3][n2+1][n1], B3[n3+1][n2][n1])"""
        g = self.g
        for i, (P, B1, B2, B3) in enumerate(states):
            n1, n2, n3 = self.blocks[i]["n"]
            self.P[i][:, g:g + n3, g:g + n2, g:g + n1] = P
            self.B[i][0, g:g + n3, g:g + n2, g:g + n1 + 1] = B1
            self.B[i][1, g:g + n3, g:g + n2 + 1, g:g + n1] = B2
            self.B[i][2, g:g + n3 + 1, g:g + n2, g:g + n1] = B3

    def get_blocks(self):
        g = self.g
        out = []
        for i, b in enumerate(self.blocks):
            n1, n2, n3 = b["n"]
            out.append((self.P[i][:, g:g + n3, g:g + n2, g:g + n1].copy(),
                        self.B[i][0, g:g + n3, g:g + n2, g:g + n1 + 1].copy(),
                        self.B[i][1, g:g + n3, g:g + n2 + 1, g:g + n1].copy(),
                        self.B[i][2, g:g + n3 + 1, g:g + n2, g:g + n1].copy()))
        return out

    # ------------------------------------------------------------------ views
    def _put_same(self, GP, GB, n, Pn, Bn):
        g = self.g
        o, m = self.blocks[n]["org"], self.blocks[n]["n"]
        GP[:, g + o[2]:g + o[2] + m[2], g + o[1]:g + o[1] + m[1], g + o[0]:g + o[0] + m[0]] = \
            Pn[:, g:g + m[2], g:g + m[1], g:g + m[0]]
        GB[0, g + o[2]:g + o[2] + m[2], g + o[1]:g + o[1] + m[1], g + o[0]:g + o[0] + m[0] + 1] = \
            Bn[0, g:g + m[2], g:g + m[1], g:g + m[0] + 1]
        GB[1, g + o[2]:g + o[2] + m[2], g + o[1]:g + o[1] + m[1] + 1, g + o[0]:g + o[0] + m[0]] = \
            Bn[1, g:g + m[2], g:g + m[1] + 1, g:g + m[0]]
        GB[2, g + o[2]:g + o[2] + m[2] + 1, g + o[1]:g + o[1] + m[1], g + o[0]:g + o[0] + m[0]] = \
            Bn[2, g:g + m[2] + 1, g:g + m[1], g:g + m[0]]

    def _put_restrict(self, GP, GB, n, Pn, Bn, r):
        """block n, finer by r[d] in dimension d, restricted into a coarser view"""
        g = self.g
        o, m = self.blocks[n]["org"], self.blocks[n]["n"]
        oc = [o[d] >> r[d] for d in range(3)]
        mc = [m[d] >> r[d] for d in range(3)]
        s = [1 + r[d] for d in range(3)]
        Pi = Pn[:, g:g + m[2], g:g + m[1], g:g + m[0]]
        W = self.gdet[n]
        num = np.zeros((5, mc[2], mc[1], mc[0]))
        den = np.zeros((1, 1, mc[1], mc[0]))
        for ok, oj, oi in itertools.product(range(s[2]), range(s[1]), range(s[0])):
            w = W[oj::s[1], oi::s[0]][None, None]
            num = num + w * Pi[:, ok::s[2], oj::s[1], oi::s[0]]
            den = den + w
        GP[:, g + oc[2]:g + oc[2] + mc[2], g + oc[1]:g + oc[1] + mc[1], g + oc[0]:g + oc[0] + mc[0]] = num / den
        for d in range(3):
            # interior faces of the block along d: [m[d] + 1] normal, m[e] transverse
            hi = [m[x] + (1 if x == d else 0) for x in range(3)]
            F = Bn[d, g:g + hi[2], g:g + hi[1], g:g + hi[0]]
            step = [s[x] for x in range(3)]
            offs = [range(1) if x == d else range(s[x]) for x in range(3)]
            acc = 0.0
            cnt = 0
            for ok, oj, oi in itertools.product(offs[2], offs[1], offs[0]):
                acc = acc + F[ok::step[2], oj::step[1], oi::step[0]]
                cnt += 1
            val = acc * (1.0 / cnt)
            shp = [mc[x] + (1 if x == d else 0) for x in range(3)]
            GB[d, g + oc[2]:g + oc[2] + shp[2], g + oc[1]:g + oc[1] + shp[1],
               g + oc[0]:g + oc[0] + shp[0]] = val

    def _put_prolong(self, GP, GB, n, VP, VB, r):
        """block n, coarser by r[d] in dimension d, prolonged into a finer view from the
        view VP/VB at its own level"""
        g = self.g
        o, m = self.blocks[n]["org"], self.blocks[n]["n"]
        of = [o[d] << r[d] for d in range(3)]
        mf = [m[d] << r[d] for d in range(3)]
        # cells: coarse padded index and the +-1/4 weight of every fine cell
        cidx = [g + o[d] + (np.arange(mf[d]) >> r[d]) for d in range(3)]
        sgn = [np.where(np.arange(mf[d]) & 1, 0.25, -0.25) for d in range(3)]

        def at(A, dk, dj, di):
            return A[..., (cidx[2] + dk)[:, None, None], (cidx[1] + dj)[None, :, None],
                     (cidx[0] + di)[None, None, :]]

        c0 = at(VP, 0, 0, 0)
        val = c0.copy()
        for d in range(3):
            if not r[d]:
                continue
            e = [0, 0, 0]
            e[d] = 1
            minus = at(VP, -e[2], -e[1], -e[0])
            plus = at(VP, e[2], e[1], e[0])
            w = sgn[d].reshape([-1 if x == d else 1 for x in (2, 1, 0)])
            val = val + w * minmod(c0 - minus, plus - c0)
        GP[:, g + of[2]:g + of[2] + mf[2], g + of[1]:g + of[1] + mf[1], g + of[0]:g + of[0] + mf[0]] = val
        # faces
        for d in range(3):
            A = VB[d]
            nf = [mf[x] + (1 if x == d else 0) for x in range(3)]
            tidx = [g + o[x] + (np.arange(nf[x]) >> r[x]) for x in range(3)]

            def coarse_face(Fc):
                """prolonged value on coarse faces of normal index Fc (padded) at the
                fine transverse positions; Fc is an array over the fine normal index"""
                idx = [None, None, None]
                for x in range(3):
                    idx[x] = Fc if x == d else tidx[x]

                def at_f(dk, dj, di):
                    return A[(idx[2] + dk)[:, None, None], (idx[1] + dj)[None, :, None],
                             (idx[0] + di)[None, None, :]]

                c = at_f(0, 0, 0)
                v = c.copy()
                for x in range(3):
                    if x == d or not r[x]:
                        continue
                    e = [0, 0, 0]
                    e[x] = 1
                    sx = np.where(np.arange(nf[x]) & 1, 0.25, -0.25)
                    w = sx.reshape([-1 if y == x else 1 for y in (2, 1, 0)])
                    v = v + w * minmod(c - at_f(-e[2], -e[1], -e[0]), at_f(e[2], e[1], e[0]) - c)
                return v

            q = np.arange(nf[d])
            if r[d]:
                lo = coarse_face(g + o[d] + (q >> 1))
                hi = coarse_face(g + o[d] + ((q + 1) >> 1))
                odd = (q & 1).reshape([-1 if y == d else 1 for y in (2, 1, 0)]).astype(bool)
                val = np.where(odd, 0.5 * (lo + hi), lo)
            else:
                val = coarse_face(g + o[d] + q)
            GB[d, g + of[2]:g + of[2] + nf[2], g + of[1]:g + of[1] + nf[1],
               g + of[0]:g + of[0] + nf[0]] = val

    def _view(self, lam, i, stage, s, cache):
        if lam in cache:
            return cache[lam]
        G = self._vg(lam)
        GP, GB = G.zeros()
        GP[:] = np.nan
        GB[:] = np.nan
        li = self.blocks[i]["lat"]
        order = sorted((n for n in range(len(self.blocks)) if n != i),
                       key=lambda n: (self.blocks[n]["lat"] == li, sum(self.blocks[n]["lev"]), n)) + [i]
        for n in order:
            rel = tuple(self.blocks[n]["lev"][d] - lam[d] for d in range(3))
            if max(abs(x) for x in rel) > 1 or (max(rel) > 0 and min(rel) < 0):
                continue
            if max(rel) <= 0 and min(rel) < 0:
                VP, VB = self._view(self.blocks[n]["lev"], i, stage, s, cache)
                self._put_prolong(GP, GB, n, VP, VB, tuple(-x for x in rel))
                continue
            Pn, Bn = self._source(i, n, stage, s)
            if max(rel) == 0:
                self._put_same(GP, GB, n, Pn, Bn)
            else:
                self._put_restrict(GP, GB, n, Pn, Bn, rel)
        self._seams(GB, lam, i)
        G.fill_bc(GP, GB)
        cache[lam] = (GP, GB)
        return GP, GB

    def _seams(self, GB, lam, i):
        """A face on a periodic seam is stored twice in a view (as the upper face of the
        last cell and the lower face of the first); both copies take the value of the
        holder the face rule picks (the viewing block, else one at the viewing time level,
        then the finest, then the higher block index)."""
        g = self.g
        N = self.nlev(lam)
        li = self.blocks[i]["lat"]

        def rank(n):
            bn = self.blocks[n]
            return (n == i, bn["lat"] == li, sum(bn["lev"]), n)

        for d in range(3):
            if self.cfg["bc"][2 * d] != oracle.BC_PERIODIC:
                continue
            t = [x for x in range(3) if x != d]
            for c1 in range(N[t[1]]):
                for c0 in range(N[t[0]]):
                    lo = [0, 0, 0]
                    lo[t[0]], lo[t[1]] = c0, c1
                    hi = list(lo)
                    hi[d] = N[d] - 1
                    w0, w1 = self._owner(lam, lo), self._owner(lam, hi)
                    if w0 is None or w1 is None or w0 == w1:
                        continue
                    p0 = [g + x for x in lo]
                    p1 = list(p0)
                    p1[d] = g + N[d]
                    a, b = (p0, p1) if rank(w0) >= rank(w1) else (p1, p0)
                    GB[d, b[2], b[1], b[0]] = GB[d, a[2], a[1], a[0]]

    def patch(self, i, stage, s):
        GP, GB = self._view(self.blocks[i]["lev"], i, stage, s, {})
        o = self.blocks[i]["org"]
        npd = self.ctx[i].np
        sl = (slice(None), slice(o[2], o[2] + npd[2]), slice(o[1], o[1] + npd[1]), slice(o[0], o[0] + npd[0]))
        return np.ascontiguousarray(GP[sl]), np.ascontiguousarray(GB[sl])

    # ------------------------------------------------------------------ refinement faces
    def _face_maps(self, link):
        """index arrays of the coarse faces of a refinement patch and of the fine faces
        averaged onto each, plus the same for the edges of the patch"""
        c, f, d, side, e, lo, hi = link
        g = self.g
        bc, bf = self.blocks[c], self.blocks[f]
        Ic = g + (bc["n"][d] if side == 1 else 0)
        If = g + (0 if side == 1 else bf["n"][d])
        return Ic, If

    def _fix_fluxes(self, ids):
        """coarse fluxes on refinement faces <- means of the fine ones; EMFs <- their
        dominant holder's at this time level"""
        g = self.g
        for link in self.links:
            c, f, d, side, e, lo, hi = link
            if c not in ids:
                continue
            Ic, If = self._face_maps(link)
            oc, of = self.blocks[c]["org"], self.blocks[f]["org"]
            Fc, Ff = self.ctx[c].flux_view(), self.ctx[f].flux_view()
            Ec, Ef = self.ctx[c].emf_view(), self.ctx[f].emf_view()
            t = [x for x in range(3) if x != d]
            # faces: coarse transverse cells lo..hi-1
            for cell in itertools.product(*[range(lo[x], hi[x]) if x != d else [0] for x in (2, 1, 0)]):
                cg = list(reversed(cell))
                pc = [0, 0, 0]
                pc[d] = Ic
                for x in t:
                    pc[x] = g + cg[x] - oc[x]
                acc = np.zeros(9)
                cnt = 0
                for off in itertools.product(*[range(1 + e[x]) if x != d else [0] for x in (2, 1, 0)]):
                    ofs = list(reversed(off))
                    pf = [0, 0, 0]
                    pf[d] = If
                    for x in t:
                        pf[x] = g + (cg[x] << e[x]) + ofs[x] - of[x]
                    acc = acc + Ff[d, :, pf[2], pf[1], pf[0]]
                    cnt += 1
                Fc[d, :, pc[2], pc[1], pc[0]] = acc * (1.0 / cnt)
        # EMFs whose dominant holder is finer at this time level
        for b in ids:
            Eb = self.ctx[b].emf_view()
            for a, e, D, subs in self.stage_edges[b]:
                ED = self.ctx[D].emf_view()
                acc = 0.0
                for (K, J, I) in subs:
                    acc = acc + ED[a, K, J, I]
                Eb[a, e[0], e[1], e[2]] = acc * (1.0 / len(subs))

    def _sync_faces(self, ids, Bout):
        """coarse copies of refinement faces <- mean of the fine faces"""
        g = self.g
        for link in self.links:
            c, f, d, side, e, lo, hi = link
            if c not in ids:
                continue
            Ic, If = self._face_maps(link)
            oc, of = self.blocks[c]["org"], self.blocks[f]["org"]
            t = [x for x in range(3) if x != d]
            for cell in itertools.product(*[range(lo[x], hi[x]) if x != d else [0] for x in (2, 1, 0)]):
                cg = list(reversed(cell))
                pc = [0, 0, 0]
                pc[d] = Ic
                for x in t:
                    pc[x] = g + cg[x] - oc[x]
                acc = 0.0
                cnt = 0
                for off in itertools.product(*[range(1 + e[x]) if x != d else [0] for x in (2, 1, 0)]):
                    ofs = list(reversed(off))
                    pf = [0, 0, 0]
                    pf[d] = If
                    for x in t:
                        pf[x] = g + (cg[x] << e[x]) + ofs[x] - of[x]
                    acc = acc + Bout[f][d, pf[2], pf[1], pf[0]]
                    cnt += 1
                Bout[c][d, pc[2], pc[1], pc[0]] = acc * (1.0 / cnt)

    # ------------------------------------------------------------------ stepping
    def step_level(self, lev, s):
        dt = self.dt_min * 2 ** lev
        ids = [i for i, b in enumerate(self.blocks) if b["lat"] == lev]
        self.trace += [(s, 0, lev, i) for i in ids]
        for i in ids:
            self.Pold[i] = self.P[i].copy()
            self.Bold[i] = self.B[i].copy()
        views = {}
        for i in ids:
            VP, VB = self.patch(i, "pred", s)
            views[i] = (VP, VB)
            self.ctx[i].stage_flux(VP, VB)
        self._fix_fluxes(ids)
        for i in ids:
            VP, VB = views[i]
            self.Ps[i] = VP.copy()
            self.Bs[i] = VB.copy()
            self.ctx[i].stage_apply(VP, VB, VP, 0.5 * dt, self.Ps[i], self.Bs[i])
        self._sync_faces(ids, self.Bs)
        for i in ids:
            VP, VB = self.patch(i, "corr", s)
            views[i] = (VP, VB)
            self.ctx[i].stage_flux(VP, VB)
        self._fix_fluxes(ids)
        newP = {i: self.P[i].copy() for i in ids}
        newB = {i: self.B[i].copy() for i in ids}
        for i in ids:
            VP, VB = views[i]
            self.ctx[i].stage_apply(self.P[i], self.B[i], VP, dt, newP[i], newB[i])
            self._registers(i, dt, s)
        for i in ids:
            self.P[i], self.B[i] = newP[i], newB[i]
        self._sync_faces(ids, self.B)
        self.steps[lev] += 1

    # ------------------------------------------------------------------ time levels
    def _registers(self, i, dt, s):
        """dt-weighted corrector fluxes and EMFs of block i (after the same-level fixes):
        this step, and the sum over the pair of steps a slower neighbour spans"""
        lat = self.blocks[i]["lat"]
        F = dt * self.ctx[i].last_flux()
        E = dt * self.ctx[i].last_emf()
        self.reg_step[i] = {"F": F, "E": E}
        if s % (2 ** (lat + 1)) == 0 or not self.reg_pair[i]:
            self.reg_pair[i] = {"F": F.copy(), "E": E.copy()}
        else:
            self.reg_pair[i]["F"] += F
            self.reg_pair[i]["E"] += E

    def _sync_block(self, b):
        """end of block b's step: refluxing, EMF correction, shared faces, re-inversion"""
        g = self.g
        n = self.blocks[b]["n"]
        lam = self.blocks[b]["lev"]
        dx = self.bdx[b]
        mine = self.reg_step[b]
        dU = {}
        touched = set()
        Bnew = self.B[b].copy()
        for d, side, f, D, subs in self.reflux[b]:
            theirs = 0.0
            for (K, J, I) in subs:
                theirs = theirs + self.reg_pair[D]["F"][d, :, K, J, I]
            theirs = theirs * (1.0 / len(subs))
            cell = list(f)
            if side == 1:
                cell[2 - d] -= 1
            cell = tuple(cell)
            sgn = 1.0 if side == 1 else -1.0
            dU[cell] = dU.get(cell, 0.0) + (mine["F"][d, :, f[0], f[1], f[2]] - theirs) / dx[d] * sgn

        def owned_face(c, loc):
            x = (loc[2], loc[1], loc[0])
            return all(g <= x[e] <= g + n[e] - (0 if e == c else 1) for e in range(3))

        for a, e, D, subs in self.sync_edges[b]:
            theirs = 0.0
            for (K, J, I) in subs:
                theirs = theirs + self.reg_pair[D]["E"][a, K, J, I]
            theirs = theirs * (1.0 / len(subs))
            dE = theirs - mine["E"][a, e[0], e[1], e[2]]
            x = [e[2], e[1], e[0]]
            for p in range(3):
                if p == a:
                    continue
                q = 3 - a - p
                sign = 1.0 if a == (p + 1) % 3 else -1.0
                for tq, sq in ((x[q] - 1, 1.0), (x[q], -1.0)):
                    fx = list(x)
                    fx[q] = tq
                    loc = (fx[2], fx[1], fx[0])
                    if not owned_face(p, loc):
                        continue
                    Bnew[p, loc[0], loc[1], loc[2]] += sign * sq * dE / dx[q]
                    for cp in (fx[p] - 1, fx[p]):
                        if g <= cp < g + n[p]:
                            cx = list(fx)
                            cx[p] = cp
                            touched.add((cx[2], cx[1], cx[0]))
        for d, side, f, D, subs in self.reflux[b]:
            if any(self.blocks[D]["lev"][x] < lam[x] for x in range(3)):
                continue            # the faster side is coarser: its face covers several
            acc = 0.0
            for (K, J, I) in subs:
                acc = acc + self.B[D][d, K, J, I]
            Bnew[d, f[0], f[1], f[2]] = acc * (1.0 / len(subs))
            for cp in (f[2 - d] - 1, f[2 - d]):
                if g <= cp < g + n[d]:
                    cx = list(f)
                    cx[2 - d] = cp
                    touched.add(tuple(cx))
        zero = np.zeros(9)
        for cell in sorted(set(dU) | touched):
            self.ctx[b].reinvert(self.P[b], self.B[b], Bnew, cell[0], cell[1], cell[2],
                                 dU.get(cell, zero))
        self.B[b] = Bnew

    def sync(self, s):
        for i, b in enumerate(self.blocks):
            lat = b["lat"]
            if lat == 0 or (s + 1) % (2 ** lat) != 0:
                continue
            if not self.reflux[i] and not self.sync_edges[i]:
                continue
            self.trace.append((s, 1, lat, i))
            self._sync_block(i)

    def divb(self):
        """max |div B| over the interior cells of all blocks (each with its own spacing)"""
        mx = 0.0
        for i in range(len(self.blocks)):
            mx = max(mx, self.ctx[i].divb(self.B[i]))
        return mx
