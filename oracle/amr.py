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
        one, else of the finest block, then the block at the viewing time level, then
        the block listed last.
  * Blocks across a refinement face run at the same time level.  In each stage, after
    all fluxes and EMFs are computed and before any update, the coarse block's fluxes on
    faces shared with finer blocks are replaced by the area mean of the fine fluxes, and
    its EMFs on edges of those faces by the mean of the fine EMFs along the coarse edge.
    After the update, the coarse copy of each shared face takes the mean of the fine
    faces (the finer side owns shared faces).
  * Time-level interfaces lie on x1 faces between blocks of one refinement level and
    are treated as in the local time-stepping driver (registers, refluxing, EMF and face
    correction, re-inversion).
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
        self.xnb = [self._x1_neighbours(i) for i in range(len(self.blocks))]
        self.links = self._refinement_faces()

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

    def _x1_neighbours(self, i):
        b = self.blocks[i]
        N1 = self.nlev(b["lev"])[0]
        periodic = self.cfg["bc"][0] == oracle.BC_PERIODIC
        out = {}
        for j, c in enumerate(self.blocks):
            if c["lev"] != b["lev"] or c["org"][1:] != b["org"][1:] or c["n"][1:] != b["n"][1:]:
                continue
            if c["org"][0] + c["n"][0] == b["org"][0] or (
                    periodic and b["org"][0] == 0 and c["org"][0] + c["n"][0] == N1):
                out["lo"] = j
            if b["org"][0] + b["n"][0] == c["org"][0] or (
                    periodic and c["org"][0] == 0 and b["org"][0] + b["n"][0] == N1):
                out["hi"] = j
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
                        if hit:
                            assert bc["lat"] == bf["lat"], "refinement faces join one time level"
                            out.append((c, f, d, side, e, lo, hi))
        return out

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
                       key=lambda n: (sum(self.blocks[n]["lev"]), self.blocks[n]["lat"] == li, n)) + [i]
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
        G.fill_bc(GP, GB)
        cache[lam] = (GP, GB)
        return GP, GB

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
        """coarse fluxes and EMFs on refinement faces <- means of the fine ones"""
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
            # edges along a (a != d) at face positions along b = the third dimension
            for a in t:
                b = [x for x in t if x != a][0]
                for ca in range(lo[a], hi[a]):
                    for cb in range(lo[b], hi[b] + 1):
                        pc = [0, 0, 0]
                        pc[d], pc[a], pc[b] = Ic, g + ca - oc[a], g + cb - oc[b]
                        acc = 0.0
                        cnt = 0
                        for oa in range(1 + e[a]):
                            pf = [0, 0, 0]
                            pf[d] = If
                            pf[a] = g + (ca << e[a]) + oa - of[a]
                            pf[b] = g + (cb << e[b]) - of[b]
                            acc = acc + Ef[a, pf[2], pf[1], pf[0]]
                            cnt += 1
                        Ec[a, pc[2], pc[1], pc[0]] = acc * (1.0 / cnt)

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

    def divb(self):
        """max |div B| over the interior cells of all blocks (each with its own spacing)"""
        mx = 0.0
        for i in range(len(self.blocks)):
            mx = max(mx, self.ctx[i].divb(self.B[i]))
        return mx
