"""Plain numpy replay of the library's ghost-gather lists (test helper).

It applies the plain copy lists and the refinement lists that the planner exports
(grmhd_plan_dump) to packed host arrays, following the documented meaning of each entry,
and checks every index against the block layout on the way.  Tests compare the result
with the oracle's block views, so the planner's integer tables are checked on the CPU
before any kernel runs them."""
from __future__ import annotations

import numpy as np

from paper_1912_10192_amd import grmhd

GF_FLIP, GF_CLAMP_NEG, GF_CLAMP_POS, GF_ZERO, GF_SLOW = 1, 2, 4, 8, 16


def minmod(a, b):
    if a > 0.0 and b > 0.0:
        return min(a, b)
    if a < 0.0 and b < 0.0:
        return max(a, b)
    return 0.0


class Replay:
    def __init__(self, desc: grmhd.Desc, cfg):
        self.desc = desc
        self.cfg = cfg
        nb = desc.d.n_blocks
        self.lay = [desc.layout(b) for b in range(nb)]
        self.ops = [desc.plan_dump(k) for k in range(4)]
        self.aops = [desc.plan_dump(4 + k) for k in range(4)]
        self.samp = desc.plan_dump(8)
        lmax = [max(desc.blocks[b].lev[d] for b in range(nb)) for d in range(3)]
        self.dx = []
        for b in range(nb):
            bd = desc.blocks[b]
            N = [cfg["n"][d] >> (lmax[d] - bd.lev[d]) for d in range(3)]
            self.dx.append([(cfg["xhi"][d] - cfg["xlo"][d]) / N[d] for d in range(3)])
        self._gd = {}
        self.outside = []   # sources read outside their block's interior (see interior())
        self.slow = set()   # sources read as the old state of a slower block: (b, loc, comp)

    def interior(self, b, loc, comp):
        """whether local index loc of block b is an interior cell (comp None) or a face of
        component comp on or inside the block's boundary (normal index g .. g + n)"""
        n1p, n2p, _ = self.lay[b][1]
        idx = (loc % n1p, (loc // n1p) % n2p, loc // (n1p * n2p))
        g = self.cfg["ng"]
        n = self.desc.blocks[b].n
        return all(g <= idx[d] < g + n[d] + (1 if comp == d else 0) for d in range(3))

    def _src(self, b, loc, comp, fl):
        if not self.interior(b, loc, comp):
            self.outside.append((b, loc, comp))
        if fl & GF_SLOW:
            self.slow.add((b, loc, comp))

    def vol(self, b):
        n = self.lay[b][1]
        return n[0] * n[1] * n[2]

    def gdet(self, b, loc):
        n1p, n2p, _ = self.lay[b][1]
        I, J = loc % n1p, (loc // n1p) % n2p
        key = (b, I, J)
        if key not in self._gd:
            if self.cfg["coords"] == 0:
                self._gd[key] = 1.0
            else:
                g = self.cfg["ng"]
                bd = self.desc.blocks[b]
                x1 = self.cfg["xlo"][0] + (bd.org[0] + I - g + 0.5) * self.dx[b][0]
                x2 = self.cfg["xlo"][1] + (bd.org[1] + J - g + 0.5) * self.dx[b][1]
                self._gd[key] = grmhd.geometry_point(1, self.cfg["a"], x1, x2)[0][13]
        return self._gd[key]

    def _cell(self, prim, s, v):
        blkf, loc, mask, _ = (int(x) for x in s)
        b, fl = blkf & 0xFFFFFF, (blkf >> 24) & 0xFF
        off, (n1p, n2p, n3p) = self.lay[b]
        V = n1p * n2p * n3p
        if mask == 0:
            assert 0 <= loc < V
            self._src(b, loc, None, fl)
            x = prim[5 * off + v * V + loc]
        else:
            num = den = 0.0
            for ok in range(2 if mask & 4 else 1):
                for oj in range(2 if mask & 2 else 1):
                    for oi in range(2 if mask & 1 else 1):
                        l = loc + (ok * n2p + oj) * n1p + oi
                        assert 0 <= l < V
                        self._src(b, l, None, fl)
                        w = self.gdet(b, l)
                        num = num + w * prim[5 * off + v * V + l]
                        den = den + w
            x = num / den
        if v == 3 and fl & GF_FLIP:
            x = -x
        if v == 2 and fl & GF_CLAMP_NEG and x > 0.0:
            x = 0.0
        if v == 2 and fl & GF_CLAMP_POS and x < 0.0:
            x = 0.0
        return x

    def _face(self, bface, s, comp):
        blkf, loc, mask, _ = (int(x) for x in s)
        b, fl = blkf & 0xFFFFFF, (blkf >> 24) & 0xFF
        if fl & GF_ZERO:
            return 0.0
        off, (n1p, n2p, n3p) = self.lay[b]
        V = n1p * n2p * n3p
        if mask == 0:
            assert 0 <= loc < V
            self._src(b, loc, comp, fl)
            x = bface[3 * off + comp * V + loc]
        else:
            acc = 0.0
            cnt = 0
            for ok in range(2 if mask & 4 else 1):
                for oj in range(2 if mask & 2 else 1):
                    for oi in range(2 if mask & 1 else 1):
                        l = loc + (ok * n2p + oj) * n1p + oi
                        assert 0 <= l < V
                        self._src(b, l, comp, fl)
                        acc = acc + bface[3 * off + comp * V + l]
                        cnt += 1
            x = acc * (1.0 / cnt)
        if fl & GF_FLIP:
            x = -x
        return x

    def fill(self, prim, bface):
        """fill every ghost of the packed host arrays in place"""
        for kind in range(4):
            for dst_b, dst_loc, srcf, src_loc in self.ops[kind]:
                sb, fl = int(srcf) & 0xFFFFFF, (int(srcf) >> 24) & 0xFF
                doff, _ = self.lay[dst_b]
                soff, _ = self.lay[sb]
                Vd, Vs = self.vol(dst_b), self.vol(sb)
                assert 0 <= dst_loc < Vd and 0 <= src_loc < Vs
                if not (fl & GF_ZERO):
                    self._src(sb, src_loc, None if kind == 0 else kind - 1, fl)
                if kind == 0:
                    for v in range(5):
                        x = prim[5 * soff + v * Vs + src_loc]
                        if v == 3 and fl & GF_FLIP:
                            x = -x
                        if v == 2 and fl & GF_CLAMP_NEG and x > 0.0:
                            x = 0.0
                        if v == 2 and fl & GF_CLAMP_POS and x < 0.0:
                            x = 0.0
                        prim[5 * doff + v * Vd + dst_loc] = x
                else:
                    c = kind - 1
                    x = bface[3 * soff + c * Vs + src_loc]
                    if fl & GF_ZERO:
                        x = 0.0
                    elif fl & GF_FLIP:
                        x = -x
                    bface[3 * doff + c * Vd + dst_loc] = x
        for kind in range(4):
            for dst_b, dst_loc, mode, first in self.aops[kind]:
                doff, _ = self.lay[dst_b]
                Vd = self.vol(dst_b)
                assert 0 <= dst_loc < Vd
                pd = mode & 7
                ofl = (mode >> 16) & 0xFF
                S = self.samp[first:]
                if kind == 0:
                    for v in range(5):
                        c = self._cell(prim, S[0], v)
                        x = c
                        k = 1
                        for d in range(3):
                            if not (pd >> d) & 1:
                                continue
                            sm, sp = self._cell(prim, S[k], v), self._cell(prim, S[k + 1], v)
                            k += 2
                            sg = 0.25 if (mode >> (4 + d)) & 1 else -0.25
                            x = x + sg * minmod(c - sm, sp - c)
                        if v == 3 and ofl & GF_FLIP:
                            x = -x
                        if v == 2 and ofl & GF_CLAMP_NEG and x > 0.0:
                            x = 0.0
                        if v == 2 and ofl & GF_CLAMP_POS and x < 0.0:
                            x = 0.0
                        prim[5 * doff + v * Vd + dst_loc] = x
                else:
                    comp = kind - 1
                    t = pd & ~(1 << comp)
                    nst = 1 + 2 * bin(t).count("1")
                    vals = []
                    for q in range(2 if mode & 256 else 1):
                        R = S[q * nst:]
                        c = self._face(bface, R[0], comp)
                        x = c
                        k = 1
                        for d in range(3):
                            if not (t >> d) & 1:
                                continue
                            sm, sp = self._face(bface, R[k], comp), self._face(bface, R[k + 1], comp)
                            k += 2
                            sg = 0.25 if (mode >> (4 + d)) & 1 else -0.25
                            x = x + sg * minmod(c - sm, sp - c)
                        vals.append(x)
                    x = 0.5 * (vals[0] + vals[1]) if len(vals) == 2 else vals[0]
                    if ofl & GF_ZERO:
                        x = 0.0
                    elif ofl & GF_FLIP:
                        x = -x
                    bface[3 * doff + comp * Vd + dst_loc] = x
