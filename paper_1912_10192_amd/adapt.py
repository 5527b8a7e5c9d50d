"""Refinement during the run (Sec. 3.3): a block-level criterion, the new layout it asks
for (blocks split into eight children, or six on the polar axis; children merged back
into their parent), nesting kept at one level between touching blocks (none across the
polar axis), and a cycle loop that regrids every so many cycles (grmhd_regrid).

Blocks form a tree: a child records its parent, and only children whose siblings are
all present and all ask for it are merged back; blocks of the starting layout are roots.
Host logic on the block list; the state never leaves the device."""
from __future__ import annotations

from paper_1912_10192_amd import configs, grmhd

BC_POLAR, BC_PERIODIC = 1, 2


def _lmax(blocks):
    return [max(b["lev"][d] for b in blocks) for d in range(3)]


def _box(b, L):
    lo = [b["org"][d] << (L[d] - b["lev"][d]) for d in range(3)]
    hi = [(b["org"][d] + b["n"][d]) << (L[d] - b["lev"][d]) for d in range(3)]
    return lo, hi


class Layout:
    """a block list over a grid whose level-0 cells are N0 per dimension"""

    def __init__(self, cfg, blocks):
        self.cfg = cfg
        L = _lmax(blocks)
        self.N0 = [cfg["n"][d] >> L[d] for d in range(3)]
        self.blocks = [dict(b) for b in blocks]

    def n_eff(self, blocks=None):
        L = _lmax(blocks if blocks is not None else self.blocks)
        return tuple(self.N0[d] << L[d] for d in range(3))

    # ------------------------------------------------------------------ contacts
    def contacts(self, blocks):
        """(b, s, across_axis) for every block s that meets block b's box grown by ng
        cells of b's levels (across the polar axis mirrored to phi + pi, along phi
        periodic, clipped at the x1 ends): every block b's ghost cells can come from"""
        import numpy as np

        L = _lmax(blocks)
        Nf = np.array([self.N0[d] << L[d] for d in range(3)])
        lev = np.array([b["lev"] for b in blocks])
        org = np.array([b["org"] for b in blocks])
        n = np.array([b["n"] for b in blocks])
        sh = np.array(L)[None, :] - lev
        lo = org << sh
        hi = (org + n) << sh
        g = self.cfg["ng"]
        glo = lo - (g << sh)
        ghi = hi + (g << sh)
        glo[:, 0] = np.maximum(glo[:, 0], 0)
        ghi[:, 0] = np.minimum(ghi[:, 0], Nf[0])
        out = []

        def overlap(alo, ahi, across):
            hit = np.ones((len(blocks), len(blocks)), dtype=bool)
            for d in range(3):
                a0, a1 = alo[:, d][:, None], ahi[:, d][:, None]
                b0, b1 = lo[:, d][None, :], hi[:, d][None, :]
                t = (a0 < b1) & (b0 < a1)
                if d == 2 or self.cfg["bc"][2 * d] == BC_PERIODIC:
                    N = Nf[d]
                    t = t | ((a0 - N < b1) & (b0 < a1 - N)) | ((a0 + N < b1) & (b0 < a1 + N))
                hit &= t
            if not across:
                np.fill_diagonal(hit, False)
            out.extend((int(i), int(j), across) for i, j in zip(*np.nonzero(hit)))

        if self.cfg["bc"][2] == BC_POLAR:
            a_lo, a_hi = glo.copy(), ghi.copy()
            a_lo[:, 1], a_hi[:, 1] = np.maximum(glo[:, 1], 0), np.minimum(ghi[:, 1], Nf[1])
            overlap(a_lo, a_hi, False)
            h = Nf[2] // 2
            for side in (0, 1):
                beyond = glo[:, 1] < 0 if side == 0 else ghi[:, 1] > Nf[1]
                if not beyond.any():
                    continue
                m_lo, m_hi = glo.copy(), ghi.copy()
                if side == 0:
                    m_lo[:, 1], m_hi[:, 1] = 0, np.where(beyond, -glo[:, 1], 0)
                else:
                    m_lo[:, 1], m_hi[:, 1] = np.where(beyond, 2 * Nf[1] - ghi[:, 1], Nf[1]), Nf[1]
                m_lo[:, 2] += h
                m_hi[:, 2] += h
                overlap(m_lo, m_hi, True)
        else:
            overlap(glo, ghi, False)
        return out

    def violations(self, blocks):
        """pairs (b, s) from contacts() more than one level apart in a dimension, finer in
        one and coarser in another, or at different levels across the axis.  The grown
        box holds every ghost cell the planner builds, so these pairs include all it
        would refuse (violations_cells checks cell by cell)"""
        bad = set()
        for i, j, across in self.contacts(blocks):
            r = [blocks[j]["lev"][d] - blocks[i]["lev"][d] for d in range(3)]
            if (max(abs(x) for x in r) > 1 or (max(r) > 0 and min(r) < 0)
                    or (across and any(r))):
                bad.add((i, j))
        return sorted(bad)

    def time_levels(self, blocks, dt, nlev):
        """time levels from each block's Courant step (Sec. 3.5): the largest l below nlev
        with 2^l dt_min <= dt_b, then lowered until blocks in contact differ by at most
        one level"""
        import math

        dmin = min(dt)
        lat = [min(nlev - 1, int(math.floor(math.log2(d / dmin) + 1e-12))) for d in dt]
        pairs = [(i, j) for i, j, _ in self.contacts(blocks) if i != j]
        changed = True
        while changed:
            changed = False
            for i, j in pairs:
                if lat[i] > lat[j] + 1:
                    lat[i] = lat[j] + 1
                    changed = True
        return lat

    def violations_cells(self, blocks):
        """pairs (b, s) where a ghost cell of block b (ng deep at b's levels; across the
        polar axis mirrored to phi + pi, along phi periodic, beyond the x1 ends clamped)
        lies in block s and the two are more than one level apart in a dimension, finer
        in one and coarser in another, or at different levels across the axis (the
        planner's rules for the ghost values it can build)"""
        import numpy as np

        L = _lmax(blocks)
        Nf = [self.N0[d] << L[d] for d in range(3)]
        own = np.full((Nf[2], Nf[1], Nf[0]), -1, dtype=np.int64)
        for i, b in enumerate(blocks):
            lo, hi = _box(b, L)
            own[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = i
        g = self.cfg["ng"]
        polar = self.cfg["bc"][2] == BC_POLAR
        lev = np.array([b["lev"] for b in blocks])
        bad = set()
        for i, b in enumerate(blocks):
            lam, o, n = b["lev"], b["org"], b["n"]
            N = [self.N0[d] << lam[d] for d in range(3)]
            ax = [np.arange(o[d] - g, o[d] + n[d] + g) for d in range(3)]
            K, J, I = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
            ghost = ((I < o[0]) | (I >= o[0] + n[0]) | (J < o[1]) | (J >= o[1] + n[1])
                     | (K < o[2]) | (K >= o[2] + n[2]))
            I, J, K = I[ghost], J[ghost], K[ghost]
            across = np.zeros(I.shape, dtype=bool)
            if polar:
                across = (J < 0) | (J >= N[1])
                K = np.where(across, K + N[2] // 2, K)
                J = np.where(J < 0, -1 - J, np.where(J >= N[1], 2 * N[1] - 1 - J, J))
            else:
                J = np.mod(J, N[1])
            K = np.mod(K, N[2])
            I = np.clip(I, 0, N[0] - 1)
            src = own[K << (L[2] - lam[2]), J << (L[1] - lam[1]), I << (L[0] - lam[0])]
            for s_, acr in set(zip(src.tolist(), across.tolist())):
                r = lev[s_] - np.array(lam)
                if (np.abs(r).max() > 1 or (r.max() > 0 and r.min() < 0)
                        or (acr and np.abs(r).max() > 0)):
                    bad.add((i, int(s_)))
        return sorted(bad)

    # ------------------------------------------------------------------ edits
    def _pole(self, b, blocks):
        if self.cfg["bc"][2] != BC_POLAR:
            return None
        n2 = self.N0[1] << b["lev"][1]
        if b["org"][1] == 0:
            return "north"
        if b["org"][1] + b["n"][1] == n2:
            return "south"
        return None

    def split(self, blocks, i):
        b = blocks[i]
        kids = configs.split_block({k: v for k, v in b.items() if k != "parent"},
                                   self.N0[1] << b["lev"][1], self._pole(b, blocks))
        for k in kids:
            k["parent"] = b
        return blocks[:i] + kids + blocks[i + 1:]

    def refine(self, flags, max_level=None):
        """split every flagged block, then whatever the nesting rules need"""
        blocks = list(self.blocks)
        todo = sorted((i for i, f in enumerate(flags) if f > 0), reverse=True)
        for i in todo:
            if max_level is None or max(blocks[i]["lev"]) < max_level:
                blocks = self.split(blocks, i)
        for _ in range(64):
            bad = self.violations(blocks)
            if not bad:
                return blocks
            # split the coarser block of every offending pair (each once), then look again
            coarse = set()
            for a, c in bad:
                coarse.add(a if sum(blocks[a]["lev"]) < sum(blocks[c]["lev"]) else c)
            for i in sorted(coarse, reverse=True):
                blocks = self.split(blocks, i)
        raise RuntimeError("nesting not reached")

    def coarsen(self, blocks, flags):
        """merge sibling groups whose members all ask for it, where the parent keeps the
        nesting rules (repeated until no group merges: one merge can allow another)"""
        ask = {id(b) for b, f in zip(blocks, flags) if f < 0}
        out = list(blocks)
        changed = True
        while changed:
            changed = False
            groups = {}
            for b in out:
                if "parent" in b and id(b) in ask:
                    groups.setdefault(id(b["parent"]), []).append(b)
            complete = [k for k in groups.values()
                        if len(k) == (6 if self._pole(k[0]["parent"], out) else 8)]
            for kids in complete:
                trial = [b for b in out if all(b is not k for k in kids)] + [kids[0]["parent"]]
                if not self.violations(trial):
                    out = trial
                    changed = True
            if not changed and len(complete) > 1:
                # groups that only merge together (blocks facing each other across the
                # polar axis must share their levels)
                gone = [k for kids in complete for k in kids]
                trial = ([b for b in out if all(b is not k for k in gone)]
                         + [kids[0]["parent"] for kids in complete])
                if not self.violations(trial):
                    out = trial
                    changed = True
        return out


def estimate_steps(old, dt_old, new):
    """Courant steps of the blocks of a new layout from those of the old one: a block
    kept keeps its step, a child takes half of its nearest ancestor's in the old layout
    per generation between them, a merged parent twice the smallest of its children's"""
    by_id = {id(b): d for b, d in zip(old, dt_old)}
    out = []
    for b in new:
        if id(b) in by_id:
            out.append(by_id[id(b)])
            continue
        a, f = b, 1.0
        while "parent" in a and id(a) not in by_id:
            a, f = a["parent"], 0.5 * f
        if id(a) in by_id:
            out.append(f * by_id[id(a)])
            continue
        kids = [by_id[id(o)] for o in old if o.get("parent") is b]
        out.append(2.0 * min(kids))
    return out


def block_max(grid, var=0):
    """per-block maximum of a primitive over the interior cells, from the device state"""
    torch = grid.torch
    g = grid.cfg["ng"]
    vals = []
    for b in range(len(grid.desc.blocks)):
        off, (n1p, n2p, n3p) = grid.desc.layout(b)
        V = n1p * n2p * n3p
        n = grid.desc.blocks[b].n
        v = grid.prim[5 * off + var * V:5 * off + (var + 1) * V].view(n3p, n2p, n1p)
        vals.append(v[g:g + n[2], g:g + n[1], g:g + n[0]].max())
    return torch.stack(vals).cpu().tolist()


class AdaptiveGrid:
    """A grid that regrids every `every` cycles on a density criterion: blocks whose
    densest cell exceeds rho_refine are split (up to max_level), sibling groups whose
    densest cell lies below rho_coarsen are merged."""

    def __init__(self, cfg, blocks, states, rho_refine, rho_coarsen, every=1, max_level=2,
                 batched=1, pool_sizes=None, lat_levels=None):
        """pool_sizes: (prim, bface, work) element counts of the largest layout to expect;
        two buffer sets of that size are then allocated once, and the grid alternates
        between them at every regrid (the old layout's set is free again once the regrid
        has filled the new one), so regrids allocate no device memory for the state.
        lat_levels: assign the new layout's time levels (at most that many) from the
        blocks' Courant steps at each regrid (a child takes half its parent's step, a
        merged parent twice its children's smallest); None keeps the levels the blocks
        had (children inherit theirs)"""
        self.layout = Layout(cfg, blocks)
        self.pools = None
        if pool_sizes is not None:
            import torch

            npr, nbf, nwk = pool_sizes
            self.pools = [(torch.zeros(npr, dtype=torch.float64, device="cuda"),
                           torch.zeros(nbf, dtype=torch.float64, device="cuda"),
                           torch.empty(nwk + 256, dtype=torch.uint8, device="cuda"))
                          for _ in range(2)]
            self.active = 0
        self.grid = grmhd.Grid(cfg, blocks=blocks, batched=batched,
                               pool=self.pools[0] if self.pools else None)
        self.grid.set_blocks(states)
        self.rho_refine, self.rho_coarsen = rho_refine, rho_coarsen
        self.every, self.max_level = every, max_level
        self.lat_levels = lat_levels
        self.cycles = 0
        self.history = []

    def decide(self):
        rho = block_max(self.grid)
        flags = [1 if r > self.rho_refine else (-1 if r < self.rho_coarsen else 0) for r in rho]
        blocks = self.layout.refine(flags, self.max_level)
        # flags of the refined list: children of this decision keep 0
        idx = {id(b): f for b, f in zip(self.layout.blocks, flags)}
        flags2 = [idx.get(id(b), 0) for b in blocks]
        return self.layout.coarsen(blocks, flags2)

    def _with_time_levels(self, new):
        """the new layout with time levels from the Courant steps of the current grid's
        blocks (see estimate_steps)"""
        dts = estimate_steps(self.layout.blocks, self.grid.block_dt(), new)
        lat = self.layout.time_levels(new, dts, self.lat_levels)
        out = []
        for b, l in zip(new, lat):
            b2 = dict(b)
            b2["lat"] = l
            out.append(b2)
        return out

    def adapt(self, blocks=None):
        """regrid to `blocks`, or to the criterion's layout; returns whether it changed"""
        new = blocks if blocks is not None else self.decide()
        key = lambda bl: [(b["lev"], b["org"], b["n"]) for b in bl]
        if key(new) == key(self.layout.blocks):
            return False
        if self.lat_levels is not None:
            new = self._with_time_levels(new)
        plain = [{k: v for k, v in b.items() if k != "parent"} for b in new]
        if self.pools:
            nxt = 1 - self.active
            g = self.grid.regrid(plain, pool=self.pools[nxt])
            self.grid.close()
            self.grid, self.active = g, nxt
        else:
            self.grid = self.grid.regrid(plain)
        self.layout.blocks = list(new)
        self.layout.cfg = self.grid.cfg
        self.history.append(plain)
        return True

    def step(self, cycles):
        st = None
        for _ in range(cycles):
            st = self.grid.step(1)
            self.cycles += 1
            if self.cycles % self.every == 0:
                self.adapt()
        return st
