"""Local adaptive time-stepping on a block grid, written plainly with the oracle's stage.

TEST INFRASTRUCTURE ONLY.  Shares no code with the HIP path.

What it does (paper Sec. 3.5, with the readings stated in the design notes):
  * every block has a time level lat; with L levels a cycle is 2^(L-1) substeps of dt_min
    and a block of level l steps (full midpoint step, dt_min 2^l) at substeps s with
    s mod 2^l = 0; in a substep the slower levels go first;
  * dt_min = min over blocks of (Courant step of the block) / 2^lat, once per cycle;
  * ghost values of a block come from its neighbours as they stand at the block's stage
    time: same level -> their state at that stage, slower -> linear interpolation in time
    between their stored start and end states (weights are exact dyadic fractions),
    faster -> their current state (the start time of the slower block);
  * a face shared by two neighbours is taken from the one at the viewing block's level, else
    from the block whose cell has it as its lower face;
  * at the end of a slower block's step, the fluxes it used on faces shared with a faster
    neighbour are replaced by the faster neighbour's time-integrated fluxes, the edge EMFs
    on those faces by the faster side's time-integrated EMFs, the shared faces take the
    faster side's values, and the corrected boundary cells are inverted again.
Level interfaces lie on x1 block faces (time levels vary with radius).
"""
from __future__ import annotations

import numpy as np

import oracle


class LatGrid:
    def __init__(self, cfg: dict, blocks: list):
        self.cfg = dict(cfg)
        self.g = g = cfg["ng"]
        self.N = tuple(cfg["n"])
        self.dx = [(cfg["xhi"][d] - cfg["xlo"][d]) / self.N[d] for d in range(3)]
        self.blocks = [dict(b) for b in blocks]
        self.L = max(b["lat"] for b in blocks) + 1
        self.glob = oracle.Grid(cfg)
        self.ctx = []
        for b in self.blocks:
            o, n = b["org"], b["n"]
            bc = list(cfg["bc"])
            for d, (lo, hi) in enumerate(((0, 1), (2, 3), (4, 5))):
                if o[d] != 0:
                    bc[lo] = oracle.BC_PERIODIC
                if o[d] + n[d] != self.N[d]:
                    bc[hi] = oracle.BC_PERIODIC
            xlo = tuple(cfg["xlo"][d] + o[d] * self.dx[d] for d in range(3))
            xhi = tuple(cfg["xlo"][d] + (o[d] + n[d]) * self.dx[d] for d in range(3))
            self.ctx.append(oracle.Grid(dict(cfg, n=tuple(n), xlo=xlo, xhi=xhi, bc=tuple(bc))))
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
        self.bdx = [list(self.dx) for _ in self.blocks]
        self.trace = []     # executed schedule: (substep, 0 step / 1 sync, level, block)
        self.xnb = [self._x1_neighbours(i) for i in range(len(self.blocks))]

    # ------------------------------------------------------------------ layout
    def _x1_neighbours(self, i):
        b = self.blocks[i]
        N1 = self.N[0]
        periodic = self.cfg["bc"][0] == oracle.BC_PERIODIC
        out = {}
        for j, c in enumerate(self.blocks):
            if c["org"][1:] != b["org"][1:] or c["n"][1:] != b["n"][1:]:
                continue
            if c["org"][0] + c["n"][0] == b["org"][0] or (
                    periodic and b["org"][0] == 0 and c["org"][0] + c["n"][0] == N1):
                out["lo"] = j
            if b["org"][0] + b["n"][0] == c["org"][0] or (
                    periodic and c["org"][0] == 0 and b["org"][0] + b["n"][0] == N1):
                out["hi"] = j
        return out

    def set_state(self, P, B1, B2, B3):
        g = self.g
        for i, b in enumerate(self.blocks):
            o, n = b["org"], b["n"]
            self.P[i][:, g:g + n[2], g:g + n[1], g:g + n[0]] = P[:, o[2]:o[2] + n[2], o[1]:o[1] + n[1], o[0]:o[0] + n[0]]
            self.B[i][0, g:g + n[2], g:g + n[1], g:g + n[0] + 1] = B1[o[2]:o[2] + n[2], o[1]:o[1] + n[1], o[0]:o[0] + n[0] + 1]
            self.B[i][1, g:g + n[2], g:g + n[1] + 1, g:g + n[0]] = B2[o[2]:o[2] + n[2], o[1]:o[1] + n[1] + 1, o[0]:o[0] + n[0]]
            self.B[i][2, g:g + n[2] + 1, g:g + n[1], g:g + n[0]] = B3[o[2]:o[2] + n[2] + 1, o[1]:o[1] + n[1], o[0]:o[0] + n[0]]

    def get_state(self):
        g = self.g
        N1, N2, N3 = self.N
        P = np.zeros((5, N3, N2, N1))
        B1 = np.zeros((N3, N2, N1 + 1))
        B2 = np.zeros((N3, N2 + 1, N1))
        B3 = np.zeros((N3 + 1, N2, N1))
        for i in range(len(self.blocks)):
            b = self.blocks[i]
            o, n = b["org"], b["n"]
            P[:, o[2]:o[2] + n[2], o[1]:o[1] + n[1], o[0]:o[0] + n[0]] = self.P[i][:, g:g + n[2], g:g + n[1], g:g + n[0]]
            B1[o[2]:o[2] + n[2], o[1]:o[1] + n[1], o[0]:o[0] + n[0] + 1] = self.B[i][0, g:g + n[2], g:g + n[1], g:g + n[0] + 1]
            B2[o[2]:o[2] + n[2], o[1]:o[1] + n[1] + 1, o[0]:o[0] + n[0]] = self.B[i][1, g:g + n[2], g:g + n[1] + 1, g:g + n[0]]
            B3[o[2]:o[2] + n[2] + 1, o[1]:o[1] + n[1], o[0]:o[0] + n[0]] = self.B[i][2, g:g + n[2] + 1, g:g + n[1], g:g + n[0]]
        return P, B1, B2, B3

    # ------------------------------------------------------------------ ghosts
    def _source(self, i, n, stage, s):
        """state of block n as block i sees it at stage ('pred'/'corr') of substep s"""
        li, ln = self.blocks[i]["lat"], self.blocks[n]["lat"]
        if n == i or ln == li:
            return (self.P[n], self.B[n]) if stage == "pred" else (self.Ps[n], self.Bs[n])
        if ln > li:
            period = 2 ** ln
            t0 = s - s % period
            t = s + (0.0 if stage == "pred" else 0.5 * 2 ** li)
            w = (t - t0) / period
            return (self.Pold[n] + w * (self.P[n] - self.Pold[n]),
                    self.Bold[n] + w * (self.B[n] - self.Bold[n]))
        return self.P[n], self.B[n]

    def patch(self, i, stage, s):
        """block i's arrays with every ghost filled for this stage"""
        g = self.g
        GP, GB = self.glob.zeros()
        # A face shared by two other blocks takes the copy of the one at this block's time
        # level (the copy that same-level neighbour evolves itself), else the copy of the
        # block whose cell has it as its lower face; this block's own faces come last.
        li = self.blocks[i]["lat"]
        order = sorted((n for n in range(len(self.blocks)) if n != i),
                       key=lambda n: (self.blocks[n]["lat"] == li, n)) + [i]
        for n in order:
            b = self.blocks[n]
            o, m = b["org"], b["n"]
            Pn, Bn = self._source(i, n, stage, s)
            GP[:, g + o[2]:g + o[2] + m[2], g + o[1]:g + o[1] + m[1], g + o[0]:g + o[0] + m[0]] = \
                Pn[:, g:g + m[2], g:g + m[1], g:g + m[0]]
            GB[0, g + o[2]:g + o[2] + m[2], g + o[1]:g + o[1] + m[1], g + o[0]:g + o[0] + m[0] + 1] = \
                Bn[0, g:g + m[2], g:g + m[1], g:g + m[0] + 1]
            GB[1, g + o[2]:g + o[2] + m[2], g + o[1]:g + o[1] + m[1] + 1, g + o[0]:g + o[0] + m[0]] = \
                Bn[1, g:g + m[2], g:g + m[1] + 1, g:g + m[0]]
            GB[2, g + o[2]:g + o[2] + m[2] + 1, g + o[1]:g + o[1] + m[1], g + o[0]:g + o[0] + m[0]] = \
                Bn[2, g:g + m[2] + 1, g:g + m[1], g:g + m[0]]
        self.glob.fill_bc(GP, GB)
        b = self.blocks[i]
        o = b["org"]
        npd = self.ctx[i].np
        sl = (slice(None), slice(o[2], o[2] + npd[2]), slice(o[1], o[1] + npd[1]), slice(o[0], o[0] + npd[0]))
        return np.ascontiguousarray(GP[sl]), np.ascontiguousarray(GB[sl])

    # ------------------------------------------------------------------ stepping
    def _registers(self, i, dt, s):
        g = self.g
        n1, n2, n3 = self.blocks[i]["n"]
        F = self.ctx[i].last_flux()
        E = self.ctx[i].last_emf()
        lat = self.blocks[i]["lat"]
        first_of_pair = s % (2 ** (lat + 1)) == 0
        for side, I in (("lo", g), ("hi", g + n1)):
            vals = {"F": dt * F[0, :, g:g + n3, g:g + n2, I].copy(),
                    "E2": dt * E[1, g:g + n3 + 1, g:g + n2, I].copy(),
                    "E3": dt * E[2, g:g + n3, g:g + n2 + 1, I].copy()}
            self.reg_step[i][side] = vals
            if first_of_pair or side not in self.reg_pair[i]:
                self.reg_pair[i][side] = {k: v.copy() for k, v in vals.items()}
            else:
                for k in vals:
                    self.reg_pair[i][side][k] += vals[k]

    def step_level(self, lev, s):
        dt = self.dt_min * 2 ** lev
        ids = [i for i, b in enumerate(self.blocks) if b["lat"] == lev]
        self.trace += [(s, 0, lev, i) for i in ids]
        for i in ids:
            self.Pold[i] = self.P[i].copy()
            self.Bold[i] = self.B[i].copy()
        for i in ids:
            VP, VB = self.patch(i, "pred", s)
            self.Ps[i] = VP.copy()
            self.Bs[i] = VB.copy()
            self.ctx[i].stage(VP, VB, VP, VB, 0.5 * dt, self.Ps[i], self.Bs[i])
        new = {}
        for i in ids:
            VP, VB = self.patch(i, "corr", s)
            P2, B2 = self.P[i].copy(), self.B[i].copy()
            self.ctx[i].stage(self.P[i], self.B[i], VP, VB, dt, P2, B2)
            self._registers(i, dt, s)
            new[i] = (P2, B2)
        for i, (P2, B2) in new.items():
            self.P[i], self.B[i] = P2, B2
        self.steps[lev] += 1

    def sync(self, s):
        g = self.g
        for i, b in enumerate(self.blocks):
            lat = b["lat"]
            if lat == 0 or (s + 1) % (2 ** lat) != 0:
                continue
            dx1 = self.bdx[i][0]
            n1, n2, n3 = b["n"]
            for side, opp, sgn in (("lo", "hi", -1.0), ("hi", "lo", 1.0)):
                f = self.xnb[i].get(side)
                if f is None or self.blocks[f]["lat"] != lat - 1:
                    continue
                self.trace.append((s, 1, lat, i))
                mine, theirs = self.reg_step[i][side], self.reg_pair[f][opp]
                dF = (mine["F"] - theirs["F"]) / dx1 * sgn        # [9][n3][n2]
                dE2 = theirs["E2"] - mine["E2"]                    # [n3+1][n2]
                dE3 = theirs["E3"] - mine["E3"]                    # [n3][n2+1]
                Ic = g + n1 - 1 if side == "hi" else g
                If = g + n1 if side == "hi" else g
                Bnew = self.B[i].copy()
                Bnew[1, g:g + n3, g:g + n2 + 1, Ic] += sgn * dE3 / dx1
                Bnew[2, g:g + n3 + 1, g:g + n2, Ic] -= sgn * dE2 / dx1
                # the shared faces take the faster side's values
                Ff = g if side == "hi" else g + self.blocks[f]["n"][0]
                Bnew[0, g:g + n3, g:g + n2, If] = self.B[f][0, g:g + n3, g:g + n2, Ff]
                for k in range(n3):
                    for j in range(n2):
                        self.ctx[i].reinvert(self.P[i], self.B[i], Bnew, g + k, g + j, Ic,
                                             dF[:, k, j])
                self.B[i] = Bnew

    def cycle(self):
        dts = [self.ctx[i].dt(self.P[i], self.B[i]) / 2 ** b["lat"]
               for i, b in enumerate(self.blocks)]
        self.dt_min = min(dts)
        for s in range(2 ** (self.L - 1)):
            for lev in range(self.L - 1, -1, -1):
                if s % (2 ** lev) == 0:
                    self.step_level(lev, s)
            self.sync(s)
        self.t += self.dt_min * 2 ** (self.L - 1)
        return self.dt_min
