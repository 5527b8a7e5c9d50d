"""Exact solution of the special-relativistic hydrodynamic Riemann problem for an ideal
gas with velocities normal to the initial discontinuity (Marti & Mueller 1994, J. Fluid
Mech. 258, 317): each nonlinear wave is a shock (Taub adiabat and the invariant mass
flux across it) or a rarefaction (constant entropy and Riemann invariant), and the
pressure of the intermediate states makes the velocities on both sides of the contact
equal.  Test infrastructure: an independent check of the oracle's shock capturing."""
from __future__ import annotations

import math


class State:
    def __init__(self, rho, p, v, gam):
        self.rho, self.p, self.v, self.gam = rho, p, v, gam

    @property
    def h(self):
        return 1.0 + self.gam * self.p / ((self.gam - 1.0) * self.rho)

    @property
    def cs(self):
        return math.sqrt(self.gam * self.p / (self.rho * self.h))

    @property
    def W(self):
        return 1.0 / math.sqrt(1.0 - self.v * self.v)


def _b(cs, gam):
    """the sound-speed part of the Riemann invariants"""
    g = math.sqrt(gam - 1.0)
    return math.log((g + cs) / (g - cs)) / g


def _cs_of(rho, p, gam):
    h = 1.0 + gam * p / ((gam - 1.0) * rho)
    return math.sqrt(gam * p / (rho * h))


def _rarefaction(a: State, p, sign):
    """state behind a rarefaction of family sign (-1: moving left, +1: right) at
    pressure p < a.p"""
    gam = a.gam
    rho = a.rho * (p / a.p) ** (1.0 / gam)
    cs = _cs_of(rho, p, gam)
    # J(+) is carried through left fans, J(-) through right ones
    J = math.atanh(a.v) - sign * _b(a.cs, gam)
    v = math.tanh(J + sign * _b(cs, gam))
    return State(rho, p, v, gam)


def _shock(a: State, p, sign):
    """state behind a shock of family sign at pressure p > a.p, and the shock velocity"""
    gam = a.gam
    ha = a.h
    k = (gam - 1.0) * (p - a.p) / (gam * p)
    # Taub adiabat h^2 - ha^2 = (h/rho + ha/rho_a)(p - pa) with h/rho = k (h - 1) h/(p - pa)
    A = 1.0 - k
    Bq = k
    Cq = -ha * ha - ha * (p - a.p) / a.rho
    h = (-Bq + math.sqrt(Bq * Bq - 4.0 * A * Cq)) / (2.0 * A)
    rho = gam * p / ((gam - 1.0) * (h - 1.0))
    j2 = (p - a.p) / (ha / a.rho - h / rho)
    j = sign * math.sqrt(j2)
    ra2 = a.rho * a.rho * a.W * a.W
    Vs = (ra2 * a.v + j * math.sqrt(j2 + ra2 * (1.0 - a.v * a.v))) / (ra2 + j2)
    Ws = 1.0 / math.sqrt(1.0 - Vs * Vs)
    v = (ha * a.W * a.v + Ws * (p - a.p) / j) / (ha * a.W + (p - a.p) * (Ws * a.v / j + 1.0 / (a.rho * a.W)))
    return State(rho, p, v, gam), Vs


def _behind(a: State, p, sign):
    if p > a.p:
        s, _ = _shock(a, p, sign)
        return s
    return _rarefaction(a, p, sign)


def star_pressure(L: State, R: State):
    """the pressure of the intermediate states (bisection in log p)"""
    f = lambda p: _behind(L, p, -1).v - _behind(R, p, +1).v
    lo, hi = 1e-12 * min(L.p, R.p), 1e6 * max(L.p, R.p)
    flo = f(lo)
    for _ in range(300):
        mid = math.sqrt(lo * hi)
        fm = f(mid)
        if (fm > 0) == (flo > 0):
            lo, flo = mid, fm
        else:
            hi = mid
        if hi / lo - 1.0 < 1e-15:
            break
    return math.sqrt(lo * hi)


def _fan_state(a: State, xi, sign):
    """the state inside a rarefaction fan of family sign at similarity coordinate xi:
    the characteristic speed (v + sign cs)/(1 + sign v cs) equals xi, on the wave's
    adiabat and Riemann invariant (bisection in p)"""
    gam = a.gam
    lo, hi = 1e-14 * a.p, a.p
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        s = _rarefaction(a, mid, sign)
        lam = (s.v + sign * s.cs) / (1.0 + sign * s.v * s.cs)
        # deeper into a left fan (lower p) the characteristic speed rises
        if (lam < xi) == (sign < 0):
            hi = mid
        else:
            lo = mid
    return _rarefaction(a, 0.5 * (lo + hi), sign)


def solution(L: State, R: State):
    """a function xi -> (rho, p, v) of the similarity variable x / t"""
    ps = star_pressure(L, R)
    waves = []
    for a, sign in ((L, -1), (R, +1)):
        if ps > a.p:
            s, Vs = _shock(a, ps, sign)
            waves.append(("shock", s, Vs, Vs))
        else:
            s = _rarefaction(a, ps, sign)
            head = (a.v + sign * a.cs) / (1.0 + sign * a.v * a.cs)
            tail = (s.v + sign * s.cs) / (1.0 + sign * s.v * s.cs)
            waves.append(("fan", s, head, tail))
    (kl, sl, hl, tl), (kr, sr, hr, tr) = waves
    vc = 0.5 * (sl.v + sr.v)

    def at(xi):
        if xi < vc:
            if xi < hl:
                s = L
            elif kl == "fan" and xi < tl:
                s = _fan_state(L, xi, -1)
            else:
                s = sl
        else:
            if xi > hr:
                s = R
            elif kr == "fan" and xi > tr:
                s = _fan_state(R, xi, +1)
            else:
                s = sr
        return s.rho, s.p, s.v

    return at, ps, vc
