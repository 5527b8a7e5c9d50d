"""Relativistic shock tubes (the validation of Sec. 7.2: a 1D Cartesian Minkowski grid,
MINMOD and PPM reconstruction, and PPM with the optional shock flattener of Sec. 2.1):
the oracle against the exact solution of the hydrodynamic Riemann problem
(tests/riemann_exact.py), on two synthetic problems of this suite's own choosing -- a hot blast into a cold medium (rarefaction, contact,
shock) and two colliding streams (two shocks).  The L1 error of the density over the
region no boundary signal reaches falls with resolution, and PPM is the more accurate
limiter.  The flattening coefficient and the flattened face values against their
definitions (Colella & Woodward 1984)."""
import numpy as np
import pytest

import oracle
from tests.helpers import mink_cfg, pad_global, unpad_global
from tests.riemann_exact import State, solution

GAM = 4.0 / 3.0
PROBLEMS = {
    "blast": (State(1.0, 5.0, 0.0, GAM), State(0.25, 0.05, 0.0, GAM)),
    "collide": (State(0.5, 1.0, 0.3, GAM), State(1.0, 0.2, -0.2, GAM)),
}


def tube_cfg(N, recon, riemann=1):
    """N cells on [0, 1] along x1 (one cell across x2, x3, periodic there), outflow ends"""
    return mink_cfg((N, 1, 1), recon=recon, riemann=riemann, L=(1.0, 1.0 / N, 1.0 / N),
                    bc=(0, 0, 2, 2, 2, 2), gam=GAM)


def tube_state(N, left, right, bl=(0.0, 0.0, 0.0), br=(0.0, 0.0, 0.0)):
    """primitives (rho, u_g, utilde^1..3) and face fields of a discontinuity at x = 1/2;
    left/right are (rho, p, v^1, v^2, v^3); bl/br the cell fields (B^1 must agree)"""
    x = (np.arange(N) + 0.5) / N
    P = np.zeros((5, 1, 1, N))
    lo = x < 0.5
    for side, m in ((left, lo), (right, ~lo)):
        rho, p = side[0], side[1]
        v = np.array(side[2:5])
        W = 1.0 / np.sqrt(1.0 - v @ v)
        P[0][..., m] = rho
        P[1][..., m] = p / (GAM - 1.0)
        for c in range(3):
            P[2 + c][..., m] = W * v[c]
    B1 = np.full((1, 1, N + 1), bl[0])
    B2 = np.zeros((1, 2, N))
    B3 = np.zeros((2, 1, N))
    for c, arr in ((1, B2), (2, B3)):
        val = np.where(lo, bl[c], br[c])
        arr[...] = val
    return P, B1, B2, B3


def run_tube(N, recon, left, right, T, cfl=0.4):
    cfg = tube_cfg(N, recon)
    g = oracle.Grid(cfg)
    Pp, Bp = pad_global(cfg, *tube_state(N, left, right))
    dt = cfl / N
    n = int(round(T / dt))
    g.step(Pp, Bp, n, dt)
    return unpad_global(cfg, Pp, Bp)[0], n * dt


def l1_error(N, recon, name, T=0.25):
    L, R = PROBLEMS[name]
    P, t = run_tube(N, recon, (L.rho, L.p, L.v, 0.0, 0.0), (R.rho, R.p, R.v, 0.0, 0.0), T)
    at, _, _ = solution(L, R)
    x = (np.arange(N) + 0.5) / N
    exact = np.array([at((xi - 0.5) / t)[0] for xi in x])
    inside = np.abs(x - 0.5) < 0.5 - t          # no signal from the boundaries yet
    return np.sum(np.abs(P[0][0, 0][inside] - exact[inside])) / np.sum(np.abs(exact[inside]))


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_shock_tube_converges_to_the_exact_solution(name):
    err = {}
    for recon in (oracle.PLM_MINMOD, oracle.PPM, oracle.PPM_FLAT):
        err[recon] = [l1_error(N, recon, name) for N in (100, 200, 400)]
        e = err[recon]
        assert e[1] < 0.7 * e[0] and e[2] < 0.7 * e[1], (recon, e)
        assert e[2] < 0.06, (recon, e)
    # PPM resolves the discontinuities more sharply than the diffusive MINMOD limiter
    assert err[oracle.PPM][2] < err[oracle.PLM_MINMOD][2]


def test_exact_solver_satisfies_the_jump_conditions():
    """the exact solution's shocks conserve mass, momentum and energy across them:
    V_s [U] = [F] for U = (rho W, rho h W^2 v, rho h W^2 - p)"""
    from tests.riemann_exact import _shock

    def cons(s):
        W, h = s.W, s.h
        return np.array([s.rho * W, s.rho * h * W * W * s.v, s.rho * h * W * W - s.p])

    def flux(s):
        W, h = s.W, s.h
        return np.array([s.rho * W * s.v, s.rho * h * W * W * s.v * s.v + s.p,
                         s.rho * h * W * W * s.v])

    for a in (State(1.0, 0.1, 0.0, GAM), State(0.5, 1.0, 0.3, GAM), State(2.0, 0.05, -0.4, GAM)):
        for sign in (-1, 1):
            for ratio in (1.5, 30.0, 1000.0):
                b, vs = _shock(a, ratio * a.p, sign)
                res = vs * (cons(b) - cons(a)) - (flux(b) - flux(a))
                assert np.abs(res).max() <= 1e-13 * np.abs(np.concatenate([flux(a), flux(b)])).max()


def test_flattening_coefficient_closed_forms():
    """zero in smooth flow, for weak jumps, in expansions and where the wider jump
    vanishes; 10 (dp1/dp2 - 0.75) clipped to [0, 1] at strong compressive jumps"""
    f = oracle.flatten
    smooth = 1.0 + 0.05 * np.arange(6.0)
    comp = np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0])      # velocity falling: compression
    assert f(smooth, comp, 2) == 0.0                       # jump 0.1 < 0.33 of 1.05
    step = np.array([1.0, 1.0, 1.0, 10.0, 10.0, 10.0])
    assert f(step, comp, 2) == 1.0                         # dp1 = dp2: 10 (1 - 0.75) > 1
    assert f(step, comp[::-1].copy(), 2) == 0.0            # expansion
    # an intermediate steepness: dp1 = u3 - u1 = 7, dp2 = u4 - u0 = 9, 10 (7/9 - 0.75)
    u = np.array([1.0, 2.0, 2.0, 9.0, 10.0, 10.0])
    r = 7.0 / 9.0
    assert f(u, comp, 2) == pytest.approx(min(1.0, max(0.0, 10.0 * (r - 0.75))), abs=1e-15)
    u = np.array([1.0, 1.0, 1.0, 3.0, 9.0, 9.0])           # dp1 = 2, dp2 = 8: 10 (0.25 - 0.75) < 0
    assert f(u, comp, 2) == 0.0


def test_flattened_ppm_limits():
    """no flattening is PPM; full flattening gives each cell's mean (first order); in
    between, the interface values blend linearly before the monotonisation"""
    rng = np.random.default_rng(6)
    for _ in range(200):
        a = rng.normal(size=6)
        assert oracle.recon_face_flat(a, 0.0, 0.0) == oracle.recon_face(oracle.PPM, a)
        l, r = oracle.recon_face_flat(a, 1.0, 1.0)
        assert l == a[2] and r == a[3]
    # smooth monotone data (no limiter acts): the blend of the cubic-exact face value and
    # the cell mean
    fx = lambda x: 1.0 + 0.1 * x + 0.004 * x ** 2
    F = lambda x: x + 0.05 * x ** 2 + 0.004 / 3 * x ** 3
    a = np.array([F(c + 0.5) - F(c - 0.5) for c in range(6)])
    l, _ = oracle.recon_face_flat(a, 0.3, 0.0)
    assert l == pytest.approx(0.3 * a[2] + 0.7 * fx(2.5), rel=1e-14)


def test_flattener_removes_the_overshoot_behind_colliding_shocks():
    L, R = PROBLEMS["collide"]
    at, _, _ = solution(L, R)
    peaks = {}
    for recon in (oracle.PPM, oracle.PPM_FLAT):
        P, t = run_tube(400, recon, (L.rho, L.p, L.v, 0.0, 0.0), (R.rho, R.p, R.v, 0.0, 0.0), 0.25)
        x = (np.arange(400) + 0.5) / 400
        inside = np.abs(x - 0.5) < 0.5 - t
        exact_max = max(at((xi - 0.5) / t)[0] for xi in x[inside])
        peaks[recon] = P[0][0, 0][inside].max() / exact_max
    assert peaks[oracle.PPM] > 1.002 and peaks[oracle.PPM_FLAT] < 1.001, peaks
