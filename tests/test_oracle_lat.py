"""Pins of the oracle's local adaptive time-stepping driver (CPU)."""
import math

import numpy as np
import pytest

import oracle
from oracle.lat import LatGrid
from paper_1912_10192_amd import configs, initdata
from tests.helpers import mink_cfg, pad_global, random_periodic_state, unpad_global


def x1_blocks(n, nb1, lats, nb2=1, nb3=1):
    b1, b2, b3 = n[0] // nb1, n[1] // nb2, n[2] // nb3
    out = []
    for k in range(nb3):
        for j in range(nb2):
            for i in range(nb1):
                out.append(dict(org=(i * b1, j * b2, k * b3), n=(b1, b2, b3), lat=lats[i],
                                lev=(0, 0, 0)))
    return out


def totals(cfg, state):
    P, B1, B2, B3 = state
    gcov, gcon, gdet, alpha, _ = oracle.geom_point(cfg, 0.0, 0.0)
    n = cfg["n"]
    tot = np.zeros(9)
    for k in range(n[2]):
        for j in range(n[1]):
            for i in range(n[0]):
                Bc = np.array([0.5 * (B1[k, j, i] + B1[k, j, i + 1]), 0.5 * (B2[k, j, i] + B2[k, j + 1, i]),
                               0.5 * (B3[k, j, i] + B3[k + 1, j, i])])
                tot += oracle.prim_to_flux(P[:, k, j, i], Bc, gcov, gcon, gdet, alpha, cfg["gam"], 0)
    return tot


def divb_max(cfg, state):
    _, B1, B2, B3 = state
    n = cfg["n"]
    dx = [(cfg["xhi"][d] - cfg["xlo"][d]) / n[d] for d in range(3)]
    d = ((B1[:, :, 1:] - B1[:, :, :-1]) / dx[0] + (B2[:, 1:, :] - B2[:, :-1, :]) / dx[1]
         + (B3[1:] - B3[:-1]) / dx[2])
    return np.abs(d).max()


def test_single_level_equals_global_stepping():
    cfg = mink_cfg((12, 6, 6), recon=1, riemann=1)
    state = random_periodic_state(cfg["n"], seed=4)
    lat = LatGrid(cfg, x1_blocks(cfg["n"], 3, [0, 0, 0], nb2=2))
    lat.set_state(*state)
    g = oracle.Grid(cfg)
    Pp, Bp = pad_global(cfg, *state)
    for _ in range(2):
        dt = lat.cycle()
        g.step(Pp, Bp, 1, dt_fixed=dt)
    a = lat.get_state()
    b = unpad_global(cfg, Pp, Bp)
    for x, y in zip(a, b):
        assert np.abs(x - y).max() <= 1e-13 * max(np.abs(y).max(), 1.0)


@pytest.mark.parametrize("lats", [[0, 1, 1, 0], [0, 1, 2, 1]])
def test_lat_conserves_and_keeps_divb_in_periodic_box(lats):
    cfg = mink_cfg((16, 6, 6), recon=1, riemann=1)
    state = random_periodic_state(cfg["n"], seed=8, amp=0.05, vamp=0.2, bamp=0.2)
    lat = LatGrid(cfg, x1_blocks(cfg["n"], 4, lats, nb2=2))
    lat.set_state(*state)
    t0 = totals(cfg, state)
    for _ in range(2):
        lat.cycle()
    s1 = lat.get_state()
    t1 = totals(cfg, s1)
    scale = np.abs(t0[:5]).max()
    assert np.abs(t1[:5] - t0[:5]).max() <= 2e-13 * scale, t1[:5] - t0[:5]
    assert divb_max(cfg, s1) < 1e-11
    assert lat.steps[0] == 2 * 2 ** (lat.L - 1)


def _wave_lat(N, lats):
    """fast wave along x1 through blocks of different time levels; one period"""
    from tests.test_oracle_grid import _eigen
    gam = 4.0 / 3.0
    P0 = np.array([1.0, 1.0, 0.0, 0.0, 0.0])
    Bvec = np.array([1.0, 1.0, 0.0])
    lam, R, tb = _eigen(P0, Bvec, gam, 1)
    v = lam[6]
    r = R[:, 6] / np.abs(R[:, 6]).max()
    cfg = mink_cfg((N, 4, 4), recon=1, riemann=1, L=(1.0, 4.0 / N, 4.0 / N))
    x = (np.arange(N) + 0.5) / N
    prof = np.cos(2 * np.pi * x)[None, None, :] * np.ones((4, 4, 1))
    P = np.empty((5, 4, 4, N))
    for c in range(5):
        P[c] = P0[c] + 1e-5 * r[c] * prof
    B1 = np.full((4, 4, N + 1), Bvec[0])
    b2 = Bvec[1] + 1e-5 * r[5] * prof
    B2 = np.concatenate([b2, b2[:, :1, :]], axis=1)
    b3 = Bvec[2] + 1e-5 * r[6] * prof
    B3 = np.concatenate([b3, b3[:1]], axis=0)
    lat = LatGrid(cfg, x1_blocks(cfg["n"], len(lats), lats))
    lat.set_state(P, B1, B2, B3)
    T = 1.0 / v
    while lat.t < T - 1e-12:
        lat.cycle()
    # compare with the analytic wave at the reached time
    ph = 2 * np.pi * (x - v * lat.t)
    want = P0[:, None] + 1e-5 * r[:5, None] * np.cos(ph)[None, :]
    got = lat.get_state()[0][:, 0, 0, :]
    return np.abs(got - want).mean(axis=1).sum()


def test_wave_through_time_level_jumps_second_order():
    e1 = _wave_lat(32, [0, 1, 2, 1])
    e2 = _wave_lat(64, [0, 1, 2, 1])
    order = math.log2(e1 / e2)
    assert order > 1.8, (e1, e2, order)


def test_torus_lat_runs_and_keeps_divb():
    cfg = configs.scaled(configs.TORUS_UNIFORM, (32, 16, 16), ng=3)
    state = initdata.torus_state(cfg["n"], **configs.TORUS_INIT)
    lat = LatGrid(cfg, x1_blocks(cfg["n"], 4, [0, 1, 2, 2], nb2=2, nb3=2))
    lat.set_state(*state)
    lat.cycle()
    s = lat.get_state()
    assert np.isfinite(s[0]).all()
    scale = max(np.abs(s[1]).max(), np.abs(s[2]).max()) / (math.pi / 16)
    assert divb_max(cfg, s) <= 1e-12 * scale
