"""GPU floors in the drift frame (Sec. 2.7, Ressler et al. 2017) against the oracle: the
torus, whose atmosphere the floors hold; a magnetised box whose density and internal
energy lie below the floors everywhere (every cell takes a parcel each stage); and the
refined layout with time levels, where the re-inversion after refluxing applies the
same floors; and a box whose field is too weak to hold energy (b^2 below the smallest
double), where the drift frame still follows the field's direction.  Same bar as every
trajectory test."""
import sys

import numpy as np
import pytest

from paper_1912_10192_amd import configs, grmhd, initdata
from tests.helpers import mink_cfg, random_periodic_state
from tests.test_gpu_amr import run_pair
from tests.test_gpu_parity import TOL, check_trajectory
from tests.test_planner_amr_cpu import polar_bands

pytestmark = pytest.mark.gpu
DRIFT = grmhd.FLOOR_DRIFT


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_torus_with_drift_frame_floors_matches_oracle():
    cfg = dict(configs.TORUS_TINY, block=(32, 32, 32), floor_frame=DRIFT)
    state = initdata.torus_state(cfg["n"], **configs.TORUS_INIT)
    grid, _ = check_trajectory(cfg, state, 4)
    a, r = grid.divb()
    assert r < 1e-12


def _starved_box():
    n = (16, 16, 8)
    cfg = dict(mink_cfg(n, recon=1, riemann=1), block=(8, 8, 8), floor_frame=DRIFT,
               rho_fl_c=0.5, u_fl_c=0.5, bsq_rho_max=50.0, bsq_u_max=750.0, gamma_max=50.0)
    P, B1, B2, B3 = random_periodic_state(n, seed=21, amp=0.05, vamp=0.4, bamp=0.3)
    P[0] *= 0.1         # a fifth of the density floor
    P[1] *= 0.1         # and of the energy floor
    return cfg, (P, B1, B2, B3)


def test_starved_box_with_drift_frame_floors_matches_oracle():
    cfg, state = _starved_box()
    check_trajectory(cfg, state, 3)


def _weak_field_box(scale):
    cfg, (P, B1, B2, B3) = _starved_box()
    return cfg, (P, B1 * scale, B2 * scale, B3 * scale)


def test_weak_field_box_with_drift_frame_floors_matches_oracle():
    cfg, state = _weak_field_box(1e-170)
    check_trajectory(cfg, state, 3)


def test_drift_frame_of_a_weak_field_follows_its_direction():
    """a field 1e-200 times the starved box's, whose b^2 underflows, still sets the drift
    frame: the states after two steps differ widely from those of the same box without a
    field, where the parcels move with the fluid"""
    out = []
    for scale in (1e-200, 0.0):
        cfg, state = _weak_field_box(scale)
        g = grmhd.Grid(cfg, state=state)
        g.step(2)
        out.append(g.get_state()[0])
    assert np.isfinite(out[0]).all() and np.isfinite(out[1]).all()
    assert np.abs(out[0] - out[1]).max() > 0.1 * np.abs(out[0]).max()


def test_drift_frame_floors_change_the_solution():
    cfg, state = _starved_box()
    out = {}
    for frame in (grmhd.FLOOR_FIXED, DRIFT):
        g = grmhd.Grid(dict(cfg, floor_frame=frame), state=state)
        g.step(1)
        out[frame] = g.get_state()
    d = max(float(np.abs(a - b).max()) for a, b in zip(out[0], out[1]))
    assert d > 1e-6


def test_refined_lat_torus_with_drift_frame_floors_matches_oracle():
    eff = (32, 32, 16)
    cfg = dict(configs.scaled(configs.TORUS_UNIFORM, eff, ng=3), floor_frame=DRIFT)
    state = initdata.torus_state(eff, **configs.TORUS_INIT)
    grid, _, worst = run_pair(cfg, polar_bands(eff, (0, 1)), state, 2, batched=True)
    assert max(worst.values()) <= TOL, worst
