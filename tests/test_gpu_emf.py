"""GPU upwinded edge EMFs (Gardiner & Stone 2005 contact upwinding of the corner EMF,
the option Sec. 2.5 names) against the oracle: a uniform torus with its polar axis, a
multi-block periodic box, and refined, time-stepped layouts whose fine-EMF corrections
and EMF registers carry the upwinded values; the same bar as the averaged EMF."""
import sys

import numpy as np
import pytest

from paper_1912_10192_amd import configs, grmhd, initdata
from tests.helpers import mink_cfg, random_periodic_state
from tests.test_gpu_amr import run_pair
from tests.test_gpu_parity import TOL, check_trajectory
from tests.test_oracle_amr import band_blocks
from tests.test_planner_amr_cpu import polar_bands

pytestmark = pytest.mark.gpu
UPWIND = grmhd.EMF_UPWIND


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("recon,riemann", [(0, 0), (1, 1)])
def test_torus_uniform_upwinded_emf_trajectory(recon, riemann):
    n = (32, 32, 16)
    cfg = dict(configs.scaled(configs.TORUS_UNIFORM, n, block=(16, 16, 8), ng=3,
                              recon=recon), riemann=riemann, emf=UPWIND)
    state = initdata.torus_state(n, **configs.TORUS_INIT)
    grid, _ = check_trajectory(cfg, state, 3)
    a, r = grid.divb()
    say(f"  divB rel {r:.2e}")
    assert r < 1e-12


def test_periodic_box_upwinded_emf_blocks_bit_exact():
    """a 24x16x8 box in one block and in twelve: identical bits, and parity"""
    n = (24, 16, 8)
    base = dict(mink_cfg(n, recon=1, riemann=1), emf=UPWIND)
    state = random_periodic_state(n, seed=11, amp=0.05, vamp=0.3, bamp=0.3)
    one, _ = check_trajectory(dict(base, block=n), state, 2)
    many, _ = check_trajectory(dict(base, block=(8, 8, 4)), state, 2)
    for x, y in zip(one.get_state(), many.get_state()):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("lats", [(0, 0), (0, 1)])
def test_refined_band_upwinded_emf_matches_oracle(lats):
    cfg = dict(mink_cfg((16, 32, 8), recon=1, riemann=1, L=(1.0, 2.0, 0.5)), emf=UPWIND)
    state = random_periodic_state(cfg["n"], seed=3, amp=0.05, vamp=0.2, bamp=0.2,
                                  dx=(1 / 16, 1 / 16, 1 / 16))
    grid, _, worst = run_pair(cfg, band_blocks(lats, (16, 32, 8)), state, 2)
    assert max(worst.values()) <= TOL, worst
    a, r = grid.divb()
    say(f"  divB rel {r:.2e}")
    assert r < 1e-12


@pytest.mark.parametrize("batched", [False, True])
def test_torus_polar_caps_upwinded_emf_matches_oracle(batched):
    eff = (32, 32, 16)
    cfg = dict(configs.scaled(configs.TORUS_UNIFORM, eff, ng=3), emf=UPWIND)
    state = initdata.torus_state(eff, **configs.TORUS_INIT)
    grid, _, worst = run_pair(cfg, polar_bands(eff, (0, 1)), state, 2, batched=batched)
    assert max(worst.values()) <= TOL, worst
    a, r = grid.divb()
    say(f"  divB rel {r:.2e}")
    assert r < 1e-12


def test_upwinded_emf_changes_the_solution():
    """the option is live: one step with and without it differs beyond rounding"""
    n = (16, 16, 8)
    state = random_periodic_state(n, seed=5, amp=0.05, vamp=0.3, bamp=0.3)
    out = {}
    for emf in (grmhd.EMF_AVERAGE, UPWIND):
        g = grmhd.Grid(dict(mink_cfg(n, recon=1, riemann=1), emf=emf), state=state)
        g.step(1)
        out[emf] = g.get_state()
    d = max(float(np.abs(a - b).max()) for a, b in zip(out[0], out[1]))
    assert d > 1e-6
