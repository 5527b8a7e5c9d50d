"""GPU parity on the validation workloads of Sec. 7.2 and 7.3, on the MINMOD limiter and
on PPM with the shock flattener: 1D relativistic shock tubes on a Cartesian Minkowski
grid (the exact-solution problems of the oracle's own test, and seeded magnetised Riemann
problems with all three field and velocity components), with MINMOD, PPM and flattened
PPM reconstruction, split into blocks along x1; the torus with MINMOD and with the
flattener; and the off-centre spherical explosion through the polar axis, hydrodynamic
and magnetised, on uniform blocks and on coarse polar caps with time levels.  Same bar
as every trajectory test.  At strong shocks the limiters' switches turn rounding-level
differences (the kernels' reciprocals against the oracle's divisions) into differences
that grow about tenfold every five steps on the colliding streams with PPM, so
trajectories here run 25-30 steps."""
import sys

import numpy as np
import pytest

import oracle
from paper_1912_10192_amd import configs, initdata
from tests.test_gpu_amr import run_pair
from tests.test_gpu_parity import TOL, check_trajectory
from tests.test_oracle_shocktube import PROBLEMS, tube_cfg, tube_state
from tests.test_planner_amr_cpu import polar_bands

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("recon", [oracle.PLM_MINMOD, oracle.PPM, oracle.PPM_FLAT])
@pytest.mark.parametrize("name", list(PROBLEMS))
def test_hydro_shock_tube_matches_oracle(name, recon):
    N = 256
    L, R = PROBLEMS[name]
    cfg = dict(tube_cfg(N, recon), block=(64, 1, 1))
    state = tube_state(N, (L.rho, L.p, L.v, 0.0, 0.0), (R.rho, R.p, R.v, 0.0, 0.0))
    check_trajectory(cfg, state, 25)


def _random_riemann(seed):
    rng = np.random.default_rng(seed)

    def side():
        v = rng.uniform(-0.4, 0.4, 3)
        return (rng.uniform(0.2, 2.0), rng.uniform(0.05, 3.0), *v)

    b1 = rng.uniform(-1.0, 1.0)
    bl = (b1, *rng.uniform(-1.5, 1.5, 2))
    br = (b1, *rng.uniform(-1.5, 1.5, 2))
    return side(), side(), bl, br


@pytest.mark.parametrize("seed,recon,riemann", [(1, oracle.PLM_MINMOD, 1), (2, oracle.PPM, 1),
                                                 (3, oracle.PLM_MINMOD, 0), (4, oracle.PPM, 0),
                                                 (5, oracle.PPM_FLAT, 1), (6, oracle.PPM_FLAT, 0)])
def test_magnetised_riemann_problem_matches_oracle(seed, recon, riemann):
    N = 192
    left, right, bl, br = _random_riemann(seed)
    say(f"[tube] seed {seed}: left {np.round(left, 3)} right {np.round(right, 3)} "
        f"B {np.round(bl, 3)} / {np.round(br, 3)}")
    cfg = dict(tube_cfg(N, recon, riemann), block=(48, 1, 1))
    check_trajectory(cfg, tube_state(N, left, right, bl, br), 25)


@pytest.mark.parametrize("recon", [oracle.PLM_MINMOD, oracle.PPM_FLAT])
def test_torus_with_minmod_or_flattener_matches_oracle(recon):
    cfg = dict(configs.TORUS_TINY, recon=recon, ng=3, block=(32, 32, 32))
    state = initdata.torus_state(cfg["n"], **configs.TORUS_INIT)
    grid, _ = check_trajectory(cfg, state, 4)
    a, r = grid.divb()
    assert r < 1e-12


@pytest.mark.parametrize("magnetised", [False, True])
def test_off_centre_explosion_through_the_pole_matches_oracle(magnetised):
    """the explosion of Sec. 7.3 (centred at (3, 0, 10), radius 2) on a log-spherical
    Kerr-Schild grid in eight blocks: its edge starts 0.1 rad from the axis, so the blast
    works through the polar boundary during the 30 compared steps"""
    cfg = dict(configs.EXPLOSION)
    state = initdata.explosion_state(cfg["n"], cfg["xlo"], cfg["xhi"], magnetised=magnetised)
    grid, _ = check_trajectory(cfg, state, 30)
    a, r = grid.divb()
    say(f"  divB rel {r:.2e}")
    assert r < 1e-12


def test_off_centre_explosion_with_polar_refinement_and_time_levels():
    """the magnetised explosion on coarse polar caps (external refinement) with two time
    levels along x1, against the oracle's refinement driver"""
    cfg = dict(configs.EXPLOSION)
    state = initdata.explosion_state(cfg["n"], cfg["xlo"], cfg["xhi"], magnetised=True)
    grid, _, worst = run_pair(cfg, polar_bands(cfg["n"], (0, 1)), state, 3, batched=True)
    assert max(worst.values()) <= TOL, worst
    a, r = grid.divb()
    say(f"  divB rel {r:.2e}")
    assert r < 1e-12
