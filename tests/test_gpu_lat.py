"""GPU local adaptive time-stepping against the oracle's LAT driver: time-interpolated
ghosts, flux/EMF registers, reflux and re-inversion, on a periodic Minkowski box with
three time levels and on the Kerr-Schild torus with levels by radius; graph-captured
cycles against directly launched ones."""
import sys

import numpy as np
import pytest

from oracle.lat import LatGrid
from paper_1912_10192_amd import configs, grmhd, initdata
from tests.helpers import mink_cfg, random_periodic_state
from tests.test_gpu_parity import TOL, parity_err

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run_pair(cfg, lats, state, cycles, batched=False):
    blocks = grmhd.uniform_blocks(cfg["n"], cfg["block"], lats=lats)
    say(f"[lat] n={cfg['n']} block={cfg['block']} lats={lats} cycles={cycles} batched={batched}")
    ref = LatGrid(cfg, blocks)
    ref.set_state(*state)
    grid = grmhd.Grid(cfg, state=state, blocks=blocks, batched=batched)
    worst = {}
    for c in range(cycles):
        ref.cycle()
        st = grid.step(1)
        e = parity_err(grid.get_state(), ref.get_state())
        say(f"  cycle {c}: dt {st.dt_min:.6e} vs {ref.dt_min * 1:.6e} steps/level "
            f"{list(st.steps_per_level)[:len(set(lats))]} " + " ".join(f"{k}={v:.1e}" for k, v in e.items()))
        for k, v in e.items():
            worst[k] = max(worst.get(k, 0.0), v)
    return grid, ref, worst


def test_minkowski_three_levels_matches_oracle():
    cfg = dict(mink_cfg((16, 6, 6), recon=1, riemann=1), block=(4, 3, 6))
    state = random_periodic_state(cfg["n"], seed=8, amp=0.05, vamp=0.2, bamp=0.2)
    grid, ref, worst = run_pair(cfg, [0, 1, 2, 1], state, 2)
    assert max(worst.values()) <= TOL, worst
    a, r = grid.divb()
    assert r < 1e-12


def test_torus_levels_by_radius_matches_oracle():
    cfg = configs.scaled(configs.TORUS_UNIFORM, (32, 16, 16), block=(8, 8, 8))
    state = initdata.torus_state(cfg["n"], **configs.TORUS_INIT)
    grid, ref, worst = run_pair(cfg, [0, 1, 2, 2], state, 2)
    assert max(worst.values()) <= TOL, worst
    a, r = grid.divb()
    say(f"  divB rel {r:.2e}")
    assert r < 1e-12


def test_graph_captured_cycle_is_bit_identical():
    cfg = configs.scaled(configs.TORUS_UNIFORM, (32, 16, 16), block=(8, 8, 8))
    state = initdata.torus_state(cfg["n"], **configs.TORUS_INIT)
    blocks = grmhd.uniform_blocks(cfg["n"], cfg["block"], lats=[0, 1, 2, 2])
    say("[lat] plain vs graph, 3 cycles")
    a = grmhd.Grid(cfg, state=state, blocks=blocks, batched=False)
    b = grmhd.Grid(cfg, state=state, blocks=blocks, batched=True)
    sa = a.step(3)
    sb = b.step(3)
    assert sa.real_zone_cycles == sb.real_zone_cycles
    for x, y in zip(a.get_state(), b.get_state()):
        assert np.array_equal(x, y)


def test_headline_path_matches_oracle():
    """the benchmarked path at reduced size: 32^3 blocks (the update runs brick by brick
    with LDS-staged column geometry), four time levels 0..3 along x1, the learned first
    guess on, the cycle captured as a graph with the three flux directions on three
    streams -- against the oracle's LAT driver (plain guess), two cycles"""
    from tests.test_gpu_mlp import _trained_blob

    cfg = configs.scaled(configs.TORUS_UNIFORM, (128, 32, 32), block=(32, 32, 32))
    state = initdata.torus_state(cfg["n"], **configs.TORUS_INIT)
    blob, _ = _trained_blob(configs.scaled(configs.TORUS_UNIFORM, (64, 32, 32),
                                           block=(32, 32, 32)),
                            initdata.torus_state((64, 32, 32), **configs.TORUS_INIT), steps=300)
    lats = [0, 1, 2, 3]
    blocks = grmhd.uniform_blocks(cfg["n"], cfg["block"], lats=lats)
    say(f"[lat headline] n={cfg['n']} block={cfg['block']} lats={lats} learned guess, graph")
    ref = LatGrid(cfg, blocks)
    ref.set_state(*state)
    grid = grmhd.Grid(cfg, state=state, blocks=blocks, batched=True, mlp_blob=blob)
    worst = {}
    for c in range(2):
        ref.cycle()
        st = grid.step(1)
        e = parity_err(grid.get_state(), ref.get_state())
        say(f"  cycle {c}: dt {st.dt_min:.6e} vs {ref.dt_min:.6e} learned starts "
            f"{st.mlp_guesses} steps/level {list(st.steps_per_level)[:4]} "
            + " ".join(f"{k}={v:.1e}" for k, v in e.items()))
        assert list(st.steps_per_level)[:4] == [8, 4, 2, 1]
        for k, v in e.items():
            worst[k] = max(worst.get(k, 0.0), v)
    assert max(worst.values()) <= TOL, worst
    a, r = grid.divb()
    say(f"  divB rel {r:.2e}")
    assert r < 1e-12
