"""GPU regrid (Sec. 3.3 refinement and derefinement, Balsara's divergence-free
prolongation of the face field) through the C ABI against the oracle's regrid: from
identical states on Minkowski and Kerr-Schild layouts, for refinement in every
combination of dimensions; and on the torus after two LAT cycles of the polar-cap
layout, regridded to its inverse (fine caps, coarse equatorial band) and run on for two
more cycles on both sides.  Every new layout keeps div B at rounding level."""
import sys

import pytest

from oracle.amr import AmrGrid
from oracle.regrid import regrid
from paper_1912_10192_amd import configs, grmhd, initdata
from tests.helpers import random_periodic_state
from tests.test_gpu_amr import block_err, run_pair
from tests.test_gpu_parity import TOL
from tests.test_oracle_regrid import PATTERNS, _mink, halves
from tests.test_planner_amr_cpu import polar_bands

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _pair(cfg, old, new, state):
    lmax = [max(b["lev"][d] for b in old) for d in range(3)]
    bs = initdata.block_states(state, old, lmax)
    ref = AmrGrid(cfg, old)
    ref.set_blocks(bs)
    want = regrid(ref, new)
    g = grmhd.Grid(cfg, blocks=old)
    g.set_blocks(bs)
    g2 = g.regrid(new)
    return g2, want


@pytest.mark.parametrize("pattern", list(PATTERNS))
def test_regrid_matches_oracle(pattern):
    fine = PATTERNS[pattern]
    N = (16, 16, 8)
    cfg = _mink(N)
    say(f"[regrid] minkowski halves, refinement {fine}")
    state = random_periodic_state(N, seed=3, bamp=0.5)
    g2, want = _pair(cfg, halves(N, fine, True), halves(N, fine, False), state)
    e = block_err(g2.get_blocks(), want)
    say("  " + " ".join(f"{k}={v:.1e}" for k, v in e.items()))
    assert max(e.values()) <= 1e-13, e
    a, r = g2.divb()
    assert r < 1e-13


def test_regrid_on_kerr_schild_matches_oracle():
    import math

    N = (16, 16, 8)
    cfg = dict(configs.scaled(configs.TORUS_UNIFORM, N, ng=3),
               xlo=(math.log(2.0), 0.3, 0.0), xhi=(math.log(20.0), math.pi - 0.3, 2 * math.pi),
               bc=(0, 0, 2, 2, 2, 2), rho_fl_c=0.0, u_fl_c=0.0)
    dx0 = [(cfg["xhi"][d] - cfg["xlo"][d]) / N[d] for d in range(3)]
    state = random_periodic_state(N, seed=5, bamp=0.5, dx=dx0)
    for fine in ((1, 1, 1), (0, 1, 1)):
        say(f"[regrid] kerr-schild halves, refinement {fine}")
        g2, want = _pair(cfg, halves(N, fine, True), halves(N, fine, False), state)
        e = block_err(g2.get_blocks(), want)
        say("  " + " ".join(f"{k}={v:.1e}" for k, v in e.items()))
        assert max(e.values()) <= 1e-12, e
        a, r = g2.divb()
        assert r < 1e-12


def inverted_bands(eff, lat=(0, 0)):
    """the polar-cap layout turned round: fine caps (split in x1 and x3), a coarse
    equatorial band (two x1 blocks)"""
    N1, N2, N3 = eff
    c1, c2, c3 = N1 // 2, N2 // 2, N3 // 2
    out = []
    for org2 in (0, 3 * N2 // 4):
        for h in range(2):
            for kk in range(2):
                out.append(dict(org=(h * N1 // 2, org2, kk * N3 // 2), n=(N1 // 2, N2 // 4, N3 // 2),
                                lev=(1, 1, 1), lat=lat[h]))
    for h in range(2):
        out.append(dict(org=(h * c1 // 2, c2 // 4, 0), n=(c1 // 2, c2 // 2, c3), lev=(0, 0, 0),
                        lat=lat[h]))
    return out


def test_torus_regrid_after_lat_cycles_matches_oracle():
    eff = (32, 32, 16)
    lats = (0, 1)
    cfg = configs.scaled(configs.TORUS_UNIFORM, eff, ng=3)
    state = initdata.torus_state(eff, **configs.TORUS_INIT)
    grid, ref, worst = run_pair(cfg, polar_bands(eff, lats), state, 2, batched=True)
    assert max(worst.values()) <= TOL, worst
    new = inverted_bands(eff, lats)
    say("[regrid] polar caps refined, equatorial band derefined")
    want = regrid(ref, new)
    g2 = grid.regrid(new)
    e = block_err(g2.get_blocks(), want)
    say("  after regrid " + " ".join(f"{k}={v:.1e}" for k, v in e.items()))
    assert max(e.values()) <= TOL, e
    a, r = g2.divb()
    say(f"  divB rel {r:.2e}")
    assert r < 1e-12
    ref2 = AmrGrid(cfg, new)
    ref2.set_blocks(want)
    for c in range(2):
        ref2.cycle()
        g2.step(1)
        e = block_err(g2.get_blocks(), ref2.get_blocks())
        say(f"  cycle {c} on the new layout " + " ".join(f"{k}={v:.1e}" for k, v in e.items()))
        assert max(e.values()) <= TOL, e
    a, r = g2.divb()
    assert r < 1e-12


def test_regrid_rejects_layouts_that_break_the_rules():
    N = (16, 16, 8)
    cfg = _mink(N)
    state = random_periodic_state(N, seed=3)
    old = halves(N, (1, 1, 1), True)
    lmax = (1, 1, 1)
    g = grmhd.Grid(cfg, blocks=old)
    g.set_blocks(initdata.block_states(state, old, lmax))
    # a different finest level
    bad = halves(N, (1, 1, 0), False)
    with pytest.raises(grmhd.GrmhdError, match="finest levels"):
        g.regrid(bad)
