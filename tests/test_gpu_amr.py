"""GPU static refinement against the oracle's refinement driver: restriction and
prolongation ghosts, fine-flux and fine-EMF correction of the coarse side, fine-owned
shared faces, alone and together with local time stepping, on a periodic Minkowski box
and on the Kerr-Schild torus with coarse polar caps."""
import sys

import numpy as np
import pytest

from oracle.amr import AmrGrid
from paper_1912_10192_amd import configs, grmhd, initdata
from tests.helpers import mink_cfg, random_periodic_state
from tests.test_gpu_parity import TOL
from tests.test_oracle_amr import band_blocks
from tests.test_planner_amr_cpu import polar_bands

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def block_err(got, want):
    """rho pointwise relative, u_g relative to rho + u_g, velocities and fields norm-wise,
    over all blocks"""
    e = {}
    for (P, B1, B2, B3), (Q, C1, C2, C3) in zip(got, want):
        parts = {"rho": np.abs(P[0] - Q[0]) / np.abs(Q[0]),
                 "u": np.abs(P[1] - Q[1]) / (np.abs(Q[0]) + np.abs(Q[1]))}
        for k, name in ((2, "ut1"), (3, "ut2"), (4, "ut3")):
            parts[name] = np.abs(P[k] - Q[k]) / max(np.abs(Q[2:5]).max(), 1e-300)
        bmax = max(np.abs(C1).max(), np.abs(C2).max(), np.abs(C3).max(), 1e-300)
        for name, a, b in (("B1", B1, C1), ("B2", B2, C2), ("B3", B3, C3)):
            parts[name] = np.abs(a - b) / bmax
        for k, v in parts.items():
            e[k] = max(e.get(k, 0.0), float(v.max()))
    return e


def run_pair(cfg, blocks, state, cycles, batched=False, bs=None):
    """the GPU grid and the oracle's driver from one initial state (a global state on
    the finest grid, or per-block states bs), `cycles` cycles; the worst differences"""
    say(f"[amr] n={cfg['n']} blocks={len(blocks)} lats={[b['lat'] for b in blocks]} "
        f"cycles={cycles} batched={batched}")
    ref = AmrGrid(cfg, blocks)
    if bs is None:
        bs = initdata.block_states(state, ref.blocks, ref.Lmax)
    ref.set_blocks(bs)
    grid = grmhd.Grid(cfg, blocks=blocks, batched=batched)
    grid.set_blocks(bs)
    worst = {}
    for c in range(cycles):
        ref.cycle()
        st = grid.step(1)
        e = block_err(grid.get_blocks(), ref.get_blocks())
        say(f"  cycle {c}: dt {st.dt_min:.6e} vs {ref.dt_min:.6e} "
            + " ".join(f"{k}={v:.1e}" for k, v in e.items()))
        for k, v in e.items():
            worst[k] = max(worst.get(k, 0.0), v)
    return grid, ref, worst


@pytest.mark.parametrize("lats", [(0, 0), (0, 1)])
def test_minkowski_refined_band_matches_oracle(lats):
    cfg = mink_cfg((16, 32, 8), recon=1, riemann=1, L=(1.0, 2.0, 0.5))
    state = random_periodic_state(cfg["n"], seed=3, amp=0.05, vamp=0.2, bamp=0.2,
                                  dx=(1 / 16, 1 / 16, 1 / 16))
    grid, ref, worst = run_pair(cfg, band_blocks(lats, (16, 32, 8)), state, 2)
    assert max(worst.values()) <= TOL, worst
    a, r = grid.divb()
    say(f"  divB rel {r:.2e}")
    assert r < 1e-12


@pytest.mark.parametrize("lats", [(0, 0), (0, 1)])
def test_torus_coarse_polar_caps_match_oracle(lats):
    eff = (32, 32, 16)
    cfg = configs.scaled(configs.TORUS_UNIFORM, eff, ng=3)
    state = initdata.torus_state(eff, **configs.TORUS_INIT)
    grid, ref, worst = run_pair(cfg, polar_bands(eff, lats), state, 2)
    assert max(worst.values()) <= TOL, worst
    a, r = grid.divb()
    say(f"  divB rel {r:.2e}")
    assert r < 1e-12


def test_refined_graph_cycle_is_bit_identical():
    eff = (32, 32, 16)
    cfg = configs.scaled(configs.TORUS_UNIFORM, eff, ng=3)
    state = initdata.torus_state(eff, **configs.TORUS_INIT)
    blocks = polar_bands(eff, (0, 1))
    ref = AmrGrid(cfg, blocks)
    bs = initdata.block_states(state, ref.blocks, ref.Lmax)
    say("[amr] plain vs graph, 3 cycles")
    a = grmhd.Grid(cfg, blocks=blocks, batched=False)
    a.set_blocks(bs)
    b = grmhd.Grid(cfg, blocks=blocks, batched=True)
    b.set_blocks(bs)
    sa = a.step(3)
    sb = b.step(3)
    assert sa.real_zone_cycles == sb.real_zone_cycles
    for x, y in zip(a.get_blocks(), b.get_blocks()):
        for u, v in zip(x, y):
            assert np.array_equal(u, v)


def test_torus_three_level_polar_bands_match_oracle():
    """coarse mid-latitude bands (half resolution) and polar caps (a quarter in phi),
    with two time levels along x1"""
    eff = (32, 64, 32)
    cfg = configs.scaled(configs.TORUS_UNIFORM, eff, ng=3)
    state = initdata.torus_state(eff, **configs.TORUS_INIT)
    grid, ref, worst = run_pair(cfg, configs.polar_smr_blocks(eff, 16, [0, 1]), state, 2,
                                batched=True)
    assert max(worst.values()) <= TOL, worst
    a, r = grid.divb()
    say(f"  divB rel {r:.2e}")
    assert r < 1e-12


def test_full_size_refined_lat_grid_properties():
    """The 512x256x256-effective refined grid with four time levels as the batched
    workload specifies it (1344 blocks of 64x32x32, 32x16x16 and 16x8x8), one batched
    (graph-captured) cycle with the learned guess off: every cell finite, every inversion
    converged without the last-resort tier, div B at round-off, the schedule's step counts
    per level, and the refined-and-LAT-effective accounting."""
    cfg = dict(configs.TORUS_AMR3)
    blocks = configs.amr_lat_blocks(cfg["n"], lat_edges=cfg["lat_edges"])
    lats = sorted({b["lat"] for b in blocks})
    assert len(blocks) == 1344 and lats == [0, 1, 2, 3]
    say(f"[amr] full size {cfg['n']}, {len(blocks)} blocks, levels {lats}")
    state = initdata.torus_state(cfg["n"], **configs.TORUS_INIT)
    lmax = [max(b["lev"][d] for b in blocks) for d in range(3)]
    bs = initdata.block_states(state, blocks, lmax)
    del state
    grid = grmhd.Grid(cfg, blocks=blocks, batched=True)
    grid.set_blocks(bs)
    del bs
    st = grid.step(1)
    L = max(lats) + 1
    assert list(st.steps_per_level)[:L] == [2 ** (L - 1 - l) for l in range(L)]
    cells = sum(b["n"][0] * b["n"][1] * b["n"][2] for b in blocks)
    eff = cfg["n"][0] * cfg["n"][1] * cfg["n"][2]
    assert st.lat_eff_zone_cycles == cells * 2 ** (L - 1)
    assert st.amr_lat_eff_zone_cycles == eff * 2 ** (L - 1)
    assert st.c2p_tier[4] == 0
    a, r = grid.divb()
    say(f"  dt {st.dt_min:.4e} tiers {list(st.c2p_tier)} divB rel {r:.2e}")
    assert r < 1e-12
    for P, B1, B2, B3 in grid.get_blocks():
        assert np.isfinite(P).all() and (P[0] > 0).all() and (P[1] > 0).all()


def test_divb_stays_at_roundoff_over_100_cycles():
    """div B across refinement and time-level faces after 100 cycles (the torus with
    coarse polar caps and two time levels)"""
    eff = (32, 32, 16)
    cfg = configs.scaled(configs.TORUS_UNIFORM, eff, ng=3)
    state = initdata.torus_state(eff, **configs.TORUS_INIT)
    blocks = polar_bands(eff, (0, 1))
    lmax = [max(b["lev"][d] for b in blocks) for d in range(3)]
    grid = grmhd.Grid(cfg, blocks=blocks, batched=True)
    grid.set_blocks(initdata.block_states(state, blocks, lmax))
    st = grid.step(100)
    a, r = grid.divb()
    say(f"[amr] 100 cycles: t {st.t_sim:.3f} divB rel {r:.2e} tiers {list(st.c2p_tier)}")
    assert r < 1e-12
    for P, *_ in grid.get_blocks():
        assert np.isfinite(P).all()
