"""Refinement during the run on the GPU (Sec. 3.3): the torus on coarse polar caps with
two time levels, regridded after every cycle on a density criterion (blocks whose densest
cell exceeds 0.3 split, up to level 2), then every block asked to merge back; the oracle
replays the same layouts with its own regrid and driver.  Parity after every cycle and
every regrid, and div B at rounding level throughout (against the grid's field scale: in
cells next to refinement faces whose own field is at rounding level, the EMF corrections
leave differences of that size, on the oracle's grid alike)."""
import sys

import pytest

from oracle.amr import AmrGrid
from oracle.regrid import regrid
from paper_1912_10192_amd import adapt, configs, initdata
from tests.test_gpu_amr import block_err
from tests.test_gpu_parity import TOL
from tests.test_planner_amr_cpu import polar_bands

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _div_scaled(grid):
    """max |div B| times the finest spacing over the largest face value"""
    a, _ = grid.divb()
    bmax = max(float(abs(x).max()) for st in grid.get_blocks() for x in st[1:])
    dx = min((grid.cfg["xhi"][d] - grid.cfg["xlo"][d]) / grid.cfg["n"][d] for d in range(3))
    return a * dx / bmax


def test_density_driven_refinement_and_merge_match_oracle():
    eff = (32, 32, 16)
    cfg = configs.scaled(configs.TORUS_UNIFORM, eff, ng=3)
    blocks = polar_bands(eff, (0, 1))
    state = initdata.torus_state(eff, **configs.TORUS_INIT)
    ref = AmrGrid(cfg, blocks)
    bs = initdata.block_states(state, ref.blocks, ref.Lmax)
    ref.set_blocks(bs)
    ag = adapt.AdaptiveGrid(cfg, blocks, bs, rho_refine=0.3, rho_coarsen=-1.0, every=1,
                            max_level=2, batched=1)
    layouts = [blocks]
    for c in range(3):
        ref.cycle()
        ag.step(1)
        new = [{k: v for k, v in b.items() if k != "parent"} for b in ag.layout.blocks]
        if len(ag.history) > len(layouts) - 1:
            say(f"[adapt] cycle {c}: regrid to {len(new)} blocks, levels "
                f"{sorted(set(tuple(b['lev']) for b in new))}")
            want = regrid(ref, new)
            ref = AmrGrid(dict(cfg, n=ag.grid.cfg["n"]), new)
            ref.set_blocks(want)
            layouts.append(new)
        e = block_err(ag.grid.get_blocks(), ref.get_blocks())
        say(f"  cycle {c}: " + " ".join(f"{k}={v:.1e}" for k, v in e.items()))
        assert max(e.values()) <= TOL, e
        assert _div_scaled(ag.grid) < 1e-13
    assert len(layouts) >= 2, "the criterion refined nothing"
    # every block asks to merge: the layout returns to the starting one
    ag.rho_coarsen = 1e30
    ag.rho_refine = 1e30
    assert ag.adapt()
    back = [{k: v for k, v in b.items() if k != "parent"} for b in ag.layout.blocks]
    key = lambda bl: sorted((tuple(b["lev"]), tuple(b["org"]), tuple(b["n"])) for b in bl)
    assert key(back) == key(blocks)
    want = regrid(ref, back)
    ref = AmrGrid(dict(cfg, n=ag.grid.cfg["n"]), back)
    ref.set_blocks(want)
    e = block_err(ag.grid.get_blocks(), ref.get_blocks())
    say("  after the merge " + " ".join(f"{k}={v:.1e}" for k, v in e.items()))
    assert max(e.values()) <= TOL, e
    ref.cycle()
    ag.step(1)
    e = block_err(ag.grid.get_blocks(), ref.get_blocks())
    say("  cycle after the merge " + " ".join(f"{k}={v:.1e}" for k, v in e.items()))
    assert max(e.values()) <= TOL, e
    assert _div_scaled(ag.grid) < 1e-13


def test_pooled_adaptive_run_is_identical_and_allocates_nothing():
    """the same refine-run-merge-run sequence with the state in two preallocated buffer
    sets (the grid alternating between them at each regrid): bit-identical to the run
    with fresh buffers, and torch's device allocations do not grow across the regrids"""
    import torch

    from paper_1912_10192_amd import grmhd

    eff = (32, 32, 16)
    cfg = configs.scaled(configs.TORUS_UNIFORM, eff, ng=3)
    blocks = polar_bands(eff, (0, 1))
    state = initdata.torus_state(eff, **configs.TORUS_INIT)
    lmax = [max(b["lev"][d] for b in blocks) for d in range(3)]
    bs = initdata.block_states(state, blocks, lmax)

    def run(pool_sizes, sizes_out=None):
        ag = adapt.AdaptiveGrid(cfg, blocks, bs, rho_refine=0.3, rho_coarsen=-1.0,
                                every=1000, max_level=2, batched=1, pool_sizes=pool_sizes)
        ag.step(1)
        torch.cuda.synchronize()
        mem0 = torch.cuda.memory_allocated()
        assert ag.adapt()
        refined = [{k: v for k, v in b.items() if k != "parent"} for b in ag.layout.blocks]
        if sizes_out is not None:
            sizes_out.append(grmhd.Desc(ag.grid.cfg, blocks=refined, batched=1).sizes())
        ag.step(1)
        assert ag.adapt(blocks)
        ag.step(1)
        torch.cuda.synchronize()
        return ag.grid.get_blocks(), torch.cuda.memory_allocated() - mem0

    sizes = [grmhd.Desc(cfg, blocks=blocks, batched=1).sizes()]
    fresh, _ = run(None, sizes)
    pool = tuple(max(s[k] for s in sizes) for k in range(3))
    say(f"[adapt] pool of {pool[0] + pool[1]} doubles and {pool[2]} work bytes, twice")
    pooled, grown = run(pool)
    say(f"  device allocations grew by {grown} bytes across the regrids")
    for a, b in zip(fresh, pooled):
        for x, y in zip(a, b):
            assert (x == y).all()
    assert grown <= 0


def test_block_courant_steps_match_oracle():
    """grmhd_block_dt: each block's own Courant step, against the oracle's step of the
    same block's state"""
    import numpy as np

    from paper_1912_10192_amd import grmhd

    eff = (32, 32, 16)
    cfg = configs.scaled(configs.TORUS_UNIFORM, eff, ng=3)
    blocks = polar_bands(eff, (0, 1))
    state = initdata.torus_state(eff, **configs.TORUS_INIT)
    ref = AmrGrid(cfg, blocks)
    bs = initdata.block_states(state, ref.blocks, ref.Lmax)
    ref.set_blocks(bs)
    g = grmhd.Grid(cfg, blocks=blocks, batched=1)
    g.set_blocks(bs)
    got = g.block_dt()
    want = np.array([ref.ctx[i].dt(ref.P[i], ref.B[i]) for i in range(len(blocks))])
    say(f"[adapt] block Courant steps {np.round(got, 5)}")
    assert np.abs(got - want).max() <= 1e-12 * want.max()


def test_refinement_with_courant_time_levels_matches_oracle():
    """refinement on density with the new layout's time levels set from the blocks'
    Courant steps (at most three levels, four substeps a cycle), then a cycle; the oracle
    replays the layouts and levels.  (Over further cycles the face fields of the weakly
    magnetised polar blocks, compared against their own block's largest value, drift
    past the 1e-11 bar by rounding growth, as in the other long trajectories.)"""
    eff = (32, 32, 16)
    cfg = configs.scaled(configs.TORUS_UNIFORM, eff, ng=3)
    blocks = polar_bands(eff, (0, 1))
    state = initdata.torus_state(eff, **configs.TORUS_INIT)
    ref = AmrGrid(cfg, blocks)
    bs = initdata.block_states(state, ref.blocks, ref.Lmax)
    ref.set_blocks(bs)
    ag = adapt.AdaptiveGrid(cfg, blocks, bs, rho_refine=0.3, rho_coarsen=-1.0, every=1000,
                            max_level=2, batched=1, lat_levels=3)
    ref.cycle()
    ag.step(1)
    assert ag.adapt()
    new = [{k: v for k, v in b.items() if k != "parent"} for b in ag.layout.blocks]
    lats = sorted(set(b["lat"] for b in new))
    say(f"[adapt] {len(new)} blocks, time levels {lats}")
    assert len(lats) >= 2
    want = regrid(ref, new)
    ref = AmrGrid(dict(cfg, n=ag.grid.cfg["n"]), new)
    ref.set_blocks(want)
    ref.cycle()
    ag.step(1)
    e = block_err(ag.grid.get_blocks(), ref.get_blocks())
    say("  cycle on the new layout: " + " ".join(f"{k}={v:.1e}" for k, v in e.items()))
    assert max(e.values()) <= TOL, e
    assert _div_scaled(ag.grid) < 1e-13


def test_adaptive_run_over_many_regrids_stays_physical():
    """the torus on the polar-cap layout, regridded every other cycle for twelve cycles on
    a density criterion that splits (rho_max > 0.3; twice here, down to level 3) and
    would merge (rho_max < 0.05), with time levels from the Courant steps and the state
    in two pooled buffer sets: no unphysical state, and div B small and not growing.  (Where a new block boundary lies
    on an old change of level, the two blocks' copies of the shared face come from old
    data of different levels and differ at the prolongation's truncation level; the
    first face synchronisation after the regrid leaves that difference as div B in the
    boundary cells of one side, constant afterwards: about 1e-12 of the field scale on
    this run.)"""
    from paper_1912_10192_amd import grmhd

    eff = (32, 32, 16)
    cfg = configs.scaled(configs.TORUS_UNIFORM, eff, ng=3)
    blocks = polar_bands(eff, (0, 1))
    state = initdata.torus_state(eff, **configs.TORUS_INIT)
    lmax = [max(b["lev"][d] for b in blocks) for d in range(3)]
    bs = initdata.block_states(state, blocks, lmax)
    # room for any layout of the run: three times what a uniform grid four times as fine
    # needs (the padding of many small blocks, their tables, ghost lists and LAT lists
    # grow with the number of blocks and levels)
    one = grmhd.Desc(dict(cfg, n=tuple(4 * x for x in eff)), blocks=[
        dict(org=(0, 0, 0), n=tuple(4 * x for x in eff), lev=(0, 0, 0), lat=0)]).sizes()
    sizes = tuple(3 * x for x in one)
    ag = adapt.AdaptiveGrid(cfg, blocks, bs, rho_refine=0.3, rho_coarsen=0.05, every=2,
                            max_level=3, batched=1, lat_levels=3, pool_sizes=sizes)
    divs, last_regrid = [], 0
    for c in range(12):
        nh = len(ag.history)
        st = ag.step(1)
        if len(ag.history) > nh:
            last_regrid = c
        assert st.bad_states == 0
        divs.append(_div_scaled(ag.grid))
    say(f"[adapt] regrids {len(ag.history)}, last after cycle {last_regrid}; scaled div B "
        + " ".join(f"{x:.1e}" for x in divs))
    assert len(ag.history) >= 2
    assert max(divs) < 1e-11
    steady = divs[last_regrid + 1:]
    assert max(steady) <= 1.1 * min(steady)
