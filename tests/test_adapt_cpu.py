"""Host logic of refinement during the run (Sec. 3.3, the six-child polar split of Sec.
3.4): flagged blocks split into eight children (six on the polar axis), the nesting rules
then split what they need, and every layout produced is one the planner accepts; merging
all children of a split returns the layout it came from."""
import numpy as np
import pytest

from paper_1912_10192_amd import adapt, configs, grmhd
from tests.test_oracle_regrid import ks_sphere, polar_quarters
from tests.test_planner_amr_cpu import polar_bands


def _accepts(cfg, layout, blocks):
    plain = [{k: v for k, v in b.items() if k != "parent"} for b in blocks]
    grmhd.Desc(dict(cfg, n=layout.n_eff(blocks)), blocks=plain).sizes()


def _torus_bands():
    eff = (32, 32, 16)
    cfg = configs.scaled(configs.TORUS_UNIFORM, eff, ng=3)
    return cfg, polar_bands(eff, (0, 1))


def test_polar_block_splits_into_six_and_the_layout_is_valid():
    N0 = (16, 16, 8)
    cfg = ks_sphere(N0)
    lay = adapt.Layout(cfg, polar_quarters(N0))
    new = lay.refine([1, 0, 0, 0])
    # the flagged block gives six children; the outer block on the same pole, which it
    # touches across the axis, is split too
    assert sum(1 for b in new if b.get("parent") is lay.blocks[0]) == 6
    assert sum(1 for b in new if b.get("parent") is lay.blocks[1]) == 6
    assert not lay.violations(new)
    _accepts(cfg, lay, new)


def test_refined_band_block_splits_into_eight():
    cfg, blocks = _torus_bands()
    lay = adapt.Layout(cfg, blocks)
    i = next(k for k, b in enumerate(blocks) if b["lev"] == (1, 1, 1))
    new = lay.refine([1 if k == i else 0 for k in range(len(blocks))])
    kids = [b for b in new if b.get("parent") is lay.blocks[i]]
    assert len(kids) == 8 and all(b["lev"] == (2, 2, 2) for b in kids)
    assert not lay.violations(new)
    _accepts(cfg, lay, new)


@pytest.mark.parametrize("seed", range(6))
def test_random_flags_give_layouts_the_planner_accepts(seed):
    rng = np.random.default_rng(seed)
    for cfg, blocks in (_torus_bands(), (ks_sphere((16, 16, 8)), polar_quarters((16, 16, 8)))):
        lay = adapt.Layout(cfg, blocks)
        flags = list(rng.integers(0, 2, len(blocks)))
        new = lay.refine(flags, max_level=3)
        assert not lay.violations(new)
        _accepts(cfg, lay, new)
        # a second round on the refined layout
        lay2 = adapt.Layout(dict(cfg, n=lay.n_eff(new)), new)
        new2 = lay2.refine(list(rng.integers(0, 2, len(new))), max_level=3)
        assert not lay2.violations(new2)
        _accepts(cfg, lay2, new2)


def test_merging_all_children_returns_the_layout():
    cfg, blocks = _torus_bands()
    lay = adapt.Layout(cfg, blocks)
    new = lay.refine([1] * len(blocks))
    back = lay.coarsen(new, [-1] * len(new))
    key = lambda bl: sorted((b["lev"], b["org"], b["n"]) for b in bl)
    assert key(back) == key(blocks)


def test_merge_that_would_break_nesting_is_skipped():
    cfg, blocks = _torus_bands()
    lay = adapt.Layout(cfg, blocks)
    i = next(k for k, b in enumerate(blocks) if b["lev"] == (1, 1, 1))
    once = lay.refine([1 if k == i else 0 for k in range(len(blocks))])
    lay2 = adapt.Layout(dict(cfg, n=lay.n_eff(once)), once)
    # refine one grandchild, then ask every child of the first split to merge
    j = next(k for k, b in enumerate(once) if b.get("parent") is lay.blocks[i])
    twice = lay2.refine([1 if k == j else 0 for k in range(len(once))], max_level=3)
    flags = [-1 if b.get("parent") is lay.blocks[i] else 0 for b in twice]
    out = lay2.coarsen(twice, flags)
    assert not lay2.violations(out)


@pytest.mark.parametrize("seed", range(4))
def test_grown_box_check_covers_the_cell_by_cell_check(seed):
    """the one-pass check (each block's box grown by its ghost depth) finds every pair the
    cell-by-cell emulation of the planner's ghost rules finds, on layouts with nesting
    violations planted by splitting random blocks twice without repair"""
    rng = np.random.default_rng(seed)
    for cfg, blocks in (_torus_bands(), (ks_sphere((16, 16, 8)), polar_quarters((16, 16, 8)))):
        lay = adapt.Layout(cfg, blocks)
        bl = list(lay.blocks)
        for _ in range(2):
            i = int(rng.integers(len(bl)))
            bl = lay.split(bl, i)
        fast, exact = set(lay.violations(bl)), set(lay.violations_cells(bl))
        assert exact <= fast, (exact - fast)


def test_time_levels_from_courant_steps_keep_contacts_within_one_level():
    """time levels from per-block Courant steps: the largest level whose step fits, then
    lowered where blocks in contact would differ by more than one; the layout with these
    levels is one the planner accepts"""
    cfg, blocks = _torus_bands()
    lay = adapt.Layout(cfg, blocks)
    rng = np.random.default_rng(3)
    new = lay.refine([1 if b["lev"] == (1, 1, 1) else 0 for b in blocks], max_level=3)
    dt = list(0.01 * 2.0 ** rng.uniform(0, 5, len(new)))
    lat = lay.time_levels(new, dt, 4)
    dmin = min(dt)
    for l, d in zip(lat, dt):
        assert 0 <= l <= 3 and 2 ** l * dmin <= d * (1 + 1e-12)
    for i, j, _ in lay.contacts(new):
        assert abs(lat[i] - lat[j]) <= 1
    _accepts(cfg, lay, [dict(b, lat=l) for b, l in zip(new, lat)])


def test_step_estimates_follow_the_block_tree():
    """kept blocks keep their Courant step, children (also grandchildren from nesting
    splits) take half their ancestor's per generation, merged parents twice their
    children's smallest"""
    cfg, blocks = _torus_bands()
    lay = adapt.Layout(cfg, blocks)
    dt = [float(i + 1) for i in range(len(blocks))]
    once = lay.refine([1 if i == 4 else 0 for i in range(len(blocks))], max_level=3)
    est = adapt.estimate_steps(lay.blocks, dt, once)
    for b, e in zip(once, est):
        if b.get("parent") is lay.blocks[4]:
            assert e == 0.5 * dt[4]
        elif "parent" not in b:
            assert e == dt[lay.blocks.index(b)]
    kid = next(k for k, b in enumerate(once) if b.get("parent") is lay.blocks[4])
    twice = lay.split(list(once), kid)
    est2 = adapt.estimate_steps(lay.blocks, dt, twice)
    assert 0.25 * dt[4] in est2
    back = adapt.estimate_steps(once, est, lay.coarsen(once, [-1] * len(once)))
    assert 2.0 * min(e for b, e in zip(once, est) if b.get("parent") is lay.blocks[4]) in back
