"""GPU time levels independent of refinement levels and face direction (paper Sec. 3.5,
Sec. 3.3), against the oracle's driver through the C ABI: time-level interfaces on x1,
x2 and x3 faces, edges and corners (a checkerboard of levels), three levels across x2 or
x3, refinement faces that are also time-level faces (the finer side faster, or slower),
and the Kerr-Schild torus on polar bands whose refined equatorial band runs one level
faster than the coarser bands around it (graph-captured cycles)."""
import sys

import numpy as np
import pytest

from paper_1912_10192_amd import configs, initdata
from tests.helpers import mink_cfg, random_periodic_state
from tests.test_gpu_amr import run_pair
from tests.test_gpu_parity import TOL
from tests.test_oracle_amr import band_blocks, checker_blocks

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def _check(grid, worst):
    assert max(worst.values()) <= TOL, worst
    a, r = grid.divb()
    say(f"  divB rel {r:.2e}")
    assert r < 1e-12


@pytest.mark.parametrize("batched", [False, True])
def test_checkerboard_of_time_levels_matches_oracle(batched):
    cfg = mink_cfg((8, 8, 8), recon=1, riemann=1)
    blocks = checker_blocks((8, 8, 8), (2, 2, 2), lambda i, j, k: (i + j + k) % 2)
    state = random_periodic_state(cfg["n"], seed=3, amp=0.05, vamp=0.2, bamp=0.2)
    grid, ref, worst = run_pair(cfg, blocks, state, 2, batched=batched)
    _check(grid, worst)


@pytest.mark.parametrize("axis", [1, 2])
def test_three_time_levels_across_x2_or_x3_match_oracle(axis):
    cfg = mink_cfg((8, 16, 16), recon=1, riemann=1, L=(1.0, 2.0, 2.0))
    lv = [0, 1, 2, 1]
    blocks = checker_blocks((8, 16, 16), (1, 4, 4), lambda i, j, k: lv[j] if axis == 1 else lv[k])
    state = random_periodic_state(cfg["n"], seed=4, amp=0.05, vamp=0.2, bamp=0.2,
                                  dx=(1 / 8, 1 / 8, 1 / 8))
    grid, ref, worst = run_pair(cfg, blocks, state, 2)
    _check(grid, worst)


@pytest.mark.parametrize("lats", [(1, 0, 1), (0, 1, 0)])
def test_refinement_faces_between_time_levels_match_oracle(lats):
    cfg = mink_cfg((16, 32, 8), recon=1, riemann=1, L=(1.0, 2.0, 0.5))
    blocks = band_blocks((0, 0), (16, 32, 8))
    for k, b in enumerate(blocks):
        band = k // 2
        b["lat"] = lats[band] + (k % 2 if lats[band] == 0 else 0)
    state = random_periodic_state(cfg["n"], seed=3, amp=0.05, vamp=0.2, bamp=0.2,
                                  dx=(1 / 16, 1 / 16, 1 / 16))
    grid, ref, worst = run_pair(cfg, blocks, state, 2)
    _check(grid, worst)


def test_torus_fast_refined_equator_matches_oracle():
    """three-level polar bands with the refined equatorial band one time level faster
    than the mid-latitude bands and polar caps (time levels on refinement faces in x2)"""
    eff = (32, 64, 32)
    cfg = configs.scaled(configs.TORUS_UNIFORM, eff, ng=3)
    blocks = configs.polar_smr_blocks(eff, 16, [0, 1])
    for b in blocks:
        b["lat"] = 0 if b["lev"] == (1, 1, 2) else 1
    state = initdata.torus_state(eff, **configs.TORUS_INIT)
    grid, ref, worst = run_pair(cfg, blocks, state, 2, batched=True)
    _check(grid, worst)


def test_cfg3_shaped_layout_matches_oracle():
    """the batched refinement + time-level workload's layout at reduced size: uneven
    blocks (16x8x8 and 32x16x16 in the equatorial band, 16x4x8 mid-latitude and 16x4x4
    cap blocks), phi halved per level toward each pole (3 levels), 4 time levels by
    radius, refinement faces between time levels; one graph-captured cycle with the
    learned guess off"""
    eff = (128, 64, 16)
    shapes = dict(eq_in=(16, 8, 8), eq_out=(32, 16, 16), mid=(16, 4, 8), cap=(16, 4, 4))
    blocks = configs.amr_lat_blocks(eff, shapes)
    assert max(b["lat"] for b in blocks) == 3
    cfg = configs.scaled(configs.TORUS_UNIFORM, eff, ng=3)
    state = initdata.torus_state(eff, **configs.TORUS_INIT)
    grid, ref, worst = run_pair(cfg, blocks, state, 1, batched=True)
    _check(grid, worst)
