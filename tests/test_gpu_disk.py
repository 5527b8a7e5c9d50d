"""GPU runs of the tilted thin disk workload (density-refined block tree with phi-halved
polar caps and time levels from the initial Courant step) through the C ABI: the reduced
layout against the oracle's driver for one graph-captured cycle, and the full effective
1024x384x384 grid (4104 blocks, 56.8 M cells, five time levels) for one cycle with its
properties."""
import os
import sys

import numpy as np
import pytest

from paper_1912_10192_amd import configs, grmhd, initdata
from tests.test_gpu_amr import run_pair
from tests.test_gpu_parity import TOL

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_reduced_disk_matches_oracle():
    n, block = (64, 96, 24), (16, 12, 6)
    cfg = configs.scaled(configs.DISK5, n, ng=3)
    blocks = configs.disk_blocks(n, block=block)
    bs = initdata.disk_block_states(cfg, blocks)
    from oracle.amr import AmrGrid
    g0 = AmrGrid(cfg, blocks)
    g0.set_blocks(bs)
    rel0 = max(g0.ctx[q].divb_rel(g0.B[q])[1] for q in range(len(blocks)))
    del g0
    say(f"[disk] reduced {n}: {len(blocks)} blocks, initial div B rel {rel0:.2e}")
    grid, ref, worst = run_pair(cfg, blocks, None, 1, batched=True, bs=bs)
    assert max(worst.values()) <= TOL, worst
    a, r = grid.divb()
    say(f"  divB rel {r:.2e}")
    assert r < max(100 * rel0, 1e-12)


def test_full_size_disk_properties():
    cfg = dict(configs.DISK5)
    blocks = configs.disk_blocks(cfg["n"])
    procs = min(16, len(os.sched_getaffinity(0)))
    bs = initdata.disk_block_states(cfg, blocks, procs=procs)
    say(f"[disk] full size {cfg['n']}: {len(blocks)} blocks, initial data on {procs} processes")
    grid = grmhd.Grid(cfg, blocks=blocks, batched=True)
    grid.set_blocks(bs)
    del bs
    # the toroidal field's vector potential cannot vanish around the disk (it carries the
    # toroidal flux), so outside the disk the face values are rounding residuals of O(1)
    # potential differences: their relative divergence is the initial field's own
    # rounding level, which the evolution must keep
    a0, r0 = grid.divb()
    st = grid.step(1)
    L = max(b["lat"] for b in blocks) + 1
    assert L == 5 and list(st.steps_per_level)[:L] == [16, 8, 4, 2, 1]
    cells = sum(b["n"][0] * b["n"][1] * b["n"][2] for b in blocks)
    assert st.lat_eff_zone_cycles == cells * 16
    eff = cfg["n"][0] * cfg["n"][1] * cfg["n"][2]
    assert st.amr_lat_eff_zone_cycles == eff * 16
    # the synthetic disk is not an equilibrium; the last-resort tier (keep the previous
    # state) stays a small fraction of the inversions
    inv = sum(st.c2p_tier)
    say(f"  inversions {inv}, last-resort tier {st.c2p_tier[4]} ({st.c2p_tier[4] / inv:.1e})")
    assert st.c2p_tier[4] <= 1e-4 * inv
    a, r = grid.divb()
    say(f"  dt {st.dt_min:.4e} tiers {list(st.c2p_tier)} floors {st.floor_hits} divB rel "
        f"{r:.2e} (initial {r0:.2e}), abs {a:.2e} (initial {a0:.2e})")
    assert r < max(100 * r0, 1e-11) and a < max(100 * a0, 1e-12)
    for P, *_ in grid.get_blocks():
        assert np.isfinite(P).all() and (P[0] > 0).all() and (P[1] > 0).all()
