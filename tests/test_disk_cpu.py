"""The tilted thin disk workload on the CPU: the layout rules of its density-refined block
tree (2:1 refinement between blocks that touch, one refinement level across the polar
axis, phi-halved polar caps, time levels at most one apart), its full-size figures, and
pins of the initial data (closed-form density, exactly zero axis faces, a divergence-free
field whose coarse faces are the means of their fine sub-faces)."""
import math

import numpy as np
import pytest

import oracle
from oracle.amr import AmrGrid
from paper_1912_10192_amd import configs, grmhd, initdata

SMALL = dict(n=(64, 96, 24), block=(16, 12, 6))


def _boxes(blocks, lmax):
    lo = np.array([[b["org"][d] << (lmax[d] - b["lev"][d]) for d in range(3)] for b in blocks])
    hi = lo + np.array([[b["n"][d] << (lmax[d] - b["lev"][d]) for d in range(3)] for b in blocks])
    return lo, hi


def _rules(blocks, n):
    lmax = [max(b["lev"][d] for b in blocks) for d in range(3)]
    lo, hi = _boxes(blocks, lmax)
    T, P = configs._touching(lo, hi, n)
    tree = np.array([b["lev"][0] for b in blocks])
    lat = np.array([b["lat"] for b in blocks])
    assert not (T & (np.abs(tree[:, None] - tree[None, :]) > 1)).any()
    assert not (P & (tree[:, None] != tree[None, :])).any()
    assert not ((T | P) & (np.abs(lat[:, None] - lat[None, :]) > 1)).any()
    N2 = n[1]
    for b, l, h in zip(blocks, lo, hi):
        cap = h[1] <= N2 // 8 or l[1] >= N2 - N2 // 8
        assert b["lev"][0] == b["lev"][1]
        assert b["lev"][2] == b["lev"][0] + (0 if cap else 1)
    return lat


def test_small_disk_layout_rules():
    blocks = configs.disk_blocks(SMALL["n"], block=SMALL["block"])
    lat = _rules(blocks, SMALL["n"])
    assert sorted(set(lat)) == [0, 1, 2, 3]
    assert {b["lev"] for b in blocks} == {(1, 1, 2), (2, 2, 2), (2, 2, 3)}
    cfg = configs.scaled(configs.DISK5, SMALL["n"], ng=3)
    grmhd.Desc(cfg, blocks=blocks).sizes()


def test_full_size_disk_layout():
    """effective 1024x384x384 on r in [1.2, 1000]: 4104 blocks, 56.8 M cells, five time
    levels, accepted by the planner within a 61.5 GB work buffer"""
    blocks = configs.disk_blocks(configs.DISK5["n"])
    lat = _rules(blocks, configs.DISK5["n"])
    cells = sum(b["n"][0] * b["n"][1] * b["n"][2] for b in blocks)
    assert len(blocks) == 4104 and cells == 56770560
    assert sorted(set(lat)) == [0, 1, 2, 3, 4]
    prim, bface, work = grmhd.Desc(dict(configs.DISK5), blocks=blocks).sizes()
    assert (prim + bface) * 8 + work < 80e9


def test_disk_initial_data_pins():
    n = SMALL["n"]
    cfg = configs.scaled(configs.DISK5, n, ng=3)
    blocks = configs.disk_blocks(n, block=SMALL["block"])
    bs = initdata.disk_block_states(cfg, blocks)
    lmax = [max(b["lev"][d] for b in blocks) for d in range(3)]
    # closed-form density (disk frame tilted 45 degrees about x) at the densest disk cell
    i = max(range(len(blocks)), key=lambda q: bs[q][0][0].max())
    b = blocks[i]
    k, j, ii = np.unravel_index(np.argmax(bs[i][0][0]), bs[i][0][0].shape)
    Nl = [n[d] >> (lmax[d] - b["lev"][d]) for d in range(3)]
    x = [cfg["xlo"][d] + (b["org"][d] + q + 0.5) * (cfg["xhi"][d] - cfg["xlo"][d]) / Nl[d]
         for d, q in enumerate((ii, j, k))]
    r, th, ph = math.exp(x[0]), x[1], x[2]
    X = (r * math.sin(th) * math.cos(ph), r * math.sin(th) * math.sin(ph), r * math.cos(th))
    t = math.pi / 4
    xp, yp, zp = X[0], math.cos(t) * X[1] + math.sin(t) * X[2], -math.sin(t) * X[1] + math.cos(t) * X[2]
    R = math.hypot(xp, yp)
    sm = lambda u: min(max(u, 0.0), 1.0) ** 2 * (3.0 - 2.0 * min(max(u, 0.0), 1.0))
    taper = sm((R - 6.0) / 0.6) * sm((200.0 - R) / 20.0)
    Rs = np.linspace(6.0, 200.0, 200001)
    smv = lambda u: np.clip(u, 0.0, 1.0) ** 2 * (3.0 - 2.0 * np.clip(u, 0.0, 1.0))
    peak = float(np.max((Rs / 6.0) ** -1.5 * smv((Rs - 6.0) / 0.6) * smv((200.0 - Rs) / 20.0)))
    want = (R / 6.0) ** -1.5 * math.exp(-zp * zp / (2.0 * (0.03 * R) ** 2)) * taper
    got = bs[i][0][0][k, j, ii]
    assert abs(got / want * peak - 1.0) < 0.0101     # the seeded 1 % noise
    # exact zeros on the polar axis (x2 faces at theta = 0, pi)
    for b, (P, B1, B2, B3) in zip(blocks, bs):
        N2 = n[1] >> (lmax[1] - b["lev"][1])
        if b["org"][1] == 0:
            assert np.all(B2[:, 0, :] == 0.0)
        if b["org"][1] + b["n"][1] == N2:
            assert np.all(B2[:, -1, :] == 0.0)
    # divergence-free field, coarse copies of refinement faces = means of fine sub-faces
    g = AmrGrid(cfg, blocks)
    g.set_blocks(bs)
    rel = max(g.ctx[q].divb_rel(g.B[q])[1] for q in range(len(blocks)))
    assert rel < 1e-12
    from tests.test_oracle_amr import shared_face_mismatch
    assert shared_face_mismatch(g) < 1e-12


def test_pool_gives_the_same_blocks():
    n = SMALL["n"]
    cfg = configs.scaled(configs.DISK5, n, ng=3)
    blocks = configs.disk_blocks(n, block=SMALL["block"])[:6]
    a = initdata.disk_block_states(cfg, blocks)
    b = initdata.disk_block_states(cfg, blocks, procs=2)
    for x, y in zip(a, b):
        for u, v in zip(x, y):
            assert np.array_equal(u, v)
