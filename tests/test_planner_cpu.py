"""Host-side checks of libgrmhd.so that need no GPU: exported symbols, the planner's
geometry tables against the oracle's independent geometry, and the ghost gather
lists bit-exact against the oracle's sequential boundary fill."""
import math
import re

import numpy as np
import pytest

import oracle
from paper_1912_10192_amd import configs, grmhd
from tests.helpers import mink_cfg

HEADER = "include/grmhd.h"


def test_library_exports_every_declared_symbol():
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    text = open(os.path.join(root, HEADER)).read()
    declared = set(re.findall(r"^\s*(?:int|const char\*)\s+(grmhd_\w+)\s*\(", text, re.M))
    assert declared == set(grmhd.EXPORTS)
    L = grmhd.lib()
    for name in declared:
        assert hasattr(L, name), name


def test_invalid_descriptors_are_rejected():
    cfg = dict(configs.TORUS_TINY)
    d = grmhd.Desc(cfg)
    d.d.n_ghost = 1
    with pytest.raises(grmhd.GrmhdError, match="n_ghost"):
        d.sizes()
    d = grmhd.Desc(cfg)
    d.d.abi_version = 99
    with pytest.raises(grmhd.GrmhdError, match="abi_version"):
        d.sizes()
    d = grmhd.Desc(dict(cfg, ng=2, recon=1))
    with pytest.raises(grmhd.GrmhdError, match="PPM"):
        d.sizes()
    bad = grmhd.uniform_blocks(cfg["n"], cfg["n"])
    bad[0]["org"] = (1, 0, 0)
    with pytest.raises(grmhd.GrmhdError):
        grmhd.Desc(cfg, blocks=bad).sizes()


@pytest.mark.parametrize("coords", [0, 1])
def test_planner_geometry_matches_oracle(coords):
    a = 0.9375
    cfg = dict(mink_cfg((4, 4, 4))) if coords == 0 else dict(
        coords=1, a=a, gam=4 / 3, n=(8, 8, 8), ng=3, recon=1, riemann=1, bc=(0, 0, 1, 1, 2, 2),
        xlo=(0, 0, 0), xhi=(1, math.pi, 2 * math.pi))
    rng = np.random.default_rng(0)
    for _ in range(100):
        x1 = rng.uniform(math.log(1.1), math.log(80.0))
        x2 = rng.uniform(0.02, math.pi - 0.02)
        gcov, gcon, gdet, alpha, conn = oracle.geom_point(cfg, x1, x2)
        out, cn = grmhd.geometry_point(coords, a, x1, x2)
        want = [gcov[0, 0], gcov[0, 1], gcov[0, 3], gcov[1, 1], gcov[1, 3], gcov[2, 2], gcov[3, 3],
                gcon[0, 0], gcon[0, 1], gcon[1, 1], gcon[1, 3], gcon[2, 2], gcon[3, 3], gdet, alpha]
        scale = np.abs(want).max()
        assert np.allclose(out, want, rtol=1e-13, atol=1e-15 * scale)
        # every entry the planner treats as zero is zero in the oracle's general metric
        for (m, n) in [(0, 2), (1, 2), (2, 3)]:
            assert gcov[m, n] == 0.0
        for (m, n) in [(0, 2), (0, 3), (1, 2), (2, 3)]:
            assert abs(gcon[m, n]) <= 1e-15 * np.abs(gcon).max()
        pairs = [(m, n) for m in range(4) for n in range(m, 4)]
        for l in range(4):
            for p, (m, n) in enumerate(pairs):
                ref = conn[l, m, n]
                assert cn[l * 10 + p] == pytest.approx(ref, rel=1e-11, abs=1e-12 * np.abs(conn).max())


def _global_labels(cfg):
    """oracle-filled padded arrays whose interior holds unique labels; a face on a
    periodic seam is one face stored twice (normal index 0 and N), so both copies carry
    one label"""
    g = oracle.Grid(cfg)
    ng = cfg["ng"]
    N = cfg["n"]
    P, B = g.zeros()
    lab = np.arange(1, P[0].size + 1, dtype=float).reshape(P[0].shape)
    P[0] = lab
    P[3] = 1.0
    for c in range(3):
        B[c] = lab + (c + 1) * 1e7
        if cfg["bc"][2 * c] == oracle.BC_PERIODIC:
            lo = [slice(None)] * 3
            hi = [slice(None)] * 3
            lo[2 - c] = ng
            hi[2 - c] = ng + N[c]
            B[c][tuple(hi)] = B[c][tuple(lo)]
    g.fill_bc(P, B)
    return P, B


@pytest.mark.parametrize("case", ["torus", "mink"])
def test_ghost_maps_match_oracle_fill(case):
    if case == "torus":
        cfg = configs.scaled(configs.TORUS_TINY, (12, 8, 8), block=(6, 4, 4), ng=3, recon=1)
    else:
        cfg = dict(mink_cfg((8, 6, 4), ng=3), block=(4, 3, 4))
    desc = grmhd.Desc(cfg)
    P, B = _global_labels(cfg)
    ng = cfg["ng"]
    layouts = [desc.layout(b) for b in range(desc.d.n_blocks)]
    org = [tuple(desc.blocks[b].org) for b in range(desc.d.n_blocks)]

    def to_global(b, loc):
        _, (n1p, n2p, n3p) = layouts[b]
        I = loc % n1p
        J = (loc // n1p) % n2p
        K = loc // (n1p * n2p)
        return (K - ng + org[b][2] + ng, J - ng + org[b][1] + ng, I - ng + org[b][0] + ng)

    for what in range(4):
        ops = desc.plan_dump(what)
        assert len(ops) > 0
        arr = P[0] if what == 0 else B[what - 1]
        for dst_b, dst_loc, srcf, src_loc in ops:
            src_b = srcf & 0xFFFFFF
            flags = srcf >> 24
            want = arr[to_global(dst_b, dst_loc)]
            if flags & 8:
                assert want == 0.0
                continue
            got = arr[to_global(src_b, src_loc)]
            if what == 0:
                assert got == want
                flip = P[3][to_global(dst_b, dst_loc)] < 0
                assert bool(flags & 1) == flip
            else:
                sign = -1.0 if flags & 1 else 1.0
                assert sign * got == want


def test_lat_layout_checks():
    cfg = configs.scaled(configs.TORUS_UNIFORM, (32, 16, 16), block=(8, 8, 8))
    ok = grmhd.Desc(cfg, blocks=grmhd.uniform_blocks(cfg["n"], cfg["block"], lats=[0, 1, 2, 2]))
    ok.sizes()
    with pytest.raises(grmhd.GrmhdError, match="more than one"):
        grmhd.Desc(cfg, blocks=grmhd.uniform_blocks(cfg["n"], cfg["block"], lats=[0, 2, 2, 2])).sizes()
    bl = grmhd.uniform_blocks(cfg["n"], cfg["block"], lats=[0, 1, 1, 1])
    bl[-1]["lat"] = 0        # an x2/x3 neighbour at another level: time levels on any face
    grmhd.Desc(cfg, blocks=bl).sizes()
    assert grmhd.lat_levels_by_radius(configs.TORUS_UNIFORM, [2.4, 4.8, 9.6]) == [0, 0, 1, 2, 2, 3, 3, 3]


@pytest.mark.parametrize("lats", [[0, 1, 2, 1], [0, 0, 1, 2, 2, 3, 2, 1], [1, 0, 1, 2]])
def test_lat_schedule_matches_oracle_driver(lats):
    """the library's cycle schedule (which blocks step at which substep, slowest level
    first, and which slow blocks synchronise when) equals the order the oracle's driver
    executes, entry for entry"""
    from oracle.amr import AmrGrid
    n = (8 * len(lats), 6, 6)
    cfg = dict(mink_cfg(n, recon=1, riemann=1), block=(8, 3, 6))
    blocks = grmhd.uniform_blocks(cfg["n"], cfg["block"], lats=lats)
    desc = grmhd.Desc(cfg, blocks=blocks)
    mine = [tuple(int(x) for x in r) for r in desc.plan_dump(10)]
    ref = AmrGrid(cfg, blocks)
    from tests.helpers import random_periodic_state
    ref.set_state(*random_periodic_state(cfg["n"], seed=2, amp=0.02, vamp=0.05, bamp=0.05))
    ref.cycle()
    want = ref.trace
    # steps: identical sequence; syncs at a sync point: the same set (order-free)
    assert [t for t in mine if t[1] == 0] == [t for t in want if t[1] == 0]
    key = lambda t: (t[0], t[2], t[3])
    assert sorted((t for t in mine if t[1] == 1), key=key) == sorted((t for t in want if t[1] == 1), key=key)
    # and the sync points fall between the same steps
    pos = lambda seq: [(seq[i - 1][:2] if i else None, t[0]) for i, t in enumerate(seq) if t[1] == 1]
    assert sorted(set(pos(mine))) == sorted(set(pos(want)))
