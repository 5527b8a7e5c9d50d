"""The planner's synchronisation tables checked against the oracle's on the CPU, entry
for entry (integer tables, bit-exact): refinement faces between blocks of one time level,
the faces each slower block refluxes from a faster neighbour, the edges whose dominant
holder is faster (time-integrated EMFs at the end of the slower step) and the edges whose
finest holder at the block's own time level is finer (EMFs replaced in each stage).
Layouts cover time levels on x1, x2 and x3 faces, edges and corners, refinement faces
within and across time levels, polar bands of a Kerr-Schild grid and periodic seams."""
import numpy as np
import pytest

from oracle.amr import AmrGrid
from paper_1912_10192_amd import configs, grmhd
from tests.helpers import mink_cfg
from tests.test_oracle_amr import band_blocks, checker_blocks


def _bands_across_levels(lats):
    blocks = band_blocks((0, 0), (16, 32, 8))
    for k, b in enumerate(blocks):
        band = k // 2
        b["lat"] = lats[band] + (k % 2 if lats[band] == 0 else 0)
    return blocks


def cases():
    mk = mink_cfg((16, 32, 8), recon=1, riemann=1, L=(1.0, 2.0, 0.5))
    box = mink_cfg((8, 8, 8), recon=1, riemann=1)
    slab = mink_cfg((8, 16, 16), recon=1, riemann=1, L=(1.0, 2.0, 2.0))
    ks = configs.scaled(configs.TORUS_UNIFORM, (32, 64, 32), ng=3)
    lv = [0, 1, 2, 1]
    fast_band = configs.polar_smr_blocks((32, 64, 32), 16, [0, 1])
    for b in fast_band:          # the refined equatorial band one level faster than the rest
        b["lat"] = 0 if b["lev"] == (1, 1, 2) else 1
    return {
        "bands-same-level": (mk, band_blocks((0, 0), (16, 32, 8))),
        "bands-x1-levels": (mk, band_blocks((0, 1), (16, 32, 8))),
        "bands-fine-faster": (mk, _bands_across_levels((1, 0, 1))),
        "bands-fine-slower": (mk, _bands_across_levels((0, 1, 0))),
        "checkerboard": (box, checker_blocks((8, 8, 8), (2, 2, 2), lambda i, j, k: (i + j + k) % 2)),
        "levels-across-x2": (slab, checker_blocks((8, 16, 16), (1, 4, 4), lambda i, j, k: lv[j])),
        "levels-across-x3": (slab, checker_blocks((8, 16, 16), (1, 4, 4), lambda i, j, k: lv[k])),
        "ks-polar-bands": (ks, configs.polar_smr_blocks((32, 64, 32), 16, [0, 1])),
        "ks-fast-equator": (ks, fast_band),
    }


def _loc(blocks, g, b, kji):
    np_ = [blocks[b]["n"][d] + 2 * g + 1 for d in range(3)]
    K, J, I = kji
    return (K * np_[1] + J) * np_[0] + I


@pytest.mark.parametrize("case", list(cases()))
def test_sync_tables_match_oracle(case):
    cfg, blocks = cases()[case]
    g = cfg["ng"]
    orc = AmrGrid(cfg, blocks)
    desc = grmhd.Desc(cfg, blocks=blocks)
    # refinement faces at one time level
    mine = [tuple(int(x) for x in r) for r in desc.plan_dump(9)]
    want = [(c, f, d, side) + tuple(e) + tuple(lo) + tuple(hi) for c, f, d, side, e, lo, hi in orc.links]
    assert mine == want
    # reflux faces
    mine = [tuple(int(x) for x in r[:6 + int(r[5])]) for r in desc.plan_dump(12)]
    want = []
    for b in range(len(blocks)):
        for d, side, f, D, subs in orc.reflux[b]:
            want.append((b, d, side, _loc(blocks, g, b, f), D, len(subs))
                        + tuple(_loc(blocks, g, D, s) for s in subs))
    assert mine == want
    # sync edges and stage edges
    for what, table in ((13, orc.sync_edges), (14, orc.stage_edges)):
        mine = [tuple(int(x) for x in r[:5 + int(r[4])]) for r in desc.plan_dump(what)]
        want = []
        for b in range(len(blocks)):
            for a, e, D, subs in table[b]:
                want.append((b, a, _loc(blocks, g, b, e), D, len(subs))
                            + tuple(_loc(blocks, g, D, s) for s in subs))
        assert mine == want, what


def test_cases_exercise_every_table():
    got = {}
    for case, (cfg, blocks) in cases().items():
        desc = grmhd.Desc(cfg, blocks=blocks)
        got[case] = [len(desc.plan_dump(w)) for w in (9, 12, 13, 14)]
    assert got["checkerboard"][1] == 4 * 6 * 16 and got["checkerboard"][2] > 0
    assert got["bands-fine-faster"][1] > 0 and got["bands-fine-slower"][1] > 0
    assert got["ks-fast-equator"][1] > 0 and got["ks-fast-equator"][2] > 0
    assert got["ks-polar-bands"][0] > 0 and got["ks-polar-bands"][3] > 0


def test_time_levels_two_apart_across_a_corner_are_rejected():
    cfg = mink_cfg((8, 8, 8), recon=1, riemann=1)
    ok = checker_blocks((8, 8, 8), (2, 2, 2), lambda i, j, k: (i + j + k) % 2)
    grmhd.Desc(cfg, blocks=ok).sizes()
    # levels 0 and 2 on diagonally opposite blocks only (they meet at a corner)
    bad = checker_blocks((8, 8, 8), (2, 2, 2), lambda i, j, k: 1 + (i == j == k == 1) - (i == j == k == 0))
    with pytest.raises(grmhd.GrmhdError, match="more than one"):
        grmhd.Desc(cfg, blocks=bad).sizes()


MEAN = np.dtype([("dst", "<i8"), ("src", "<i8", 4), ("n", "<i4"), ("ncomp", "<i4"),
                 ("dstride", "<i4"), ("sstride", "<i4"), ("kind", "<i4"), ("pad", "<i4")])
REG = np.dtype([("src", "<i8"), ("slot", "<i4"), ("kind", "<i4"), ("stride", "<i4"), ("pad", "<i4")])
FTERM = np.dtype([("mine", "<i4"), ("th", "<i4", 4), ("nth", "<i4"), ("sgn", "<i4"), ("pad", "<i4"),
                  ("dx", "<f8")])
SCELL = np.dtype([("blk", "<i4"), ("loc", "<i4"), ("nt", "<i4"), ("pad", "<i4"), ("t", FTERM, 3)])
ETERM = np.dtype([("mine", "<i4"), ("th", "<i4", 2), ("nth", "<i4"), ("sgn", "<i4"), ("pad", "<i4"),
                  ("dx", "<f8")])
SFACE = np.dtype([("blk", "<i4"), ("comp", "<i4"), ("loc", "<i4"), ("nt", "<i4"), ("cblk", "<i4"),
                  ("ncopy", "<i4"), ("csrc", "<i4", 4), ("t", ETERM, 4)])


@pytest.mark.parametrize("case", list(cases()))
def test_device_lists_stay_in_bounds(case):
    """every element index of the uploaded lists lies inside its block's part of the array
    it addresses, every register slot inside the registers, every sync cell in a block's
    interior and every corrected face on or inside its block's boundary"""
    cfg, blocks = cases()[case]
    g = cfg["ng"]
    desc = grmhd.Desc(cfg, blocks=blocks)
    nb = len(blocks)
    lay = [desc.layout(b) for b in range(nb)]
    off = np.array([o for o, _ in lay])
    vol = np.array([int(np.prod(npd)) for _, npd in lay])

    def owner(elem, nv):
        b = np.searchsorted(nv * off, elem, side="right") - 1
        assert 0 <= b < nb
        return b

    def inside(elem, nv, ncomp, stride):
        b = owner(elem, nv)
        lo, hi = nv * off[b], nv * (off[b] + vol[b])
        assert lo <= elem and elem + (ncomp - 1) * stride < hi
        if ncomp > 1:
            assert stride == vol[b]

    for what in (15, 16):
        items = desc.plan_raw(what).view(MEAN)
        for it in items:
            assert it["n"] in (1, 2, 4)
            nv = 24 if it["kind"] == 0 else 3
            assert it["ncomp"] == (8 if it["kind"] == 0 else 1)
            inside(int(it["dst"]), nv, int(it["ncomp"]), int(it["dstride"]))
            for i in range(it["n"]):
                inside(int(it["src"][i]), nv, int(it["ncomp"]), int(it["sstride"]))
    regs = desc.plan_raw(17).view(REG)
    nf = int((regs["kind"] == 0).sum())
    ne = int((regs["kind"] == 1).sum())
    assert sorted(regs["slot"][regs["kind"] == 0]) == list(range(nf))
    assert sorted(regs["slot"][regs["kind"] == 1]) == list(range(ne))
    for r in regs:
        if r["kind"] == 0:
            inside(int(r["src"]), 24, 8, int(r["stride"]))
        else:
            inside(int(r["src"]), 3, 1, 0)

    def coords(b, loc):
        npd = lay[b][1]
        return loc % npd[0], (loc // npd[0]) % npd[1], loc // (npd[0] * npd[1])

    cells = desc.plan_raw(18).view(SCELL)
    seen = set()
    for c in cells:
        b, loc = int(c["blk"]), int(c["loc"])
        assert (b, loc) not in seen
        seen.add((b, loc))
        x = coords(b, loc)
        assert all(g <= x[d] < g + blocks[b]["n"][d] for d in range(3))
        assert 0 <= c["nt"] <= 3
        for t in c["t"][:c["nt"]]:
            assert 0 <= t["mine"] < nf and 1 <= t["nth"] <= 4
            assert all(0 <= s < nf for s in t["th"][:t["nth"]]) and t["dx"] > 0
    faces = desc.plan_raw(19).view(SFACE)
    seen = set()
    for f in faces:
        b, comp, loc = int(f["blk"]), int(f["comp"]), int(f["loc"])
        assert (b, comp, loc) not in seen
        seen.add((b, comp, loc))
        x = coords(b, loc)
        assert all(g <= x[d] <= g + blocks[b]["n"][d] - (0 if d == comp else 1) for d in range(3))
        if f["ncopy"] > 0:
            cb = int(f["cblk"])
            assert 0 <= cb < nb and all(0 <= s < vol[cb] for s in f["csrc"][:f["ncopy"]])
        assert 0 <= f["nt"] <= 4
        for t in f["t"][:f["nt"]]:
            assert 0 <= t["mine"] < ne and all(0 <= s < ne for s in t["th"][:t["nth"]])
