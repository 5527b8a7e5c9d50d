"""Pins of the oracle's regrid (Sec. 3.3 refinement and derefinement of blocks, with the
divergence-free prolongation of Balsara 2001): the face field of every new block is
divergence-free, for refinement in every combination of dimensions, on Minkowski and
Kerr-Schild grids; a layout regridded to itself is unchanged; refining and derefining
returns the original state; linear data are prolonged and restricted exactly; and the
magnetic flux through every new coarse face is the sum over the fine faces it replaces."""
import math

import numpy as np
import pytest

from oracle.amr import AmrGrid
from oracle.regrid import regrid
from paper_1912_10192_amd import initdata
from tests.helpers import mink_cfg, random_periodic_state

PATTERNS = {"all": (1, 1, 1), "x1": (1, 0, 0), "x3": (0, 0, 1), "x1x2": (1, 1, 0),
            "x2x3": (0, 1, 1)}


def halves(N, fine, left_fine):
    """two blocks splitting x1 in half: one at levels `fine`, one at level 0"""
    out = []
    for side in (0, 1):
        lev = tuple(fine) if (side == 0) == left_fine else (0, 0, 0)
        Nl = [N[d] >> (fine[d] - lev[d]) for d in range(3)]
        out.append(dict(org=(side * Nl[0] // 2, 0, 0), n=(Nl[0] // 2, Nl[1], Nl[2]), lev=lev,
                        lat=0))
    return out


def _grid(cfg, blocks, state):
    og = AmrGrid(cfg, blocks)
    lmax = [max(b["lev"][d] for b in blocks) for d in range(3)]
    og.set_blocks(initdata.block_states(state, blocks, lmax))
    return og


def _spacing(cfg, b, Lmax):
    N = cfg["n"]
    return [(cfg["xhi"][d] - cfg["xlo"][d]) / (N[d] >> (Lmax[d] - b["lev"][d])) for d in range(3)]


def _div(st, dx):
    P, B1, B2, B3 = st
    return ((B1[..., 1:] - B1[..., :-1]) / dx[0] + (B2[:, 1:] - B2[:, :-1]) / dx[1]
            + (B3[1:] - B3[:-1]) / dx[2])


def _mink(N):
    return dict(mink_cfg(N), bc=(2, 2, 2, 2, 2, 2))


@pytest.mark.parametrize("pattern", list(PATTERNS))
def test_regridded_face_field_is_divergence_free(pattern):
    fine = PATTERNS[pattern]
    N = (16, 16, 8)
    cfg = _mink(N)
    state = random_periodic_state(N, seed=3, bamp=0.5)
    old = halves(N, fine, left_fine=True)
    new = halves(N, fine, left_fine=False)
    out = regrid(_grid(cfg, old, state), new)
    for b, st in zip(new, out):
        dx = _spacing(cfg, b, fine)
        scale = max(np.abs(x).max() for x in st[1:]) / min(dx)
        assert np.abs(_div(st, dx)).max() <= 1e-13 * scale, (pattern, b["lev"])


def test_regrid_on_kerr_schild_is_divergence_free():
    N = (16, 16, 8)
    cfg = dict(coords=1, a=0.9375, gam=4.0 / 3.0, n=N, ng=3, recon=1, riemann=1,
               xlo=(math.log(2.0), 0.3, 0.0), xhi=(math.log(20.0), math.pi - 0.3, 2 * math.pi),
               bc=(0, 0, 0, 0, 2, 2), courant=0.8, rho_fl_c=0.0, rho_fl_p=0.0, u_fl_c=0.0,
               u_fl_p=0.0, bsq_rho_max=1e300, bsq_u_max=1e300, gamma_max=1e150, tol=1e-12,
               maxit=50)
    dx0 = [(cfg["xhi"][d] - cfg["xlo"][d]) / N[d] for d in range(3)]
    state = random_periodic_state(N, seed=5, bamp=0.5, dx=dx0)
    for fine in ((1, 1, 1), (0, 1, 1)):
        out = regrid(_grid(cfg, halves(N, fine, True), state), halves(N, fine, False))
        for b, st in zip(halves(N, fine, False), out):
            dx = _spacing(cfg, b, fine)
            scale = max(np.abs(x).max() for x in st[1:]) / min(dx)
            assert np.abs(_div(st, dx)).max() <= 1e-13 * scale


def test_regrid_to_the_same_layout_is_a_copy():
    N = (16, 16, 8)
    cfg = _mink(N)
    state = random_periodic_state(N, seed=4)
    blocks = halves(N, (1, 1, 1), True)
    og = _grid(cfg, blocks, state)
    before = og.get_blocks()
    out = regrid(og, blocks)
    for a, b in zip(before, out):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("pattern", ["all", "x3", "x1x2"])
def test_refine_then_derefine_returns_the_original(pattern):
    fine = PATTERNS[pattern]
    N = (16, 16, 8)
    cfg = _mink(N)
    state = random_periodic_state(N, seed=6)
    coarse_right = halves(N, fine, True)
    fine_both = [coarse_right[0]]
    # the right half refined in place (the layout's finest level is kept)
    b = coarse_right[1]
    fine_both.append(dict(org=tuple(b["org"][d] << fine[d] for d in range(3)),
                          n=tuple(b["n"][d] << fine[d] for d in range(3)), lev=tuple(fine), lat=0))
    og = _grid(cfg, coarse_right, state)
    orig = og.get_blocks()
    mid = regrid(og, fine_both)
    og2 = AmrGrid(cfg, fine_both)
    og2.set_blocks(mid)
    back = regrid(og2, coarse_right)
    for a, bb in zip(orig, back):
        for x, y in zip(a, bb):
            assert np.abs(x - y).max() <= 1e-14 * max(1.0, np.abs(x).max())


def _cut(arrs, b):
    o, n = b["org"], b["n"]
    P, B1, B2, B3 = arrs
    return (P[:, o[2]:o[2] + n[2], o[1]:o[1] + n[1], o[0]:o[0] + n[0]].copy(),
            B1[o[2]:o[2] + n[2], o[1]:o[1] + n[1], o[0]:o[0] + n[0] + 1].copy(),
            B2[o[2]:o[2] + n[2], o[1]:o[1] + n[1] + 1, o[0]:o[0] + n[0]].copy(),
            B3[o[2]:o[2] + n[2] + 1, o[1]:o[1] + n[1], o[0]:o[0] + n[0]].copy())


def test_linear_data_are_prolonged_and_restricted_exactly():
    """primitives linear in the coordinates and the divergence-free linear field
    B = (a x2 + b x3, c x3 + e x1, f x1 + h x2), given as exact cell and face averages,
    come out as the exact averages at the new levels (away from the periodic seams,
    where the data jump)"""
    N = (16, 16, 16)
    cfg = _mink(N)
    L = [cfg["xhi"][d] - cfg["xlo"][d] for d in range(3)]
    a, b_, c, e, f, h = 0.3, -0.2, 0.5, 0.1, -0.4, 0.25
    pr = np.array([[1.0, 0.1, 0.2, -0.1], [0.5, -0.05, 0.1, 0.2], [0.1, 0.3, -0.2, 0.1],
                   [-0.2, 0.1, 0.1, 0.3], [0.05, -0.1, 0.2, 0.1]])

    def exact(lev):
        Nl = [N[d] >> (1 - lev[d]) for d in range(3)]
        dx = [L[d] / Nl[d] for d in range(3)]

        def grid(ext):
            k, j, i = np.meshgrid(np.arange(ext[2]), np.arange(ext[1]), np.arange(ext[0]),
                                  indexing="ij")
            return i, j, k

        i, j, k = grid(Nl)
        x = [(i + 0.5) * dx[0], (j + 0.5) * dx[1], (k + 0.5) * dx[2]]
        P = np.array([p[0] + p[1] * x[0] + p[2] * x[1] + p[3] * x[2] for p in pr])
        i, j, k = grid((Nl[0] + 1, Nl[1], Nl[2]))
        B1 = a * (j + 0.5) * dx[1] + b_ * (k + 0.5) * dx[2]
        i, j, k = grid((Nl[0], Nl[1] + 1, Nl[2]))
        B2 = c * (k + 0.5) * dx[2] + e * (i + 0.5) * dx[0]
        i, j, k = grid((Nl[0], Nl[1], Nl[2] + 1))
        B3 = f * (i + 0.5) * dx[0] + h * (j + 0.5) * dx[1]
        return (P, B1, B2, B3), Nl

    old = halves(N, (1, 1, 1), True)
    new = halves(N, (1, 1, 1), False)
    og = AmrGrid(cfg, old)
    og.set_blocks([_cut(exact(bl["lev"])[0], bl) for bl in old])
    out = regrid(og, new)
    for bl, st in zip(new, out):
        ex, Nl = exact(bl["lev"])
        want = _cut(ex, bl)
        o = bl["org"]
        for q in range(4):
            got = st[q]
            sel = []
            for ax, d in enumerate((2, 1, 0)):
                idx = np.arange(got.shape[got.ndim - 3 + ax]) + o[d]
                sel.append((idx >= 3) & (idx <= Nl[d] - 3))
            m = sel[0][:, None, None] & sel[1][None, :, None] & sel[2][None, None, :]
            diff = np.abs(got - want[q])[..., m]
            assert diff.size and diff.max() <= 1e-13, (bl["lev"], q, diff.max())


def test_restriction_keeps_the_flux_through_every_coarse_face():
    N = (16, 16, 8)
    cfg = _mink(N)
    state = random_periodic_state(N, seed=8, bamp=0.4)
    old = halves(N, (1, 1, 1), True)
    new = halves(N, (1, 1, 1), False)
    og = _grid(cfg, old, state)
    fineB = og.get_blocks()[0][1:]
    out = regrid(og, new)
    coarse = out[0]              # the left half, now at level 0
    B1f, B2f, B3f = fineB
    # flux through a coarse x1 face = mean of its 2x2 fine sub-faces (equal areas)
    want = 0.25 * (B1f[0::2, 0::2, 0::2] + B1f[0::2, 1::2, 0::2] + B1f[1::2, 0::2, 0::2]
                   + B1f[1::2, 1::2, 0::2])
    assert np.abs(coarse[1] - want).max() <= 1e-15 * np.abs(want).max()


def polar_quarters(N0):
    """four level-0 blocks over the whole sphere: x1 halves times theta halves, each
    spanning all of phi"""
    return [dict(org=(h * N0[0] // 2, j * N0[1] // 2, 0), n=(N0[0] // 2, N0[1] // 2, N0[2]),
                 lev=(0, 0, 0), lat=0) for j in range(2) for h in range(2)]


def six_child_layout(N0):
    """polar_quarters with every block split into six children (each touches an axis; a
    new finest level in every dimension)"""
    from paper_1912_10192_amd import configs

    q = polar_quarters(N0)
    return (configs.split_block(q[0], N0[1], "north") + configs.split_block(q[1], N0[1], "north")
            + configs.split_block(q[2], N0[1], "south") + configs.split_block(q[3], N0[1], "south"))


def polar_state(cfg, seed):
    """primitives of order one and a face field from a random edge potential that
    vanishes on the polar axis (A_1, A_3 ~ sin^2 theta), so that the axis faces carry no
    flux, as on a real spherical grid, and div B = 0 to rounding"""
    rng = np.random.default_rng(seed)
    N1, N2, N3 = cfg["n"]
    d = [(cfg["xhi"][x] - cfg["xlo"][x]) / cfg["n"][x] for x in range(3)]

    def smooth(x1, th, ph):
        a = rng.normal(size=5)
        return np.sin(th) ** 2 * (a[0] + a[1] * np.cos(ph + a[2]) + a[3] * np.sin(2 * x1 + a[4]) * np.cos(th))

    x1c = cfg["xlo"][0] + (np.arange(N1) + 0.5) * d[0]
    x1f = cfg["xlo"][0] + np.arange(N1 + 1) * d[0]
    thf = cfg["xlo"][1] + np.arange(N2 + 1) * d[1]
    phc = cfg["xlo"][2] + (np.arange(N3) + 0.5) * d[2]
    phf = cfg["xlo"][2] + np.arange(N3 + 1) * d[2]
    K, J, I = np.meshgrid(phf, thf, x1c, indexing="ij")
    A1 = smooth(I, J, K)                                  # [N3+1][N2+1][N1]
    K, J, I = np.meshgrid(phc, thf, x1f, indexing="ij")
    A3 = smooth(I, J, K)                                  # [N3][N2+1][N1+1]
    B1 = (A3[:, 1:, :] - A3[:, :-1, :]) / d[1]
    B2 = (A1[1:] - A1[:-1]) / d[2] - (A3[:, :, 1:] - A3[:, :, :-1]) / d[0]
    B3 = -(A1[:, 1:, :] - A1[:, :-1, :]) / d[1]
    P = np.empty((5, N3, N2, N1))
    P[0] = 1.0 + 0.1 * rng.random((N3, N2, N1))
    P[1] = 0.5
    P[2:] = 0.05 * rng.normal(size=(3, N3, N2, N1))
    return P, B1, B2, B3


def ks_sphere(N):
    return dict(coords=1, a=0.9375, gam=4.0 / 3.0, n=N, ng=3, recon=1, riemann=1,
                xlo=(math.log(1.5), 0.0, 0.0), xhi=(math.log(30.0), math.pi, 2 * math.pi),
                bc=(0, 0, 1, 1, 2, 2), courant=0.8, rho_fl_c=0.0, rho_fl_p=0.0, u_fl_c=0.0,
                u_fl_p=0.0, bsq_rho_max=1e300, bsq_u_max=1e300, gamma_max=1e150, tol=1e-12,
                maxit=50)


def test_six_child_polar_split_adds_a_level_divergence_free():
    """blocks on the polar axis split into six children (Sec. 3.4: the two along the axis
    keep the parent's phi level, the four further out are refined in all dimensions),
    which adds a finest level: every new block's face field is divergence-free, and the
    children along the axis take, along phi, their parent's values unrefined"""
    N0 = (16, 16, 8)
    cfg = ks_sphere(N0)
    state = polar_state(cfg, 9)
    old = polar_quarters(N0)
    og = AmrGrid(cfg, old)
    og.set_blocks(initdata.block_states(state, old, (0, 0, 0)))
    new = six_child_layout(N0)
    out = regrid(og, new)
    cfg1 = dict(cfg, n=tuple(2 * x for x in N0))
    for b, st in zip(new, out):
        dx = _spacing(cfg1, b, (1, 1, 1))
        scale = max(np.abs(x).max() for x in st[1:]) / min(dx)
        assert np.abs(_div(st, dx)).max() <= 1e-13 * scale, b
    # an axis child's x3 faces lie on its parent's x3 faces (no phi refinement): along
    # phi they are the parent's own values, prolonged only in r and theta
    assert new[0]["lev"] == (1, 1, 0) and out[0][3].shape[0] == N0[2] + 1


def _totals(cfg, blocks, states, N):
    """sum over interior cells of U (sqrt(-g) rho u^t, energy, momenta, entropy) times the
    coordinate cell volume"""
    import oracle

    L = [max(b["lev"][d] for b in blocks) for d in range(3)]
    tot = np.zeros(9)
    for b, (P, B1, B2, B3) in zip(blocks, states):
        dx = [(cfg["xhi"][d] - cfg["xlo"][d]) / (N[d] >> (L[d] - b["lev"][d])) for d in range(3)]
        vol = dx[0] * dx[1] * dx[2]
        for k in range(P.shape[1]):
            for j in range(P.shape[2]):
                x2 = cfg["xlo"][1] + (b["org"][1] + j + 0.5) * dx[1]
                for i in range(P.shape[3]):
                    x1 = cfg["xlo"][0] + (b["org"][0] + i + 0.5) * dx[0]
                    gcov, gcon, gdet, alpha, _ = oracle.geom_point(cfg, x1, x2)
                    B = [0.5 * (B1[k, j, i] + B1[k, j, i + 1]) / gdet,
                         0.5 * (B2[k, j, i] + B2[k, j + 1, i]) / gdet,
                         0.5 * (B3[k, j, i] + B3[k + 1, j, i]) / gdet]
                    tot += vol * oracle.prim_to_flux(P[:, k, j, i], B, gcov, gcon, gdet, alpha,
                                                     cfg["gam"], 0)
    return tot


def test_conserved_regrid_keeps_the_totals():
    """the conserved form of the regrid keeps the sums of sqrt(-g) rho u^t, of the energy
    and of the momenta over the grid, to the inversion's tolerance (the entropy tracer is
    recomputed from the new primitives, as after an update); the primitive form, whose
    children do not sum to their parent when sqrt(-g) varies across it, does not"""
    N = (16, 16, 8)
    cfg = ks_sphere(N)
    st = polar_state(cfg, 11)
    old = halves(N, (1, 1, 1), True)
    new = halves(N, (1, 1, 1), False)
    before = _totals(cfg, old, _grid(cfg, old, st).get_blocks(), N)
    q = [0, 1, 2, 3, 4]
    for conserved in (True, False):
        out = regrid(_grid(cfg, old, st), new, conserved=conserved)
        after = _totals(cfg, new, out, N)
        rel = np.abs(after[q] - before[q]).max() / np.abs(before[q]).max()
        if conserved:
            assert rel <= 1e-12, rel
        else:
            assert rel > 1e-3, rel
