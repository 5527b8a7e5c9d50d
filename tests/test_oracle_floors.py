"""Pins of the oracle's floors (Sec. 2.7): at fixed utilde the minima are set exactly and
the velocity is kept; in the drift frame (Ressler et al. 2017) the missing mass and
energy arrive as a parcel moving with the field's drift frame, so that
  * without a field, or for a flow across the field, the drift frame is the fluid frame:
    the velocity is kept and rho, u_g become the minima (the stress tensor is linear in
    rho and u_g at a fixed velocity);
  * for a flow along the field the drift frame is at rest: the conserved momentum is
    unchanged, the added energy is the parcel's rest energy, and the flow slows down;
  * in general the new state's conserved vector is the old one plus the parcel's."""
import math

import numpy as np
import pytest

import oracle
from tests.helpers import mink_cfg

GAM = 4.0 / 3.0


def _mink_point():
    cfg = mink_cfg((4, 4, 4))
    return oracle.geom_point(cfg, 0.3, 0.4)


def _ks_point(rng):
    cfg = dict(coords=1, a=0.9375, gam=GAM, n=(8, 8, 8), ng=3, recon=1, riemann=1,
               bc=(0, 0, 1, 1, 2, 2), xlo=(0, 0, 0), xhi=(1, math.pi, 2 * math.pi))
    return oracle.geom_point(cfg, rng.uniform(math.log(2.0), math.log(40.0)),
                             rng.uniform(0.3, math.pi - 0.3))


def _cons(P, B, g):
    gcov, gcon, gdet, alpha, _ = g
    return oracle.prim_to_flux(P, B, gcov, gcon, gdet, alpha, GAM, 0)


def _four_vectors(P, B, gcov, gcon, alpha):
    """u^mu from utilde (normal-observer frame) and b^mu from the cell field"""
    gam_ = math.sqrt(1.0 + P[2:5] @ gcov[1:, 1:] @ P[2:5])
    beta = alpha * alpha * gcon[0, 1:]
    u = np.array([gam_ / alpha, *(P[2:5] - gam_ * beta / alpha)])
    ucov = gcov @ u
    bt = float(np.dot(B, ucov[1:]))
    b = np.array([bt, *((np.asarray(B) + bt * u[1:]) / u[0])])
    return u, b


def _floors(frame, P, B, g, rho_fl, u_fl, **kw):
    gcov, gcon, gdet, alpha, _ = g
    return oracle.floors(frame, P, B, gcov, gcon, gdet, alpha, GAM, rho_fl, u_fl, **kw)


BIG = dict(bsq_rho_max=1e300, bsq_u_max=1e300)


def test_fixed_frame_floors_set_the_minima_and_keep_utilde():
    g = _mink_point()
    P = np.array([1e-8, 1e-10, 0.3, -0.2, 0.1])
    Pn, hits = _floors(oracle.FLOOR_FIXED, P, [0.5, 0.2, 0.0], g, 1e-6, 1e-7, **BIG)
    assert hits == 2 and Pn[0] == 1e-6 and Pn[1] == 1e-7
    assert np.array_equal(Pn[2:], P[2:])


@pytest.mark.parametrize("field", ["none", "across"])
def test_drift_frame_is_the_fluid_frame_without_a_field_or_across_it(field):
    g = _mink_point()
    P = np.array([1e-8, 1e-10, 0.0, 0.6, 0.0])             # moving along y
    B = [0.0, 0.0, 0.0] if field == "none" else [0.7, 0.0, 0.4]   # field in the x-z plane
    Pn, hits = _floors(oracle.FLOOR_DRIFT, P, B, g, 1e-6, 1e-7, **BIG)
    assert hits == 2
    assert Pn[0] == pytest.approx(1e-6, rel=1e-10) and Pn[1] == pytest.approx(1e-7, rel=1e-10)
    assert np.allclose(Pn[2:], P[2:], rtol=1e-10, atol=1e-12)


def test_drift_frame_is_at_rest_for_a_flow_along_the_field():
    g = _mink_point()
    v = 0.5
    W = 1.0 / math.sqrt(1.0 - v * v)
    P = np.array([1e-8, 1e-10, W * v, 0.0, 0.0])           # along x, field along x
    B = [0.8, 0.0, 0.0]
    U0 = _cons(P, B, g)
    Pn, hits = _floors(oracle.FLOOR_DRIFT, P, B, g, 1e-6, 1e-7, **BIG)
    U1 = _cons(Pn, B, g)
    # momentum unchanged; energy and mass grow by the parcel at rest (rest mass drho,
    # energy drho + du in the conserved energy T^t_t + rho u^t)
    drho, du = 1e-6 - P[0], 1e-7 - P[1]
    assert np.allclose(U1[2:5], U0[2:5], rtol=1e-10, atol=1e-14 * abs(U0[2]))
    assert U1[0] - U0[0] == pytest.approx(drho, rel=1e-9)
    assert (U1[1] - U0[1]) == pytest.approx(-du, rel=1e-8)   # T^t_t of the parcel is -(u + 0)
    assert 0.0 < Pn[2] < P[2]                                  # slower, same direction
    assert hits == 2


def test_drift_floors_add_the_parcel_to_the_conserved_state_in_kerr_schild():
    rng = np.random.default_rng(12)
    checked = 0
    for _ in range(200):
        g = _ks_point(rng)
        gcov = g[0]
        rho = 10 ** rng.uniform(-9, -7)
        ut = rng.normal(size=3) * 0.5
        B = rng.normal(size=3) * 1e-3
        P = np.array([rho, rho * 10 ** rng.uniform(-3, 0), *ut])
        if 1.0 + P[2:5] @ gcov[1:, 1:] @ P[2:5] >= 50.0 ** 2:
            continue                      # the Lorentz-factor ceiling would act first
        U0 = _cons(P, B, g)
        Pn, hits = _floors(oracle.FLOOR_DRIFT, P, B, g, 1e-6, 1e-8, **BIG)
        if hits == 0:
            continue
        # the parcel, rebuilt from its definition
        gcov, gcon, gdet, alpha, _ = g
        u, b = _four_vectors(P, B, gcov, gcon, alpha)
        bsq = float(b @ gcov @ b)
        beta = -b[0] / (bsq * u[0])
        ud = (u + beta * b) / math.sqrt(1.0 - beta * beta * bsq)
        drho, du = max(1e-6 - P[0], 0.0), max(1e-8 - P[1], 0.0)
        Pp = np.array([drho, du, *(ud[1:] + ud[0] * alpha * alpha * gcon[0, 1:])])
        Up = _cons(Pp, [0.0, 0.0, 0.0], g)
        U1 = _cons(Pn, B, g)
        if Pn[0] > 1e-6 * (1 + 1e-9) and Pn[1] > 1e-8 * (1 + 1e-9):   # no fixed floor after it
            scale = np.abs(U0[:5] + Up[:5]).max()
            assert np.abs(U1[:5] - (U0[:5] + Up[:5])).max() <= 1e-9 * scale
            checked += 1
    assert checked > 50


@pytest.mark.parametrize("scale,tol", [(1e-100, 1e-13), (1e-160, 1e-13), (1e-200, 1e-13),
                                       (1e-300, 1e-10)])
def test_drift_frame_depends_on_the_field_direction_only(scale, tol):
    """beta b = -b^t b / (b^2 u^t) is unchanged when the field is multiplied by a constant,
    so a field whose b^2 lies below the smallest double (the traces that numerical
    diffusion leaves in an empty funnel) gives the frame of a stronger field of its
    direction; the field here carries no energy at the level of rounding either way.
    At 1e-300 the field components are subnormal and hold fewer digits."""
    g = _mink_point()
    P = np.array([1e-8, 1e-10, 0.4, 0.3, -0.2])
    B = np.array([0.7, -0.2, 0.4]) * 1e-12
    ref, _ = _floors(oracle.FLOOR_DRIFT, P, B, g, 1e-6, 1e-7, **BIG)
    weak, _ = _floors(oracle.FLOOR_DRIFT, P, B * scale, g, 1e-6, 1e-7, **BIG)
    assert np.abs(weak - ref).max() <= tol * np.abs(ref).max()
    # the direction matters: without a field the parcel moves with the fluid
    none, _ = _floors(oracle.FLOOR_DRIFT, P, [0.0, 0.0, 0.0], g, 1e-6, 1e-7, **BIG)
    assert np.abs(none[2:] - ref[2:]).max() > 1e-2
