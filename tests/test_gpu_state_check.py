"""Failure detection through the C ABI: a step with statistics checks the state it
leaves and returns GRMHD_ESTATE when an update produced a non-physical cell (a
non-finite value, rho <= 0 or u <= 0 after the floors).  The condition is forced from
the host by planting a NaN or an infinity in the initial state; every kernel runs to its
normal end (the inversion's iterations are bounded)."""
import sys

import numpy as np
import pytest

from paper_1912_10192_amd import configs, grmhd, initdata
from tests.helpers import mink_cfg, random_periodic_state

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def test_clean_steps_report_no_bad_states():
    cfg = dict(configs.TORUS_TINY, block=(32, 32, 32))
    say("[state-check] clean torus, 2 steps")
    grid = grmhd.Grid(cfg, state=initdata.torus_state(cfg["n"], **configs.TORUS_INIT))
    st = grid.step(2)
    assert st.bad_states == 0


@pytest.mark.parametrize("where", ["rho-nan", "face-inf"])
def test_planted_non_finite_value_is_reported(where):
    n = (16, 16, 8)
    cfg = dict(mink_cfg(n, recon=1, riemann=1), block=(8, 8, 8))
    P, B1, B2, B3 = random_periodic_state(n, seed=9, amp=0.05, vamp=0.2, bamp=0.2)
    if where == "rho-nan":
        P[0][3, 5, 7] = np.nan
    else:
        B1[2, 4, 6] = np.inf
    say(f"[state-check] planted {where}")
    quiet = grmhd.Grid(cfg, state=(P, B1, B2, B3))
    assert quiet.step(1, stats=False) is None            # nothing checked without stats
    grid = grmhd.Grid(cfg, state=(P, B1, B2, B3))
    with pytest.raises(grmhd.GrmhdError, match="non-finite"):
        grid.step(1)
