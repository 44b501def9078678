"""Pins of the oracle's ball-sequence volume (eq. (mmc_vol): S_i = S cap rho_i B,
billiard samples of each S_i, ratios of consecutive volumes by counting,
the last ball's volume by exact uniform draws and membership) against bodies
of known volume: a box, the centred simplex, the unit ball (arrow LMI) and the
3-D elliptope.  The estimate is random: the truth must lie within twice the
95 % interval of the per-group estimates."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2010_03817_amd import instances as I

CASES = {
    "box30": (lambda: I.box(30, 1.0), 30 * math.log(2.0)),
    "simplex12": (lambda: I.simplex(12), -math.lgamma(13.0)),
    "ball12": (lambda: I.arrow_ball(12), 6 * math.log(math.pi) - math.lgamma(7.0)),
    "elliptope3": (lambda: I.elliptope3(), math.log(math.pi**2 / 2)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_ball_sequence_volume_of_known_bodies(name):
    make, truth = CASES[name]
    o = O.Oracle(make())
    lv, lo, hi, radii, phases, rc = o.volume_balls(64, 32, 2, 10, 0.2, 40, 400, seed=7, tau=2.0)
    assert rc == O.OK
    half = 0.5 * (hi - lo)
    assert lo - half <= truth <= hi + half, (name, lv, lo, hi, truth)
    # radii shrink from rho_0 = inf, and the last ball holds S's samples
    assert np.isinf(radii[0]) and np.all(np.diff(radii[1:]) < 0)


def test_more_phases_in_higher_dimension():
    """A 60-cube needs several balls (each ratio near q): the sequence is
    longer and the estimate still holds its volume."""
    o = O.Oracle(I.box(60, 1.0))
    lv, lo, hi, radii, phases, rc = o.volume_balls(64, 32, 2, 10, 0.2, 40, 400, seed=8, tau=4.0)
    truth = 60 * math.log(2.0)
    assert rc == O.OK and phases >= 3
    half = 0.5 * (hi - lo)
    assert lo - half <= truth <= hi + half, (lv, lo, hi, truth)
