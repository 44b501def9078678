"""The ball-sequence volume on the device (eq. (mmc_vol)): the billiard walk in
S cap rho B (uniform law on a body of known shape), and volumes of known
bodies beside the oracle's estimate of the same body."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2010_03817_amd import instances as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_2010_03817_amd import spec
    return spec


def test_billiard_in_box_cap_ball_is_uniform_on_the_ball(S):
    """[-1, 1]^4 cap {|x| <= 1} is the unit ball: billiard samples are uniform
    there (E|x|^2 = n / (n + 2), Pr[|x| <= 1/2] = 2^-n), and none leaves it."""
    n = 4
    g = S.Spectrahedron(I.box(n, 1.0))
    _, smp, st, _ = g.walk(S.BILLIARD, np.zeros((512, n)), 200, seed=5, tau=2.0, thin=10, ball_radius=1.0)
    assert st["not_interior"] == 0 and st["reflections"] > 0
    r = np.linalg.norm(smp.cpu().numpy()[:, 4:], axis=-1)
    assert r.max() <= 1.0
    cm = (r**2).mean(1)
    se = cm.std() / math.sqrt(len(cm))
    assert abs(cm.mean() - n / (n + 2)) < 4 * se
    f = (r <= 0.5).mean(1)
    assert abs(f.mean() - 2.0**-n) < 4 * f.std() / math.sqrt(len(f)) + 1e-3


CASES = {
    "box40": (lambda: I.box(40, 1.0), 40 * math.log(2.0)),
    "simplex12": (lambda: I.simplex(12), -math.lgamma(13.0)),
    "ball30": (lambda: I.arrow_ball(30), 15 * math.log(math.pi) - math.lgamma(16.0)),
    "elliptope3": (lambda: I.elliptope3(), math.log(math.pi**2 / 2)),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_ball_sequence_volume_of_known_bodies(S, name):
    make, truth = CASES[name]
    g = S.Spectrahedron(make())
    lv, lo, hi, st = g.volume_balls(chains=1024, samples_per_chain=16, seed=11)
    print(f"{name}: {lv:.4f} [{lo:.4f}, {hi:.4f}] truth {truth:.4f}; {st['phases']} balls, "
          f"{st['points']:.0f} points")
    half = 0.5 * (hi - lo)
    assert lo - half <= truth <= hi + half
    assert np.all(np.diff(st["radii"]) < 0)


def test_against_the_oracle_estimate(S):
    """The same method on the CPU oracle and on the device (different random
    streams): both intervals hold the 30-cube's volume and overlap."""
    inst = I.box(30, 1.0)
    truth = 30 * math.log(2.0)
    o = O.Oracle(inst)
    olv, olo, ohi, _, _, rc = o.volume_balls(64, 32, 2, 10, 0.2, 40, 400, seed=7, tau=2.0)
    assert rc == O.OK
    g = S.Spectrahedron(inst)
    lv, lo, hi, _ = g.volume_balls(chains=1024, samples_per_chain=16, seed=12)
    assert lo - (hi - lo) <= truth <= hi + (hi - lo)
    assert max(lo, olo) - 0.5 * (hi - lo + ohi - olo) <= min(hi, ohi)
