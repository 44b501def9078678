"""Polynomial curves of degree 3 to 6 on the device (eq. (PEP)): the first
roots of det F(Phi(t)) on both sides against the oracle's companion
linearisation, a cubic with zero leading row against the degree-2 path, the
unit ball's scalar equation, diagonal rows, and the horizon."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import pep
from paper_2010_03817_amd import instances as I

pytestmark = pytest.mark.gpu
T_REL = 1e-9


@pytest.fixture(scope="module")
def S():
    from paper_2010_03817_amd import spec
    return spec


def _curves(rng, n, d, count, scale=0.6, start=0.05):
    coef = np.zeros((count, d + 1, n + 1))
    coef[:, 0, 0] = 1.0
    coef[:, 0, 1:] = start * rng.standard_normal((count, n))
    for k in range(1, d + 1):
        coef[:, k, 1:] = scale**k * rng.standard_normal((count, n))
    return coef


def _np(t):
    return t.detach().cpu().numpy()


def _check(inst, coef, tm, tp, st, horizon=np.inf):
    assert (st == 0).all(), st
    for k in range(len(coef)):
        wm, wp = pep.first_roots_companion(inst, coef[k], horizon)
        assert np.isfinite(tp[k]) == np.isfinite(wp) and np.isfinite(tm[k]) == np.isfinite(wm), (k, tp[k], wp)
        if np.isfinite(wp):
            assert abs(tp[k] - wp) <= T_REL * abs(wp), (k, tp[k], wp)
        if np.isfinite(wm):
            assert abs(tm[k] - wm) <= T_REL * abs(wm), (k, tm[k], wm)


@pytest.mark.parametrize("d", [3, 4, 6])
@pytest.mark.parametrize("name", ["config1", "gbase20"])
def test_degree_d_matches_companion(S, d, name):
    inst = I.gbase(10, 10, seed=101, scale=math.sqrt(10)) if name == "config1" else I.gbase(20, 20, seed=7)
    g = S.Spectrahedron(inst)
    coef = _curves(np.random.default_rng(d), inst.n, d, 24, scale=0.6 if d < 6 else 0.5)
    tm, tp, st = g.intersect_curve(coef, degree=d)
    _check(inst, coef, _np(tm), _np(tp), _np(st))


def test_cubic_with_zero_leading_row_equals_degree_two(S):
    inst = I.gbase(10, 10, seed=101, scale=math.sqrt(10))
    g = S.Spectrahedron(inst)
    c2 = _curves(np.random.default_rng(3), 10, 2, 32)
    c3 = np.concatenate([c2, np.zeros((32, 1, 11))], axis=1)
    tm2, tp2, st2 = [_np(t) for t in g.intersect_curve(c2, degree=2)]
    tm3, tp3, st3 = [_np(t) for t in g.intersect_curve(c3, degree=3)]
    assert (st2 == 0).all() and (st3 == 0).all()
    assert np.allclose(tp3, tp2, rtol=T_REL) and np.allclose(tm3, tm2, rtol=T_REL)


@pytest.mark.parametrize("d", [3, 5])
def test_ball_and_box(S, d):
    """The unit ball (an arrow block): roots of |Phi(t)|^2 = 1; the box
    (diagonal rows): the rows' scalar polynomials."""
    for inst in (I.arrow_ball(8), I.box(8, 1.0)):
        g = S.Spectrahedron(inst)
        coef = _curves(np.random.default_rng(20 + d), 8, d, 16)
        tm, tp, st = g.intersect_curve(coef, degree=d)
        _check(inst, coef, _np(tm), _np(tp), _np(st))


def test_horizon_and_full_size_sample(S):
    """Roots beyond the horizon are not reported; n = m = 100 on a sample."""
    inst = I.gbase(20, 20, seed=7)
    g = S.Spectrahedron(inst)
    coef = _curves(np.random.default_rng(9), 20, 3, 16)
    _, tp, _ = [_np(t) for t in g.intersect_curve(coef, degree=3)]
    h = float(np.median(tp))
    tmh, tph, sth = [_np(t) for t in g.intersect_curve(coef, horizon=h, degree=3)]
    _check(inst, coef, tmh, tph, sth, horizon=h)
    assert np.all(np.isinf(tph[tp > h]))
    big = I.gbase(100, 100, seed=102)
    gb = S.Spectrahedron(big)
    coef = _curves(np.random.default_rng(10), 100, 4, 6, scale=0.3, start=0.01)
    tm, tp, st = [_np(t) for t in gb.intersect_curve(coef, degree=4)]
    _check(big, coef, tm, tp, st)


def test_degree_limits(S):
    g = S.Spectrahedron(I.box(3, 1.0))
    with pytest.raises(S.SpecError):
        g.intersect_curve(np.zeros((1, 8, 4)), degree=7)
