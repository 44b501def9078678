"""Pins of the oracle's degree-d curve intersection (eq. (PEP), companion
linearisation) against routes that share nothing with it: the oracle's
certified Weyl stepping with Jacobi eigenvalues for d = 2, the plain
definition by bisection on Cholesky membership for d = 3 and 4, and the unit
ball, where the first root solves the scalar equation |Phi(t)|^2 = 1."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from oracle import pep
from paper_2010_03817_amd import instances as I


def _curves(rng, n, d, count, scale=0.6, start=0.05):
    coef = np.zeros((count, d + 1, n + 1))
    coef[:, 0, 0] = 1.0
    coef[:, 0, 1:] = start * rng.standard_normal((count, n))
    for k in range(1, d + 1):
        coef[:, k, 1:] = scale ** k * rng.standard_normal((count, n))
    return coef


def test_degree_two_matches_weyl_stepping():
    inst = I.gbase(10, 10, seed=101, scale=math.sqrt(10))
    o = O.Oracle(inst)
    coef = _curves(np.random.default_rng(1), 10, 2, 24)
    tm_w, tp_w, st, _ = o.intersect_curve2(coef, np.inf)
    assert (st == O.OK).all()
    for k in range(len(coef)):
        tm, tp = pep.first_roots_companion(inst, coef[k])
        assert abs(tp - tp_w[k]) <= 1e-9 * tp_w[k], (k, tp, tp_w[k])
        assert abs(tm - tm_w[k]) <= 1e-9 * abs(tm_w[k]), (k, tm, tm_w[k])


@pytest.mark.parametrize("d", [3, 4])
def test_companion_matches_bisection(d):
    inst = I.gbase(8, 9, seed=7)
    coef = _curves(np.random.default_rng(d), 8, d, 10)
    for k in range(len(coef)):
        _, tp = pep.first_roots_companion(inst, coef[k])
        ref = pep.first_root_bisect(inst, coef[k], horizon=min(4.0 * tp, 50.0) if np.isfinite(tp) else 50.0)
        assert np.isfinite(tp) and abs(tp - ref) <= 1e-9 * ref, (k, tp, ref)


@pytest.mark.parametrize("d", [3, 5])
def test_ball_first_root(d):
    """On the unit ball (arrow LMI), det F(Phi(t)) vanishes where |Phi(t)| = 1:
    the first positive root of the scalar polynomial |Phi(t)|^2 - 1."""
    n = 6
    inst = I.arrow_ball(n)
    coef = _curves(np.random.default_rng(11 + d), n, d, 12)
    for k in range(len(coef)):
        c = coef[k, :, 1:]
        g = np.zeros(2 * d + 1)
        for i in range(d + 1):
            for j in range(d + 1):
                g[i + j] += c[i] @ c[j]
        g[0] -= 1.0
        roots = np.roots(g[::-1])
        want = min(r.real for r in roots if abs(r.imag) < 1e-9 and r.real > 0)
        _, tp = pep.first_roots_companion(inst, coef[k])
        assert abs(tp - want) <= 1e-9 * want, (k, tp, want)


def test_diagonal_rows_and_horizon():
    """A box: each row's first root by bisection; past the horizon, none."""
    inst = I.box(5, 1.0)
    coef = _curves(np.random.default_rng(5), 5, 3, 10)
    for k in range(len(coef)):
        _, tp = pep.first_roots_companion(inst, coef[k])
        ref = pep.first_root_bisect(inst, coef[k], horizon=min(4.0 * tp, 50.0))
        assert abs(tp - ref) <= 1e-9 * ref
        _, tp2 = pep.first_roots_companion(inst, coef[k], horizon=0.5 * tp)
        assert tp2 == np.inf
