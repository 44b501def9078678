"""Pins of the oracle's Boltzmann walks and annealing (the paper's optimisation
section: eq. (sdp), the Boltzmann density exp(-<c, x> / T) truncated to S,
the HMC trajectory of eq. (boltz_ode), the cooling T_{i+1} = T_i (1 - 1/sqrt n)).

Each pin checks the oracle against something other than itself: the closed-form
law of a truncated exponential (exact draws of Hit-and-Run on an interval; the
product law that HMC must leave invariant on a box), the closed-form first hit
of the degree-2 trajectory on a box, and linear programs whose optima are known
(box, centred simplex, ball)."""
import math

import numpy as np
import pytest
import scipy.stats

from oracle import oracle as O
from paper_2010_03817_amd import instances as I


def trunc_exp_cdf(x, lam, a=-1.0, b=1.0):
    """CDF on [a, b] of the density proportional to exp(-lam x)."""
    if abs(lam) < 1e-12:
        return (x - a) / (b - a)
    # (e^{-lam a} - e^{-lam x}) / (e^{-lam a} - e^{-lam b}), in a stable form
    return np.expm1(-lam * (x - a)) / np.expm1(-lam * (b - a))


@pytest.mark.parametrize("c", [2.0, -3.0, 1e-14])
def test_hit_and_run_chord_is_a_truncated_exponential(c):
    """On the interval [-1, 1] every Hit-and-Run chord is the whole interval, so
    one step from any start is an exact draw of the truncated exponential with
    rate c / T (both signs of <c, v> occur, as v = +-1)."""
    o = O.Oracle(I.box(1, 1.0))
    T = 0.5
    x0 = np.full((4000, 1), 0.3)
    x, _, st = o.walk_boltz(O.HNR, x0, 1, seed=5, c=[c], T=T)
    assert st[0] == 4000 and st[3] == 0
    lam = c / T
    p = scipy.stats.kstest(x[:, 0], lambda y: trunc_exp_cdf(y, lam)).pvalue
    assert p > 1e-3, p
    # the mean against its closed form 1/lam - coth(lam)
    if abs(lam) > 1e-6:
        mean = 1.0 / lam - 1.0 / math.tanh(lam)
        assert abs(x[:, 0].mean() - mean) < 4 * x[:, 0].std() / math.sqrt(len(x))


@pytest.mark.parametrize("dense", [False, True])
def test_hmc_keeps_the_boltzmann_law_on_a_box(dense):
    """HMC with reflections on exp(-<c, x> / T) over [-1, 1]^2: the coordinates
    are independent truncated exponentials with rates c_j / T.  A wrong sign of
    the force or of the reflection moves mass to the wrong side."""
    inst = I.box_as_dense(2, 1.0) if dense else I.box(2, 1.0)
    o = O.Oracle(inst)
    c, T = np.array([1.5, -0.7]), 0.6
    x0 = np.zeros((150, 2))
    _, smp, st = o.walk_boltz(O.HMC, x0, 160, seed=9, c=c, T=T, tau=1.5, thin=16)
    assert st[3] == 0 and st[1] > 0  # reflections happen, never outside S
    pts = smp[:, 3:].reshape(-1, 2)
    for j in range(2):
        lam = c[j] / T
        p = scipy.stats.kstest(pts[:, j], lambda y: trunc_exp_cdf(y, lam)).pvalue
        assert p > 1e-3, (j, p)


def test_boltzmann_curve_first_hit_on_a_box():
    """The segment x(t) = p + t v - t^2 c / (2T) leaves [-1, 1]^n first where
    1 -+ x_j(t) = 0; the oracle's degree-2 intersection with the rows
    (1, p), (0, v), (0, -c / (2T)) finds the smallest positive such root."""
    rng = np.random.default_rng(3)
    n = 4
    o = O.Oracle(I.box(n, 1.0))
    for _ in range(20):
        p = rng.uniform(-0.8, 0.8, n)
        v = rng.standard_normal(n)
        c = rng.standard_normal(n)
        T = rng.uniform(0.2, 2.0)
        coef = np.zeros((1, 3, n + 1))
        coef[0, 0, 0], coef[0, 0, 1:] = 1.0, p
        coef[0, 1, 1:] = v
        coef[0, 2, 1:] = -c / (2 * T)
        _, tp, st, _ = o.intersect_curve2(coef)
        best = np.inf
        for j in range(n):
            for sgn in (1.0, -1.0):  # 1 - sgn x_j(t) = 0
                a2, a1, a0 = sgn * c[j] / (2 * T), -sgn * v[j], 1.0 - sgn * p[j]
                for r in np.roots([a2, a1, a0]):
                    if abs(r.imag) < 1e-12 and r.real > 0:
                        best = min(best, r.real)
        assert st[0] == O.OK
        assert abs(tp[0] - best) <= 1e-12 * best, (tp[0], best)


def _anneal(o, kind, x0, c, iters, walk_len, diam, seed=21):
    """T0 = diam |c| (the density is nearly flat over S), cooling 1 - 1/sqrt n,
    HMC travel-time scale tau0 = diam at T0."""
    n = o.n
    return o.sdp_anneal(kind, x0, c, diam * np.linalg.norm(c), 1.0 / math.sqrt(n), iters, walk_len, seed, diam)


@pytest.mark.parametrize("body", ["box", "simplex", "ball"])
def test_annealing_reaches_known_optima(body):
    """min <c, x> over a box (-|c|_1), the centred simplex (the best vertex) and
    the unit ball (-|c|): the HMC annealing of the paper's schedule with walk
    length one ends within 5 % of the optimum; no iterate is ever better than
    the optimum (every iterate lies in S), and the best iterate is inside S."""
    n = 6
    rng = np.random.default_rng(17)
    c = rng.standard_normal(n)
    if body == "box":
        inst, fstar, diam = I.box(n, 1.0), -np.abs(c).sum(), 2 * math.sqrt(n)
    elif body == "simplex":
        inst, diam = I.simplex(n), math.sqrt(2.0)
        fstar = min(0.0, c.min()) - c.sum() / (n + 1)
    else:
        inst, fstar, diam = I.arrow_ball(n), -np.linalg.norm(c), 2.0
    o = O.Oracle(inst)
    x0 = np.zeros((8, n))
    xb, fb, best = _anneal(o, O.HMC, x0, c, iters=70, walk_len=1, diam=diam)
    assert np.all(fb >= fstar - 1e-9 * abs(fstar))
    assert np.all(np.diff(best, axis=1) <= 0)  # the best value never gets worse
    rel = (fb - fstar) / abs(fstar)
    assert np.median(rel) <= 0.05, rel
    assert o.membership(xb).all()


def test_hit_and_run_annealing_on_the_ball():
    """Hit-and-Run on the Boltzmann density (walk length 4 sqrt n) also reaches
    the optimum of the ball."""
    n = 6
    c = np.arange(1.0, n + 1)
    o = O.Oracle(I.arrow_ball(n))
    xb, fb, _ = _anneal(o, O.HNR, np.zeros((6, n)), c, iters=70, walk_len=int(4 * math.sqrt(n)), diam=2.0)
    fstar = -np.linalg.norm(c)
    assert np.all(fb >= fstar - 1e-9 * abs(fstar))
    assert np.median((fb - fstar) / abs(fstar)) <= 0.05


@pytest.mark.parametrize("body", ["box", "dense_box", "simplex", "ball"])
def test_barrier_optimum_matches_closed_forms(body):
    """The log-barrier reference optimum (oracle/sdp_barrier.py) equals the
    known optima of linear programs over a box, the centred simplex and the
    ball (as LMIs: diagonal rows, a dense diagonal block, an arrow block)."""
    from oracle.sdp_barrier import sdp_min
    n = 7
    c = np.random.default_rng(23).standard_normal(n)
    if body == "box":
        inst, fstar = I.box(n, 1.0), -np.abs(c).sum()
    elif body == "dense_box":
        inst, fstar = I.box_as_dense(n, 1.0), -np.abs(c).sum()
    elif body == "simplex":
        inst, fstar = I.simplex(n), min(0.0, c.min()) - c.sum() / (n + 1)
    else:
        inst, fstar = I.arrow_ball(n), -np.linalg.norm(c)
    x, f, _ = sdp_min(inst, c)
    assert abs(f - fstar) <= 1e-9 * abs(fstar), (f, fstar)
    assert abs(c @ x - f) == 0.0


def test_annealing_against_the_barrier_optimum_on_a_paper_instance():
    """On S-8-8 of the paper's generator the oracle's annealing never goes
    below the barrier optimum and its median chain ends within 5 % of it."""
    from oracle.sdp_barrier import sdp_min
    n = 8
    inst = I.paper_random(n, n, seed=808)
    c = I.objective(n, 809)
    _, fstar, _ = sdp_min(inst, c)
    o = O.Oracle(inst)
    # diameter estimate: the longest chord through the centre along the axes
    E = np.eye(n)
    tm, tp, _ = o.intersect(np.zeros((n, n)), E)
    diam = float(np.max(tp - tm))
    iters = math.ceil(math.log(1e-7) / math.log(1 - 1 / math.sqrt(n)))
    xb, fb, best = o.sdp_anneal(O.HMC, np.zeros((8, n)), c, diam, 1 / math.sqrt(n), iters, 1, 5, diam)
    assert np.all(fb >= fstar - 1e-9 * abs(fstar))
    assert np.median((fb - fstar) / abs(fstar)) <= 0.05


def test_stored_optima_come_from_the_barrier_method():
    """The first stored optimum of the annealing workload is what the oracle's
    barrier method gives for it."""
    import json
    import os
    from oracle.sdp_barrier import sdp_min
    with open(os.path.join(os.path.dirname(__file__), "golden", "sdp_optima.json")) as fh:
        doc = json.load(fh)
    e = doc["optima"][0]
    inst = I.paper_random(e["n"], e["m"], seed=e["instance_seed"])
    _, f, _ = sdp_min(inst, I.objective(e["n"], e["objective_seed"]))
    assert abs(f - e["f_star"]) <= 1e-9 * abs(e["f_star"])
    assert len(doc["optima"]) == len(I.sdp_family())
