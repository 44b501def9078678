"""More pins of the CPU oracle (CPU only): the membership bisection that serves
as the conditioning-free reference for t+- (Lemma "PEP and S cap C": t+ is
the end of the feasible interval), the billiard segment (Alg. Billiard),
the NONSMOOTH statuses (Lemma "Gradient of det F": the normal is undefined at
a rank <= m - 2 point and at a point where two pieces of the boundary meet),
and the area of the paper's 2-D example (Figure 5 caption)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2010_03817_amd import instances as I

from test_oracle_pins import bisect_boundary

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def ball_roots(x, v):
    """Roots of |x + t v|^2 = 1 in the cancellation-free form."""
    a = (v * v).sum(1)
    b = 2 * (x * v).sum(1)
    c = (x * x).sum(1) - 1.0
    q = -0.5 * (b + np.sign(b) * np.sqrt(b * b - 4 * a * c))
    r1, r2 = q / a, c / q
    return np.minimum(r1, r2), np.maximum(r1, r2)


def test_line_bisect_ball_closed_form_at_any_conditioning():
    """On the unit ball the bisection ends equal the quadratic's roots, also
    from starts 1e-6 .. 1e-12 inside the sphere, where kappa(F(x)) reaches
    1e12: membership decides the far root without reducing the pencil.
    Membership near the far root decides the sign of 1 - |x + t v|^2, whose
    rounding error is ~n eps and whose slope there is 2|<x, v> + t| = t+ (unit
    v), so the bisection end is within ~n eps / t+ of the root."""
    n = 6
    o = O.Oracle(I.arrow_ball(n))
    rng = np.random.default_rng(11)
    d = I.random_directions(rng, 40, n)
    gap = 10.0 ** rng.uniform(-12, -1, 40)
    x = d * (1.0 - gap)[:, None]
    v = I.random_directions(rng, 40, n)
    v = np.where(((v * x).sum(1) > 0)[:, None], -v, v)  # head inwards: a far t+
    tm, tp, st = o.line_bisect(x, v)
    assert (st == O.OK).all()
    rm, rp = ball_roots(x, v)
    assert np.all(np.abs(tp - rp) <= 1e-14 * rp + 4 * n * 2.2e-16 / rp)
    # the near root is a rounding-level distance; it is still bracketed
    assert np.all(np.abs(tm - rm) <= 1e-13 + 1e-9 * np.abs(rm))


def test_line_bisect_polytope_ratio_test():
    rng = np.random.default_rng(12)
    n, rows = 5, 13
    A = rng.standard_normal((rows, n))
    b = rng.uniform(0.5, 2.0, rows)
    o = O.Oracle(I.polytope(A, b))
    x = rng.standard_normal((30, n)) * 0.05
    v = rng.standard_normal((30, n))
    tm, tp, st = o.line_bisect(x, v)
    assert (st == O.OK).all()
    for k in range(30):
        ratios = (b - A @ x[k]) / (A @ v[k])
        rate = A @ v[k]
        assert tp[k] == pytest.approx(ratios[rate > 0].min(), rel=1e-14)
        assert tm[k] == pytest.approx(ratios[rate < 0].max(), rel=1e-14)


def test_line_bisect_matches_lapack_bisection_and_jacobi():
    """Against bisection on LAPACK's Cholesky (independent code) on small
    random instances with the box block, and against the eigen route of the
    oracle (Jacobi) from interior starts, where both are accurate."""
    rng = np.random.default_rng(13)
    for n, m in [(3, 4), (5, 8), (12, 15)]:
        inst = I.gbase(n, m, seed=60 + m)
        o = O.Oracle(inst)
        d = I.random_directions(rng, 5, n)
        x = 0.5 * d * o.intersect(np.zeros((5, n)), d)[1][:, None]
        v = I.random_directions(rng, 5, n)
        tm, tp, st = o.line_bisect(x, v)
        jm, jp, js = o.intersect(x, v)
        assert (st == O.OK).all() and (js == O.OK).all()
        assert np.allclose(tp, jp, rtol=1e-12) and np.allclose(tm, jm, rtol=1e-12)
        if m <= 8:
            for k in range(5):
                assert tp[k] == pytest.approx(bisect_boundary(inst, x[k], v[k]), rel=1e-12)
                assert -tm[k] == pytest.approx(bisect_boundary(inst, x[k], v[k], -1.0), rel=1e-12)
        # the guess changes only the bracket search, not the result
        g = np.stack([jm * 1.3, jp * 0.7], 1)
        tm2, tp2, _ = o.line_bisect(x, v, guess=g)
        assert np.array_equal(tp, tp2) and np.array_equal(tm, tm2)


def test_line_bisect_statuses():
    o = O.Oracle(I.arrow_ball(3))
    tm, tp, st = o.line_bisect(np.array([[2.0, 0, 0]]), np.array([[1.0, 0, 0]]))
    assert st[0] == O.NOT_INTERIOR and np.isnan(tp[0])
    # one facet only: unbounded on the other side
    half = I.polytope(np.array([[1.0, 0.0]]), np.array([1.0]))
    tm, tp, st = O.Oracle(half).line_bisect(np.zeros((1, 2)), np.array([[1.0, 0.0]]))
    assert st[0] == O.UNBOUNDED and tp[0] == pytest.approx(1.0, rel=1e-15) and np.isneginf(tm[0])


def test_billiard_segment_on_ball():
    """One segment of Alg. Billiard on the unit ball: move the whole length
    when the sphere is farther, else stop short of the hit by the pull-back,
    reflect about the normal (the hit point) and keep the rest of the length."""
    n = 4
    o = O.Oracle(I.arrow_ball(n))
    rng = np.random.default_rng(14)
    x = I.random_directions(rng, 50, n) * rng.uniform(0, 0.9, 50)[:, None]
    v = I.random_directions(rng, 50, n)
    ell = rng.uniform(0.1, 2.5, 50)
    pb = 1e-6
    xn, vn, el, refl, st = o.billiard_segment(x, v, ell, pullback=pb)
    _, tp = ball_roots(x, v)
    hit = tp < ell
    assert np.array_equal(refl, hit) and hit.any() and (~hit).any()
    assert (st == O.OK).all()
    far = ~hit
    assert np.allclose(xn[far], x[far] + ell[far, None] * v[far], atol=1e-14)
    assert np.array_equal(vn[far], v[far]) and (el[far] == 0).all()
    p = x[hit] + tp[hit, None] * v[hit]
    w = p / np.linalg.norm(p, axis=1, keepdims=True)
    s = v[hit] - 2 * (v[hit] * w).sum(1, keepdims=True) * w
    assert np.allclose(vn[hit], s, atol=1e-9)
    assert np.allclose(xn[hit], x[hit] + ((1 - pb) * tp[hit])[:, None] * v[hit], rtol=1e-12, atol=1e-14)
    assert np.allclose(el[hit], ell[hit] - tp[hit], rtol=1e-12)
    # the new start is interior and its direction points back inside
    assert o.membership(xn).all()
    assert ((vn[hit] * w).sum(1) < 0).all()


def test_nonsmooth_statuses():
    """Where the normal is not determined the reflection still happens but
    the status says NONSMOOTH: a vertex of a box (two facets tie), two
    identical dense blocks (a tie across blocks) and a double lambda_min of
    one block (rank m - 2 at the hit).  A generic hit stays OK."""
    o = O.Oracle(I.box(2, 1.0))
    v = np.array([[1.0, 1.0]]) / math.sqrt(2)
    tp, s, w, st = o.reflect(np.zeros((1, 2)), v)
    assert st[0] == O.NONSMOOTH and tp[0] == pytest.approx(math.sqrt(2), rel=1e-15)
    tp, s, w, st = o.reflect(np.zeros((1, 2)), np.array([[1.0, 0.3]]))
    assert st[0] == O.OK
    # two identical dense blocks (n = 1): F(x) = blkdiag(G(x), G(x))
    G = np.zeros((2, 2, 2))
    G[0] = np.eye(2)
    G[1] = np.array([[-1.0, 0.2], [0.2, 0.5]])
    one = I.Instance(1, [I.Block(I.DENSE, G)], name="one")
    two = I.Instance(1, [I.Block(I.DENSE, G), I.Block(I.DENSE, G.copy())], name="two")
    x, v = np.zeros((1, 1)), np.ones((1, 1))
    assert O.Oracle(one).reflect(x, v)[3][0] == O.OK
    tp2, _, _, st2 = O.Oracle(two).reflect(x, v)
    assert st2[0] == O.NONSMOOTH and tp2[0] == pytest.approx(O.Oracle(one).reflect(x, v)[0][0], rel=1e-15)
    # a double eigenvalue: F(x) = diag(1 - x, 1 - x, 1 + x / 2)
    D = np.zeros((2, 3, 3))
    D[0] = np.eye(3)
    D[1] = np.diag([-1.0, -1.0, 0.5])
    tp3, _, _, st3 = O.Oracle(I.Instance(1, [I.Block(I.DENSE, D)], name="dbl")).reflect(x, v)
    assert st3[0] == O.NONSMOOTH and tp3[0] == pytest.approx(1.0, rel=1e-15)
    D[1] = np.diag([-1.0, -0.5, 0.5])
    tp4, _, _, st4 = O.Oracle(I.Instance(1, [I.Block(I.DENSE, D)], name="sgl")).reflect(x, v)
    assert st4[0] == O.OK and tp4[0] == pytest.approx(1.0, rel=1e-15)


def polar_area(o, centre, k):
    """Area of a planar convex body by polar quadrature about an interior
    point: (1/2) sum r(theta)^2 dtheta, r = t+ along (cos, sin) (trapezoid
    rule on the periodic integrand)."""
    th = 2 * math.pi * (np.arange(k) + 0.5) / k
    d = np.stack([np.cos(th), np.sin(th)], 1)
    _, tp, st = o.intersect(np.repeat(centre[None], k, 0), d)
    assert (st == O.OK).all()
    return 0.5 * float((tp ** 2).sum()) * (2 * math.pi / k)


def test_paper_example_area_envelope():
    """Figure 5's caption gives the example's area, 10.23, for the unrounded
    matrices; the appendix prints them to one decimal.  The quadrature is
    pinned on the unit disc (pi); the rounded matrices give 10.45, and the
    printed area lies inside the range that perturbing every printed entry
    within its rounding half-width (0.05, symmetric, the -Qt blocks kept
    exact negatives) produces."""
    g = json.load(open(os.path.join(GOLDEN, "paper_example_2d.json")))
    disc = O.Oracle(I.arrow_ball(2))
    assert polar_area(disc, np.zeros(2), 4000) == pytest.approx(math.pi, rel=1e-10)
    base = I.paper_example_2d()
    p0 = np.array(g["p0"])
    a0 = polar_area(O.Oracle(base), p0, 8000)
    assert a0 == pytest.approx(10.4531, abs=2e-3)
    rng = np.random.default_rng(15)
    A = base.blocks[0].A
    areas = []
    for _ in range(120):
        P = A.copy()
        E = rng.uniform(-0.05, 0.05, (3, 6, 6))
        E = np.triu(E) + np.triu(E, 1).transpose(0, 2, 1)
        P[0] += E[0]
        for i in (1, 2):
            q = E[i][:3, :3]
            P[i, :3, :3] += q
            P[i, 3:, 3:] -= q
        o = O.Oracle(I.Instance(2, [I.Block(I.DENSE, P)], name="perturbed"))
        if not o.membership(p0[None])[0]:
            continue
        areas.append(polar_area(o, p0, 1500))
    areas = np.array(areas)
    assert len(areas) > 100
    assert areas.min() < g["area_printed"] < areas.max()
    assert areas.min() < a0 < areas.max()


def test_near_root_rounding_bound_covers_the_oracles_two_routes():
    """The first-order rounding bound of a root next to its start (test
    helper root_bounds) covers the difference between the oracle's eigen
    route and its bisection on starts pulled back 1e-6 from the boundary,
    and is not vacuous (well under 1e-3 of the root)."""
    from root_bounds import root_bars
    inst = I.gbase(20, 24, seed=19)
    o = O.Oracle(inst)
    rng = np.random.default_rng(16)
    d = I.random_directions(rng, 24, inst.n)
    x0 = 0.3 * d * o.intersect(np.zeros((24, inst.n)), d)[1][:, None]
    u = I.random_directions(rng, 24, inst.n)
    x = x0 + (1 - 1e-6) * o.intersect(x0, u)[1][:, None] * u
    v = I.random_directions(rng, 24, inst.n)
    jm, jp, js = o.intersect(x, v)
    bm, bp, bs = o.line_bisect(x, v)
    assert (js == O.OK).all() and (bs == O.OK).all()
    bar_m, bar_p = root_bars(inst, x, v, bm, bp, 1e-9)
    assert (np.abs(jm - bm) <= bar_m).all() and (np.abs(jp - bp) <= bar_p).all()
    near = np.minimum(np.abs(bm), bp)
    nb = np.where(np.abs(bm) < bp, bar_m, bar_p)
    assert np.all(nb < 1e-3 * near)
