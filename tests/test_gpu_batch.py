"""GPU tests of uneven batching: many spectrahedra of different n and m in one
persistent launch (and the other launch strategies), HIP-graph replay, the
autotuner, and the batched volume estimate."""
import math

import numpy as np
import pytest

from paper_2010_03817_amd import instances as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_2010_03817_amd import spec
    return spec


def _mix():
    insts = [I.arrow_ball(5), I.elliptope3(), I.box(4, 1.0), I.arrow_ball(8),
             I.gbase(6, 14, seed=41, box=True), I.gbase(12, 7, seed=42, box=True)]
    truths = [2.5 * math.log(math.pi) - math.lgamma(3.5), math.log(math.pi**2 / 2), 4 * math.log(2.0),
              4 * math.log(math.pi) - math.lgamma(5.0), None, None]
    return insts, truths


PARAMS = dict(phases=12, samples_per_phase=512, chains=32, walk_len=4, groups=8, seed=23, burn_in=8)


def test_batch_strategies_and_graph_agree_with_single(S):
    """The per-chain arithmetic does not depend on how chains are launched:
    every strategy, with and without graph replay, and the single-instance
    estimate give identical results."""
    insts, truths = _mix()
    # batch rounds assemble F(x) in every round; the handles' own walks (the
    # pre-runs here, the single-instance estimate below) do the same with
    # refresh_period 1, which makes the comparison bit for bit
    specs = [S.Spectrahedron(i, refresh_period=1) for i in insts]
    b = S.Batch(specs)
    results = []
    for strategy, graph in ((1, True), (2, True), (3, False), (1, False)):
        b.set_strategy(strategy, graph)
        lv, lo, hi, calls = b.volume(**PARAMS)
        results.append((lv, lo, hi))
        assert calls > 0
    for r in results[1:]:
        assert np.array_equal(r[0], results[0][0])
        assert np.array_equal(r[1], results[0][1])
    for k in (0, 4):
        g = S.Spectrahedron(insts[k], refresh_period=1)
        lv1, lo1, hi1, _ = g.volume(**PARAMS)
        assert lv1 == results[0][0][k] and lo1 == results[0][1][k]
    lv, lo, hi = results[0]
    for k, t in enumerate(truths):
        if t is None:
            continue
        w = hi[k] - lo[k]
        assert lo[k] - w <= t <= hi[k] + w, (k, lv[k], lo[k], hi[k], t)


def test_batch_tune_picks_a_strategy(S):
    insts, _ = _mix()
    b = S.Batch([S.Spectrahedron(i) for i in insts])
    chosen, ms = b.tune(chains=64, rounds=3)
    assert chosen in (1, 2, 3)
    assert all(np.isfinite(ms)) and min(ms) == ms[chosen - 1]


def test_tune_then_volume_revalidates_the_plan(S):
    """The autotuner builds the batch plan for its chains; the volume's exact
    draws then grow the handles' workspaces.  The plan must follow the new
    workspaces (a stale plan would point at freed memory)."""
    insts, truths = _mix()
    specs = [S.Spectrahedron(i) for i in insts]
    b = S.Batch(specs)
    chosen, _ = b.tune(chains=32, rounds=2)
    lv, lo, hi, _ = b.volume(**PARAMS)
    b2 = S.Batch([S.Spectrahedron(i) for i in insts])
    b2.set_strategy(chosen, True)
    lv2, lo2, hi2, _ = b2.volume(**PARAMS)
    assert np.array_equal(lv, lv2) and np.array_equal(lo, lo2)


def _wide_mix():
    """Dense blocks from m = 200 down to m = 7 (ragged against every tile
    size), an arrow ball and a box: one launch holds items whose m differ by
    almost 30x."""
    return [I.gbase(200, 200, seed=61), I.gbase(37, 137, seed=62), I.arrow_ball(64), I.gbase(90, 65, seed=63),
            I.gbase(20, 33, seed=64), I.box(7, 1.0), I.gbase(12, 7, seed=65)]


def _wide_pairs(insts, chains, seed):
    """Per instance: interior starts at 10-90 % of the way to the boundary and
    starts 1e-6 short of it (as after a reflection), random directions."""
    from oracle import oracle as O
    rng = np.random.default_rng(seed)
    xs, vs = [], []
    for inst in insts:
        o = O.Oracle(inst)
        d = I.random_directions(rng, chains, inst.n)
        _, tp0, st0 = o.intersect(np.zeros((chains, inst.n)), d)
        assert (st0 == O.OK).all()
        f = np.where(np.arange(chains) % 3 == 2, 1 - 1e-6, rng.uniform(0.1, 0.9, chains))
        xs.append((f * tp0)[:, None] * d)
        vs.append(I.random_directions(rng, chains, inst.n))
    return xs, vs


def test_batch_intersect_wide_mix_matches_oracle(S):
    """One k_line_fused_multi launch over instances with m from 7 to 200 (and
    the per-class and per-instance launches): t- and t+ of every pair within
    1e-9 of the oracle's bisection on membership (plus the rounding bound of
    a root next to its start), statuses identical; the three strategies
    meet the same bar.  (The launches differ in workgroup size, which sets
    the summation order of the cross-wave reductions, so they agree to
    rounding, not bit for bit.)"""
    from oracle import oracle as O
    from root_bounds import root_bars
    insts = _wide_mix()
    chains = 6
    xs, vs = _wide_pairs(insts, chains, seed=71)
    b = S.Batch([S.Spectrahedron(i) for i in insts])
    out = {}
    for strategy in (1, 2, 3):
        b.set_strategy(strategy, False)
        out[strategy] = b.intersect(xs, vs)
    for k, inst in enumerate(insts):
        o = O.Oracle(inst)
        tm_e, tp_e, st_e = o.intersect(xs[k], vs[k])
        tm_r, tp_r, st_r = o.line_bisect(xs[k], vs[k], guess=np.stack([tm_e, tp_e], 1))
        bar_m, bar_p = root_bars(inst, xs[k], vs[k], tm_r, tp_r, 1e-9)
        for strategy, (tm, tp, st) in out.items():
            assert np.array_equal(st[k], st_r), (strategy, k, st[k], st_r)
            assert (np.abs(tm[k] - tm_r) <= bar_m).all(), (strategy, k, np.abs(tm[k] - tm_r) / bar_m)
            assert (np.abs(tp[k] - tp_r) <= bar_p).all(), (strategy, k, np.abs(tp[k] - tp_r) / bar_p)


def test_batch_intersect_rejects_reduced_precision(S):
    insts = [I.gbase(6, 14, seed=41), I.arrow_ball(5)]
    specs = [S.Spectrahedron(i) for i in insts]
    specs[0].set_precision(1)
    b = S.Batch(specs)
    x = [np.zeros((4, 6)), np.zeros((4, 5))]
    with pytest.raises(S.SpecError):
        b.intersect(x, [np.ones((4, 6)), np.ones((4, 5))])
