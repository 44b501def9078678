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
    specs = [S.Spectrahedron(i) for i in insts]
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
        g = S.Spectrahedron(insts[k])
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
