"""Walks on the device: identical random numbers to the oracle (first steps
match), per-segment parity on logged pairs, and stationary distributions."""
import math

import numpy as np
import pytest
import scipy.stats

from oracle import oracle as O
from paper_2010_03817_amd import instances as I
from root_bounds import root_bars

pytestmark = pytest.mark.gpu
T_REL = 1e-9
EPS = 2.220446049250313e-16


def _S():
    from paper_2010_03817_amd import spec as S
    return S


def _np(t):
    return None if t is None else t.detach().cpu().numpy()


def config1():
    return I.gbase(10, 10, seed=101, scale=math.sqrt(10))


def test_hnr_first_step_matches_oracle():
    """Same Philox stream (chain, step, draw, tag): one Hit-and-Run step from
    x0 = 0 lands on the same point as the oracle's."""
    S = _S()
    inst = config1()
    g, o = S.Spectrahedron(inst), O.Oracle(inst)
    x0 = np.zeros((64, 10))
    for kind in (S.HNR, S.CHNR):
        xg, _, st, _ = g.walk(kind, x0, 1, seed=201)
        xr, _, sr = o.walk(kind, x0, 1, seed=201)
        assert np.allclose(_np(xg), xr, rtol=1e-9, atol=1e-12)
        assert st["steps"] == 64 and st["calls"] == 64


def test_billiard_first_step_matches_oracle():
    S = _S()
    inst = config1()
    g, o = S.Spectrahedron(inst), O.Oracle(inst)
    x0 = np.zeros((64, 10))
    xg, _, st, _ = g.walk(S.BILLIARD, x0, 1, seed=202, tau=1.0)
    xr, _, sr = o.walk(O.BILLIARD, x0, 1, seed=202, tau=1.0)
    # the reflected directions agree to the Ritz-vector accuracy, so after a
    # few reflections the points agree to ~1e-6
    assert np.allclose(_np(xg), xr, atol=1e-6)
    assert st["reflections"] == sr[1] and st["calls"] == sr[0]


def test_carried_f_takes_the_same_steps():
    """Line walks assemble F(x) every refresh_period rounds and carry it over
    as F(x + s v) = F(x) + s B(v) in between: a billiard walk with the default
    period (16) and one that assembles every round take the same steps (the
    same calls and reflections, end points to the rounding that reflections
    amplify); with a reflection cap of one, chains sent back to their step
    start wait for the next assembly round, with the same cap hits and calls."""
    S = _S()
    inst = config1()
    x0 = np.zeros((64, 10))
    res = {}
    for per in (1, 16):
        g = S.Spectrahedron(inst, refresh_period=per)
        assert g.options()["refresh_period"] == per
        for rho in (0, 1):
            xg, _, st, _ = g.walk(S.BILLIARD, x0, 3, seed=505, tau=1.0, rho=rho)
            res[per, rho] = (_np(xg), st)
    for rho in (0, 1):
        (x1, s1), (x16, s16) = res[1, rho], res[16, rho]
        print(f"rho {rho}: rounds {s1['rounds']} / {s16['rounds']}, max |dx| {np.abs(x16 - x1).max():.2e}")
        for k in ("calls", "reflections", "cap_hits", "steps", "not_interior"):
            assert s1[k] == s16[k], (rho, k, s1[k], s16[k])
        assert np.allclose(x16, x1, atol=1e-6)
    assert res[1, 0][1]["rounds"] > 16  # rounds past the first refresh period
    assert res[1, 1][1]["cap_hits"] > 0
    assert res[16, 1][1]["rounds"] > res[1, 1][1]["rounds"]  # the chains sent back waited
    with pytest.raises(S.SpecError):
        S.Spectrahedron(inst, refresh_period=0)


def test_carried_f_rows_feed_the_later_passes():
    """In a round that carries F(x) over, the fused kernel writes F(x) to its
    block for the passes that read it later: the refining pass (far roots
    from a shifted origin) and the two-sided Cholesky certificate, which
    factors F(x) + t B(v) at t+ (1 -+ 1e-9).  Every certificate of a billiard
    walk over 40 rounds (two full assemblies) holds."""
    S = _S()
    inst = I.gbase(50, 60, seed=102)
    g = S.Spectrahedron(inst, certify=1)
    _, _, st, _ = g.walk(S.BILLIARD, np.zeros((256, 50)), 1 << 30, seed=303, tau=2.0, max_rounds=40)
    print(st)
    assert st["rounds"] == 40 and st["calls"] == 256 * 40
    assert st["refined"] > 0 and st["reflections"] > 0
    assert st["chol_cert_failed"] == 0 and st["not_interior"] == 0


@pytest.mark.parametrize("kind", ["hnr", "billiard"])
def test_logged_pairs_parity(kind):
    """Per-segment t+- of a running walk against the oracle recomputing the
    logged (x, v) pairs (post-reflection starts included) by bisection on
    membership (exact to adjacent doubles at any conditioning of F(x)); the
    eigen route of the oracle agrees with it from interior starts."""
    S = _S()
    inst = I.gbase(50, 60, seed=102)
    g, o = S.Spectrahedron(inst), O.Oracle(inst)
    k = S.HNR if kind == "hnr" else S.BILLIARD
    x0 = np.zeros((256, 50))
    xg, _, st, log = g.walk(k, x0, 20, seed=301, tau=2.0, log_chains=256, log_cap=400)
    log = _np(log)
    assert len(log) == 400
    n = 50
    x, v, tm, tp = log[:, :n], log[:, n:2 * n], log[:, 2 * n], log[:, 2 * n + 1]
    tm_r, tp_r, st_r = o.line_bisect(x, v)
    assert (st_r == O.OK).all()
    # the far root meets 1e-9 at every start; the root next to a start on the
    # boundary is fixed by F(x) only to the rounding bound of root_bounds
    near_m = np.abs(tm_r) < tp_r
    bar_m, bar_p = root_bars(inst, x, v, tm_r, tp_r, T_REL)
    dp = np.abs(tp - tp_r)
    assert (dp <= bar_p).all(), (dp / bar_p).max()
    assert (dp / tp_r)[near_m].max(initial=0) <= T_REL
    assert st["not_interior"] == 0
    if kind == "hnr":
        dm = np.abs(tm - tm_r)
        assert (dm <= bar_m).all(), (dm / bar_m).max()
    else:  # the billiard only converges lambda_min; t- is not reported
        assert np.isnan(tm).all()


def test_hnr_uniform_box_and_chnr():
    S = _S()
    n = 3
    g = S.Spectrahedron(I.box(n, 1.0))
    for kind in (S.HNR, S.CHNR):
        xg, smp, st, _ = g.walk(kind, np.zeros((256, n)), 200, seed=7, thin=20)
        pts = _np(smp)[:, 3:].reshape(-1, n)
        for i in range(n):
            assert scipy.stats.kstest((pts[:, i] + 1) / 2, "uniform").pvalue > 1e-3


def test_billiard_uniform_on_ball():
    S = _S()
    n = 5
    g = S.Spectrahedron(I.arrow_ball(n))
    xg, smp, st, _ = g.walk(S.BILLIARD, np.zeros((512, n)), 100, seed=8, tau=2.0, thin=10)
    r2 = (_np(smp)[:, 2:] ** 2).sum(-1).ravel()
    se = r2.std() / math.sqrt(len(r2) / 4)
    assert abs(r2.mean() - n / (n + 2)) < 4 * se


def test_gaussian_hnr_on_ball():
    S = _S()
    n, sigma = 4, 0.6
    g = S.Spectrahedron(I.arrow_ball(n))
    xg, smp, st, _ = g.walk(S.HNR, np.zeros((512, n)), 100, seed=10, gauss_a=1 / (2 * sigma**2), thin=10)
    c = 1 / sigma**2
    want = n * sigma**2 * scipy.stats.chi2.cdf(c, n + 2) / scipy.stats.chi2.cdf(c, n)
    r2 = (_np(smp)[:, 2:] ** 2).sum(-1).ravel()
    se = r2.std() / math.sqrt(len(r2) / 4)
    assert abs(r2.mean() - want) < 4 * se


@pytest.mark.parametrize("kind", ["hnr", "billiard"])
def test_config1_coordinate_means_match_oracle(kind):
    """The small workload in full: 64 chains x 1000 steps from 0 on the GPU and
    on the oracle; coordinate means of the second half agree within their
    Monte-Carlo error (chains are independent; thinned samples)."""
    S = _S()
    inst = config1()
    g, o = S.Spectrahedron(inst), O.Oracle(inst)
    k = S.HNR if kind == "hnr" else S.BILLIARD
    x0 = np.zeros((64, 10))
    _, sg, st, _ = g.walk(k, x0, 1000, seed=401, tau=1.0, thin=10)
    _, sr, _ = o.walk(k, x0, 1000, seed=402, tau=1.0, thin=10)
    a, b = _np(sg)[:, 50:], sr[:, 50:]
    ma, mb = a.mean((0, 1)), b.mean((0, 1))
    # chain-level means are independent across chains
    sa = a.mean(1).std(0) / math.sqrt(64)
    sb = b.mean(1).std(0) / math.sqrt(64)
    z = np.abs(ma - mb) / np.sqrt(sa**2 + sb**2)
    assert (z < 4.5).all(), z
    # a step can land outside S only when t+ is off by more than the 1e-6
    # pull-back
    assert st["not_interior"] == 0


def test_host_walk_matches_device_walk():
    """spec_walk_run (host arrays) runs the same chains as spec_walk_run_dev."""
    S = _S()
    inst = config1()
    g = S.Spectrahedron(inst)
    x0 = np.zeros((32, 10))
    for kind in (S.HNR, S.BILLIARD):
        xh, sh, sth = g.walk_host(kind, x0, 6, seed=55, tau=1.0, thin=2)
        xd, sd, std, _ = g.walk(kind, x0, 6, seed=55, tau=1.0, thin=2)
        assert np.array_equal(xh, _np(xd)) and np.array_equal(sh, _np(sd))
        assert sth == std
