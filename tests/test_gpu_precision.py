"""GPU tests of the reduced-precision pencil assembly (FP32 MFMA, BF16 hi+lo
pairs): the assembled pencils' rounding bounds the t+- error against the FP64
mode, which itself matches the oracle."""
import math

import numpy as np
import pytest

from paper_2010_03817_amd import instances as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_2010_03817_amd import spec
    return spec


@pytest.mark.parametrize("mode,bar", [(1, 2e-5), (2, 5e-4)])
def test_reduced_assembly_error(S, mode, bar):
    inst = I.gbase(40, 40, seed=66)
    g = S.Spectrahedron(inst)
    rng = np.random.default_rng(2)
    B = 512
    v = I.random_directions(rng, B, 40)
    x = 0.3 * I.random_directions(rng, B, 40) * rng.uniform(0, 1, (B, 1))
    tm0, tp0, st0 = g.intersect(x, v)
    g.set_precision(mode)
    tm1, tp1, st1 = g.intersect(x, v)
    tp2, s2, w2, st2 = g.reflect(x, v)
    g.set_precision(S.PREC_FP64)
    tm3, tp3, st3 = g.intersect(x, v)
    tp0, tp1, tm0, tm1 = (t.cpu().numpy() for t in (tp0, tp1, tm0, tm1))
    assert np.array_equal(tp3.cpu().numpy(), tp0)  # back to FP64: same results
    ok = (st0.cpu().numpy() == 0) & (st1.cpu().numpy() == 0)
    assert ok.mean() > 0.99
    e_tp = np.abs(tp1 - tp0)[ok] / tp0[ok]
    e_tm = np.abs(tm1 - tm0)[ok] / -tm0[ok]
    print(f"mode {mode}: t+ rel err median {np.median(e_tp):.2e} p99 {np.quantile(e_tp, .99):.2e} "
          f"max {e_tp.max():.2e}; t- max {e_tm.max():.2e}")
    assert np.median(e_tp) < bar / 10
    assert e_tp.max() < bar and e_tm.max() < bar
    # a reduced-precision assembly does change the result (not silently FP64)
    assert e_tp.max() > 1e-12


def _bisect_threads(fn, items, workers=16):
    import concurrent.futures as cf
    chunks = [c for c in np.array_split(np.arange(len(items)), min(workers, len(items))) if len(c)]
    out = [None] * len(chunks)

    def job(k):
        out[k] = fn(items[chunks[k]])

    with cf.ThreadPoolExecutor(len(chunks)) as ex:
        list(ex.map(job, range(len(chunks))))
    return [np.concatenate([o[i] for o in out]) for i in range(len(out[0]))]


def test_hmc_segments_precision_split_full_size(S):
    """The precision split on the Gaussian HMC workload at n = m = 200: the
    segments of an FP64 walk (sigma = 1, many starting next to the boundary
    after a reflection) solved with FP64, FP32 and BF16 hi+lo pencils.  With
    escalation (FP64 pencils again when the reduced-precision F(p) has min
    pivot / max pivot below 1e-3, is not definite, or the curve meets the
    boundary) every segment agrees with FP64 on whether the curve meets the
    boundary within its horizon, and the escalated ones equal FP64 to 1e-9.
    On this walk nearly every segment starts at a reflection point pulled
    back by a relative 1e-6 (kappa(F(p)) ~ 1e6) and ends at the boundary, so
    the rule sends nearly every call back to FP64; without it the reduced
    pencils disagree with FP64 on the hit in over a thousand segments.  The
    FP64 roots match the oracle's degree-2 solver on a sample."""
    from oracle import oracle as O
    n = 200
    inst = I.gbase(n, n, seed=103)
    g = S.Spectrahedron(inst)
    chains = 2048
    x0 = np.zeros((chains, n))
    _, _, st, log = g.walk(S.HMC, x0, 1 << 30, seed=77, gauss_a=0.5, tau=1.48, max_rounds=8,
                           log_chains=chains, log_cap=chains * 8)
    log = log.cpu().numpy()
    p, v = log[:, :n], log[:, n:2 * n]
    coef = np.zeros((len(log), 3, n + 1))
    coef[:, 0, 0], coef[:, 0, 1:] = 1.0, p
    coef[:, 1, 1:] = 2.0 * v
    coef[:, 2, 0], coef[:, 2, 1:] = 1.0, -p
    tp64_walk = None
    for hz in (1.0,):
        _, tp64, st64 = [t.cpu().numpy() for t in g.intersect_curve(coef, hz)]
        assert (st64 == S.OK).mean() > 0.99
        ok64 = st64 == S.OK
        if hz == 1.0:
            tp64_walk = tp64
        for mode in (S.PREC_FP32_ASM, S.PREC_BF16X2_ASM):
            g.set_precision(mode)
            try:
                _, tp, st1 = [t.cpu().numpy() for t in g.intersect_curve(coef, hz)]
                esc = (g.call_flags(len(coef)) & 128) > 0
                g.set_options(escalate_ratio=0.0)
                _, tpn, stn = [t.cpu().numpy() for t in g.intersect_curve(coef, hz)]
                g.set_options(escalate_ratio=1e-3)
            finally:
                g.set_precision(S.PREC_FP64)
            # a reduced-precision start that is not definite is decided by FP64
            assert np.all(st1[ok64] == S.OK)
            ok = ok64 & (st1 == S.OK)
            hit64, hit = np.isfinite(tp64), np.isfinite(tp)
            dis = (hit64 != hit) & ok
            dis_noesc = ((np.isfinite(tpn) != hit64) | (stn != S.OK)) & ok64
            both = ok & hit64 & hit
            rel = np.abs(tp - tp64)[both] / tp64[both]
            print(f"horizon {hz}, mode {mode}: escalated {esc.mean():.3f}; hit/no-hit disagreements "
                  f"{int(dis.sum())} (without escalation {int(dis_noesc.sum())}); segments kept reduced "
                  f"{int((~esc).sum())}")
            assert not np.any(dis)
            # every hit is redone in FP64 (its reflection needs the FP64 root)
            assert np.all(esc[ok64 & hit64])
            assert rel[esc[both]].max(initial=0) <= 1e-9
            assert dis_noesc.sum() > 0  # the rule is what removes the disagreements
    # the FP64 roots against the oracle on a sample (its Jacobi route at m = 200)
    o = O.Oracle(inst)
    idx = np.linspace(0, len(coef) - 1, 16).astype(int)
    otm, otp, ost, _ = _bisect_threads(lambda c: o.intersect_curve2(c, 1.0), coef[idx])
    sel = ost == O.OK
    assert sel.sum() >= 12
    fin = np.isfinite(otp[sel])
    assert np.array_equal(fin, np.isfinite(tp64_walk[idx][sel]))
    r = np.abs(tp64_walk[idx][sel][fin] - otp[sel][fin]) / otp[sel][fin]
    print(f"FP64 first roots against the oracle: max rel {r.max(initial=0):.2e} over {int(fin.sum())}")
    assert r.max(initial=0) <= 1e-9
