"""t+ at the full size n = m = 200 (the benchmark's instance, seed 103) on
billiard-walk segment starts, post-reflection starts included, against the
oracle's bisection on Cholesky membership: the definition of t+ (Lemma "PEP
and S cap C": the end of the feasible interval), exact to adjacent doubles and
independent of the conditioning of F(x) at the start.  The plain path and the
learned-bracket path are both held to 1e-9 relative.

The near root t- of a start pulled back 1e-6 t+ from the boundary is itself
fixed by F(x) only to the rounding of its assembly and factorisation, which
moves it by up to the first-order bound of root_bounds.near_root_bound (two
correct methods differ by that much), so t- is held to 1e-9 |t-| plus that
bound."""
import concurrent.futures as cf

import numpy as np
import pytest

from oracle import oracle as O
from paper_2010_03817_amd import instances as I
from root_bounds import root_bars

pytestmark = pytest.mark.gpu
T_REL = 1e-9
EPS = 2.220446049250313e-16
N = M = 200


def _S():
    from paper_2010_03817_amd import spec as S
    return S


def bisect_threads(o, x, v, workers=16):
    """The oracle's bisection over chunks of pairs in threads (the C library
    releases the interpreter lock while it runs)."""
    tm, tp = np.empty(len(x)), np.empty(len(x))
    st = np.empty(len(x), dtype=np.int32)
    chunks = [c for c in np.array_split(np.arange(len(x)), min(workers, len(x))) if len(c)]

    def job(ix):
        a, b, s = o.line_bisect(x[ix], v[ix])
        tm[ix], tp[ix], st[ix] = a, b, s

    with cf.ThreadPoolExecutor(len(chunks)) as ex:
        list(ex.map(job, chunks))
    return tm, tp, st


def billiard_log(S, g, chains, rounds, tau, seed):
    _, _, st, log = g.walk(S.BILLIARD, np.zeros((chains, N)), 1 << 30, seed=seed, tau=tau, max_rounds=rounds,
                           log_chains=chains, log_cap=chains * rounds)
    return st, log.cpu().numpy()


@pytest.fixture(scope="module")
def wl():
    S = _S()
    inst = I.gbase(N, M, seed=103)
    g = S.Spectrahedron(inst)
    o = O.Oracle(inst)
    # tau = 2 x the longest chord of a 64-chain Hit-and-Run pre-run (as the benchmark)
    _, _, _, log = g.walk(S.HNR, np.zeros((64, N)), 20, seed=11, log_chains=64, log_cap=64 * 20)
    lg = log.cpu().numpy()
    tau = 2.0 * float(np.max(lg[:, 2 * N + 1] - lg[:, 2 * N]))
    st, log = billiard_log(S, g, 256, 30, tau, seed=2024)
    print(f"plain walk: {st}")
    assert st["not_interior"] == 0 and st["noconv"] == 0
    pick = np.linspace(0, len(log) - 1, 96).astype(int)
    x, v, tpw = log[pick, :N].copy(), log[pick, N:2 * N].copy(), log[pick, 2 * N + 1].copy()
    rtm, rtp, rst = bisect_threads(o, x, v)
    assert (rst == O.OK).all()
    kappa = (rtp - rtm) / np.abs(rtm)
    post = kappa > 1e4  # starts next to the boundary (after a reflection)
    print(f"{post.sum()} of {len(x)} pairs start next to the boundary; kappa up to {kappa.max():.2e}")
    assert post.sum() >= 32 and (~post).sum() >= 1
    return dict(S=S, inst=inst, g=g, o=o, tau=tau, x=x, v=v, tpw=tpw, rtm=rtm, rtp=rtp, kappa=kappa, post=post,
                walk_stats=st)


def rel(a, b):
    return np.abs(a - b) / np.abs(b)


def report(name, r, kappa):
    w = np.argsort(-r)[:4]
    print(f"{name}: max {r.max():.2e} median {np.median(r):.2e}; worst at kappa "
          + ", ".join(f"{kappa[i]:.1e}" for i in w))


def test_plain_walk_logged_tplus(wl):
    """The t+ the plain walk itself used for its segments."""
    r = rel(wl["tpw"], wl["rtp"])
    report("plain walk log", r, wl["kappa"])
    assert r.max() <= T_REL
    st = wl["walk_stats"]
    assert st["refined"] > 0.5 * st["calls"]  # most segments start after a reflection


def test_plain_reflect_and_intersect(wl):
    S, g = wl["S"], wl["g"]
    tp, s, w, st = g.reflect(wl["x"], wl["v"])
    tp, st = tp.cpu().numpy(), st.cpu().numpy()
    assert set(np.unique(st)) <= {S.OK, S.NONSMOOTH}
    r = rel(tp, wl["rtp"])
    report("plain reflect", r, wl["kappa"])
    assert r.max() <= T_REL
    tm, tp2, st2 = g.intersect(wl["x"], wl["v"])
    tm, tp2 = tm.cpu().numpy(), tp2.cpu().numpy()
    assert (st2.cpu().numpy() == S.OK).all()
    r2 = rel(tp2, wl["rtp"])
    report("plain intersect t+", r2, wl["kappa"])
    assert r2.max() <= T_REL
    bar_m, _ = root_bars(wl["inst"], wl["x"], wl["v"], wl["rtm"], wl["rtp"], T_REL)
    dm = np.abs(tm - wl["rtm"])
    print(f"plain intersect t-: max |diff| / bar {np.max(dm / bar_m):.3f}")
    assert np.all(dm <= bar_m), (dm / bar_m).max()


def test_unrefined_plain_path_loses_accuracy_near_the_boundary(wl):
    """Without the refining run the far root from a start next to the
    boundary carries ~eps rho / |lambda_min| (reported; the refined path is
    the one the walks use)."""
    g = wl["g"]
    g.set_options(refine_ratio=0.0)
    try:
        tp, _, _, _ = g.reflect(wl["x"], wl["v"])
    finally:
        g.set_options(refine_ratio=1e3)
    r = rel(tp.cpu().numpy(), wl["rtp"])
    report("plain reflect without refinement", r, wl["kappa"])
    post = wl["post"]
    print(f"  next to the boundary: max {r[post].max():.2e}; interior: max {r[~post].max():.2e}")
    assert r[~post].max() <= T_REL


def check_certificates(name, g, tp, rtp, B, wl=None):
    """Every certified interval holds the oracle's t+ and is at most 2e-9 t+
    wide, with the returned value as its upper end; most calls are certified.
    The interval certifies the root of the pencil as the device rounded it;
    the oracle's root differs from that by up to the first-order effect of the
    assembly and factorisation rounding (root_bounds.near_root_bound, which
    holds for any root), so that bound is the slack."""
    from root_bounds import near_root_bound
    lo, hi = g.certificates(B)
    fl = g.call_flags(B)
    cert = (fl & 32) == 0
    slack = 1e-13 * rtp
    if wl is not None:
        slack = np.maximum(slack, [near_root_bound(wl["inst"], wl["x"][k], wl["v"][k], rtp[k]) for k in range(B)])
    print(f"{name}: {int(cert.sum())} of {B} certified; widths up to {np.max((hi - lo)[cert] / hi[cert]):.1e}; "
          f"largest gap to the oracle {np.max(np.maximum(lo - rtp, rtp - hi)[cert] / rtp[cert]):.1e} (relative)")
    assert cert.mean() >= 0.9
    assert np.all(lo[cert] <= rtp[cert] + slack[cert]) and np.all(rtp[cert] <= hi[cert] + slack[cert])
    assert np.all(hi[cert] - lo[cert] <= 2e-9 * hi[cert])
    assert np.array_equal(hi, tp)


def test_plain_certificates(wl):
    """Kato-Temple intervals of the plain path (refined from the shifted
    origin near the boundary), and the optional two-sided Cholesky
    certificate: F(x + t v) definite at t+ (1 - 1e-9), not at t+ (1 + 1e-9)."""
    g = wl["g"]
    B = len(wl["x"])
    tp = g.reflect(wl["x"], wl["v"])[0].cpu().numpy()
    check_certificates("plain reflect", g, tp, wl["rtp"], B, wl)
    g.set_options(certify=1)
    try:
        tp2 = g.reflect(wl["x"], wl["v"])[0].cpu().numpy()
        fl = g.call_flags(B)
    finally:
        g.set_options(certify=0)
    assert np.array_equal(tp, tp2)
    print(f"two-sided Cholesky certificate failures: {int(np.sum(fl & 64 > 0))} of {B}")
    assert np.sum(fl & 64 > 0) == 0


def _train(S, g, tau, seed):
    """A network of the benchmark's shape trained on the walk's own segment
    starts (labels from the device oracle)."""
    st, log = billiard_log(S, g, 256, 60, tau, seed=seed)
    x, v = log[:, :N].copy(), log[:, N:2 * N].copy()
    tm, tp, sts = [t.cpu().numpy() for t in g.intersect(x, v)]
    keep = (sts == S.OK) & np.isfinite(tm) & np.isfinite(tp) & (tm < 0) & (tp > 0)
    net = S.Mlp(N, width=256, hidden=3, bf16=True, seed=5)
    tr = net.train(x[keep], v[keep], tm[keep], tp[keep], epochs=8, batch=1024, lr=1e-3)
    return net, tr


def test_learned_reflect_and_walk(wl):
    S, g, o = wl["S"], wl["g"], wl["o"]
    net, tr = _train(S, g, wl["tau"], seed=77)
    g.set_mlp(net, tr["err_q"][0.9], 1)
    try:
        tp, s, w, st = g.reflect(wl["x"], wl["v"])
        cert = g.lanczos_info(len(wl["x"]))[:, 2]
        tp = tp.cpu().numpy()
        check_certificates("learned reflect", g, tp, wl["rtp"], len(tp), wl)
        r = rel(tp, wl["rtp"])
        report("learned reflect", r, wl["kappa"])
        print(f"  certificate fallbacks {int((cert == 1).sum())} of {len(tp)}")
        assert set(np.unique(st.cpu().numpy())) <= {S.OK, S.NONSMOOTH, S.CERT_FALLBACK}
        assert r.max() <= T_REL
        # the learned walk's own segments
        stw, log = billiard_log(S, g, 256, 20, wl["tau"], seed=31)
    finally:
        g.set_mlp(None)
    print(f"learned walk: {stw}")
    assert stw["not_interior"] == 0 and stw["noconv"] == 0
    pick = np.linspace(0, len(log) - 1, 64).astype(int)
    x, v, tpw = log[pick, :N], log[pick, N:2 * N], log[pick, 2 * N + 1]
    _, rtp, rst = bisect_threads(o, x, v)
    assert (rst == O.OK).all()
    r = rel(tpw, rtp)
    print(f"learned walk log: max {r.max():.2e}")
    assert r.max() <= T_REL


def test_refine_backoff_after_a_loose_first_pass(wl):
    """With a first pass stopped far too early (loose tolerance 0.3) the
    first refining origin often lies past t+; the REFINE pass backs off
    (t1 (1 - 2^-5), then t1 / 2) and still returns t+ to 1e-9.  A pair whose
    every origin failed carries the plain solve at the full tolerance: the
    same value as with refinement off."""
    g = wl["g"]
    g.set_options(tol_loose=0.3)
    try:
        tp, _, _, st = g.reflect(wl["x"], wl["v"])
        fl = g.call_flags(len(wl["x"]))
        g.set_options(refine_ratio=0.0)
        tp_off = g.reflect(wl["x"], wl["v"])[0].cpu().numpy()
    finally:
        g.set_options(tol_loose=1e-3, refine_ratio=1e3)
    tp = tp.cpu().numpy()
    failed = (fl & 8) > 0
    r = rel(tp, wl["rtp"])
    report("reflect after a loose first pass", r, wl["kappa"])
    print(f"  refined {int(np.sum(fl & 4 > 0))}, refine failed {int(failed.sum())}")
    assert np.sum(fl & 4 > 0) >= 32
    assert r[~failed].max() <= T_REL
    assert np.array_equal(tp[failed], tp_off[failed])


def test_paper_generator_s200_walk_pairs():
    """S-200-200 of the paper's own generator (Section 4: A0 = Z Z^T + I,
    A_i = blkdiag(Qt, -Qt), no box block; the first instance of the
    walk-length table): the billiard walk's logged segment starts, post-
    reflection starts included, and Hit-and-Run chords against the oracle's
    bisection, t+ at 1e-9 and t- at 1e-9 plus the near-root rounding bound."""
    S = _S()
    inst = I.paper_random(N, M, seed=10000 + 100 * N)
    g, o = S.Spectrahedron(inst), O.Oracle(inst)
    _, _, _, log = g.walk(S.HNR, np.zeros((64, N)), 6, seed=12, log_chains=64, log_cap=64 * 6)
    hl = log.cpu().numpy()
    tau = 2.0 * float(np.max(hl[:, 2 * N + 1] - hl[:, 2 * N]))
    st, bl = billiard_log(S, g, 64, 12, tau, seed=13)
    print(f"paper S-200-200 billiard: {st}")
    assert st["not_interior"] == 0 and st["noconv"] == 0
    pick = np.linspace(0, len(bl) - 1, 40).astype(int)
    hpick = np.linspace(0, len(hl) - 1, 16).astype(int)
    x = np.concatenate([bl[pick, :N], hl[hpick, :N]])
    v = np.concatenate([bl[pick, N:2 * N], hl[hpick, N:2 * N]])
    rtm, rtp, rst = bisect_threads(o, x, v)
    assert (rst == O.OK).all()
    kappa = (rtp - rtm) / np.minimum(np.abs(rtm), rtp)
    print(f"kappa up to {kappa.max():.2e}; {int((kappa > 1e4).sum())} starts next to the boundary")
    assert (kappa > 1e4).sum() >= 16
    # the walks' own t+ (billiard) and t-, t+ (Hit-and-Run)
    r = rel(bl[pick, 2 * N + 1], rtp[:40])
    report("paper S-200-200 billiard log", r, kappa[:40])
    assert r.max() <= T_REL
    bar_m, bar_p = root_bars(inst, x, v, rtm, rtp, T_REL)
    assert np.all(np.abs(hl[hpick, 2 * N + 1] - rtp[40:]) <= bar_p[40:])
    assert np.all(np.abs(hl[hpick, 2 * N] - rtm[40:]) <= bar_m[40:])
    # the call-level oracle on the same pairs
    tm, tp, st2 = [t.cpu().numpy() for t in g.intersect(x, v)]
    assert (st2 == S.OK).all()
    assert np.all(np.abs(tp - rtp) <= bar_p), np.max(np.abs(tp - rtp) / bar_p)
    assert np.all(np.abs(tm - rtm) <= bar_m), np.max(np.abs(tm - rtm) / bar_m)


def _sampled_round(S, g, tau, chains, seed, warm_rounds, count):
    """Segment starts of one round of `chains` billiard chains (the benchmark's
    launch: one workgroup per chain over the whole grid), taken after
    `warm_rounds` rounds from the centre: the second round of a walk call, the
    first whose F(x) is carried over (F(x) + s B(v) from the round before),
    its record of `count` chains spread evenly over the grid."""
    import torch
    x0 = torch.zeros((chains, N), dtype=torch.float64, device="cuda")
    g.walk(S.BILLIARD, x0, 1 << 30, seed=seed, tau=tau, max_rounds=warm_rounds)
    _, _, st, log = g.walk(S.BILLIARD, x0, 1 << 30, seed=seed, tau=tau, max_rounds=2, resume=True,
                           log_chains=chains, log_cap=2 * chains)
    log = log.cpu().numpy()[chains:]  # every chain logs once in the first round
    order = np.argsort(log[:, 2 * N + 2])
    log = log[order]
    pick = np.linspace(0, len(log) - 1, count).astype(int)
    return st, log[pick]


@pytest.mark.parametrize("path", ["plain", "learned"])
def test_bench_launch_of_16384_chains_sampled(wl, path):
    """The benchmark's launch configuration (16384 chains at n = m = 200): t+ of
    96 sampled segment starts of one round with F(x) carried over, 21 rounds
    from the centre (post-reflection starts included), against the oracle's
    bisection."""
    S, g, o = wl["S"], wl["g"], wl["o"]
    if path == "learned":
        net, tr = _train(S, g, wl["tau"], seed=78)
        g.set_mlp(net, tr["err_q"][0.9], 1)
    try:
        st, log = _sampled_round(S, g, wl["tau"], 16384, seed=4242, warm_rounds=20, count=96)
    finally:
        g.set_mlp(None)
    assert len(log) == 96 and st["not_interior"] == 0 and st["noconv"] == 0
    chains = log[:, 2 * N + 2].astype(int)
    assert len(np.unique(chains)) == 96 and chains.max() > 16000  # spread over the grid
    x, v, tpw = log[:, :N], log[:, N:2 * N], log[:, 2 * N + 1]
    rtm, rtp, rst = bisect_threads(o, x, v)
    assert (rst == O.OK).all()
    kappa = (rtp - rtm) / np.abs(rtm)
    r = rel(tpw, rtp)
    report(f"16384-chain {path} round", r, kappa)
    print(f"  {int((kappa > 1e4).sum())} of 96 start next to the boundary")
    assert r.max() <= T_REL
