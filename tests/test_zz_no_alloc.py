"""spec_intersect_noalloc_dev (static scratch, no allocation) against
spec_intersect_dev: identical t-, t+ and statuses on two calls in a row, the
second with a smaller batch, on billiard walk states of the n = m = 200
instance (post-reflection starts, so the refining pass runs) and on a small
instance; a batch beyond the static scratch is refused."""
import numpy as np
import pytest

from paper_2010_03817_amd import instances as I

pytestmark = pytest.mark.gpu


def _S():
    from paper_2010_03817_amd import spec as S
    return S


def _walk_pairs(S, g, n, chains, rounds):
    _, _, _, log = g.walk(S.BILLIARD, np.zeros((chains, n)), 1 << 30, seed=7, tau=1.5, max_rounds=rounds,
                          log_chains=chains, log_cap=chains * rounds)
    log = log.cpu().numpy()
    return log[:, :n].copy(), log[:, n:2 * n].copy()


@pytest.mark.parametrize("n,m,sizes", [(200, 200, (128, 37)), (20, 24, (300, 5))])
def test_noalloc_matches_intersect(n, m, sizes):
    import torch
    S = _S()
    g = S.Spectrahedron(I.gbase(n, m, seed=103 if n == 200 else 5))
    x, v = _walk_pairs(S, g, n, 64, 8)
    cap = max(sizes)
    tm = torch.full((cap,), -7.0, dtype=torch.float64, device="cuda")
    tp = torch.full((cap,), -7.0, dtype=torch.float64, device="cuda")
    st = torch.full((cap,), -7, dtype=torch.int32, device="cuda")
    for B in sizes:
        assert B <= len(x)
        xs, vs = x[-B:], v[-B:]
        a_tm, a_tp, a_st = [t.cpu().numpy() for t in g.intersect(xs, vs)]
        b_tm, b_tp, b_st = [t.cpu().numpy() for t in g.intersect_noalloc(xs, vs, tm, tp, st)]
        assert np.array_equal(a_st, b_st)
        assert np.array_equal(a_tp, b_tp)
        assert np.array_equal(np.isnan(a_tm), np.isnan(b_tm))
        assert np.array_equal(a_tm[~np.isnan(a_tm)], b_tm[~np.isnan(b_tm)])
        assert (a_st == S.OK).mean() > 0.9
    # beyond the static scratch: refused before any work
    if n == 200:
        big = 1024
        xb = np.repeat(x[:1], big, 0)
        vb = np.repeat(v[:1], big, 0)
        o = torch.empty(big, dtype=torch.float64, device="cuda")
        o2 = torch.empty(big, dtype=torch.float64, device="cuda")
        s2 = torch.empty(big, dtype=torch.int32, device="cuda")
        with pytest.raises(S.SpecError):
            g.intersect_noalloc(xb, vb, o, o2, s2)
