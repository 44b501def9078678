"""Parity of the HIP line oracle (intersect / reflect / membership) with the
FP64 CPU oracle on identical inputs, through the C ABI."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2010_03817_amd import instances as I

pytestmark = pytest.mark.gpu

# Tolerance for t+- (relative), the bar of the FP64 path.
T_REL = 1e-9


def _spec():
    from paper_2010_03817_amd import spec as S
    return S


def _np(t):
    return t.detach().cpu().numpy()


def _points(o, inst, rng, batch, frac_lo=0.0, frac_hi=0.95):
    d = I.random_directions(rng, batch, inst.n)
    tp0 = o.intersect(np.zeros((batch, inst.n)), d)[1]
    f = rng.uniform(frac_lo, frac_hi, batch)
    x = (f * np.minimum(tp0, 50.0))[:, None] * d
    v = I.random_directions(rng, batch, inst.n)
    return x, v


def test_mfma_f64_lane_layout():
    """Accumulator r of lane l holds D[l/16 + 4 r][l % 16] (the layout the
    GEMM epilogue writes)."""
    out = _spec().mfma_layout()
    got = [[(int(out[l, r]) % 1000, int(out[l, r]) // 1000) for r in range(4)] for l in range(64)]
    print(got)
    for lane in range(64):
        for r in range(4):
            assert got[lane][r] == (lane // 16 + 4 * r, lane % 16)


@pytest.mark.parametrize("transB", [False, True])
@pytest.mark.parametrize("shape", [(128, 192, 48), (256, 384, 80), (128, 128, 16), (384, 256, 208),
                                   (256, 256, 8192), (128, 256, 4112)])
def test_gemm_f64(transB, shape):
    """64- and 128-wide tilings (the latter when M and N are multiples of 128),
    odd and even numbers of K slices, and the split into two K halves added
    into a zeroed output (few tiles, long K), against numpy."""
    rng = np.random.default_rng(1)
    M, N, K = shape
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((N, K)) if transB else rng.standard_normal((K, N))
    Cg = _spec().gemm_f64(A, B, transB)
    Cr = A @ (B.T if transB else B)
    assert np.allclose(Cg, Cr, rtol=1e-13, atol=1e-13 * np.abs(Cr).max())


@pytest.mark.parametrize("shape", [(64, 208, 16), (192, 208, 4112), (640, 208, 80), (1024, 208, 4112),
                                   (16384, 208, 20112)])
def test_gemm_f64_narrow_transposed(shape):
    """The 208-column transposed product of the boundary normal (n = 200):
    one K slice, several tiles, the split into two K halves (odd slice count)
    and the full shape of 16384 chains at m = 200, against numpy (the last on
    a sample of rows)."""
    rng = np.random.default_rng(2)
    M, N, K = shape
    A = rng.standard_normal((M, K))
    B = rng.standard_normal((N, K))
    Cg = _spec().gemm_f64(A, B, True)
    rows = np.arange(M) if M <= 1024 else np.linspace(0, M - 1, 97).astype(int)
    Cr = A[rows] @ B.T
    assert np.allclose(Cg[rows], Cr, rtol=1e-13, atol=1e-13 * np.abs(Cr).max())


def _check_intersect(inst, batch, seed, frac_hi=0.95, rel=T_REL):
    S = _spec()
    o = O.Oracle(inst)
    g = S.Spectrahedron(inst)
    rng = np.random.default_rng(seed)
    x, v = _points(o, inst, rng, batch, 0.0, frac_hi)
    tm_r, tp_r, st_r = o.intersect(x, v)
    tm, tp, st = g.intersect(x, v)
    tm, tp, st = _np(tm), _np(tp), _np(st)
    assert np.array_equal(st, st_r), (st, st_r)
    ok = st_r == O.OK
    assert np.allclose(tp[ok], tp_r[ok], rtol=rel, atol=0)
    assert np.allclose(tm[ok], tm_r[ok], rtol=rel, atol=0)
    return g, o, x, v


def test_intersect_config1_small():
    """n = m = 10 with the box block (the small workload), 64 pairs."""
    _check_intersect(I.gbase(10, 10, seed=101, scale=math.sqrt(10)), 64, 1)


def test_intersect_ragged_sizes():
    """Sizes spanning several tiles with ragged tails."""
    for n, m, b in [(37, 45, 70), (70, 19, 65), (5, 130, 17)]:
        _check_intersect(I.gbase(n, m, seed=n + m), b, n)


def test_intersect_full_size_sampled():
    """n = m = 200 (+400 box rows), sampled pairs."""
    _check_intersect(I.gbase(200, 200, seed=103), 12, 3)


def test_intersect_special_bodies():
    # polytope only (no dense block), arrow ball, the paper's 2-D example
    rng = np.random.default_rng(4)
    Amat = rng.standard_normal((23, 6))
    _check_intersect(I.polytope(Amat, rng.uniform(0.5, 2, 23)), 40, 4)
    _check_intersect(I.arrow_ball(9), 40, 5)
    S = _spec()
    ex = I.paper_example_2d()
    g = S.Spectrahedron(ex)
    tm, tp, st = g.intersect(np.array([[-1.0, 1.0]]), np.array([[1.3, 0.8]]))
    tm_r, tp_r, _ = O.Oracle(ex).intersect(np.array([[-1.0, 1.0]]), np.array([[1.3, 0.8]]))
    assert _np(tp)[0] == pytest.approx(tp_r[0], rel=T_REL)
    assert _np(tm)[0] == pytest.approx(tm_r[0], rel=T_REL)


def test_extreme_scale_pivots():
    """F and B scaled by 1e285 and by 1e-285: pivots outside (1e-280, 1e280)
    send the diagonal tiles to the square-root-per-column factorisation; t+-
    and membership are invariant under the scaling, so the oracle of the
    unscaled instance is the reference."""
    S = _spec()
    inst = I.gbase(30, 40, seed=9)
    o = O.Oracle(inst)
    rng = np.random.default_rng(9)
    x, v = _points(o, inst, rng, 24)
    tm_r, tp_r, st_r = o.intersect(x, v)
    dm = I.random_directions(rng, 64, inst.n)
    xm = (rng.uniform(0.0, 1.5, 64) * o.intersect(np.zeros((64, inst.n)), dm)[1])[:, None] * dm
    mem_r = o.membership(xm)
    assert 0 < mem_r.sum() < len(mem_r)
    for c in (1e285, 1e-285):
        blocks = [I.Block(b.kind, b.A * c) for b in inst.blocks]
        g = S.Spectrahedron(I.Instance(inst.n, blocks))
        tm, tp, st = [_np(a) for a in g.intersect(x, v)]
        assert np.array_equal(st, st_r), (c, st, st_r)
        ok = st_r == O.OK
        assert np.allclose(tp[ok], tp_r[ok], rtol=T_REL, atol=0), c
        assert np.allclose(tm[ok], tm_r[ok], rtol=T_REL, atol=0), c
        assert np.array_equal(_np(g.membership(xm)), mem_r), c


def test_intersect_near_boundary():
    """Points pulled back from the boundary by 1e-6 (the post-reflection
    starts of the billiard walk), bucketed by the conditioning of F."""
    inst = I.gbase(40, 50, seed=7)
    S = _spec()
    o, g = O.Oracle(inst), S.Spectrahedron(inst)
    rng = np.random.default_rng(7)
    d = I.random_directions(rng, 48, inst.n)
    x0 = 0.3 * d * o.intersect(np.zeros((48, inst.n)), d)[1][:, None]
    u = I.random_directions(rng, 48, inst.n)
    tp0 = o.intersect(x0, u)[1]
    x = x0 + (1 - 1e-6) * tp0[:, None] * u
    v = I.random_directions(rng, 48, inst.n)
    # reference: bisection on membership (exact at any conditioning of F(x))
    tm_r, tp_r, st_r = o.line_bisect(x, v)
    tm, tp, st = [_np(a) for a in g.intersect(x, v)]
    ok = st_r == O.OK
    assert ok.sum() > 40
    # the far side meets 1e-9; the root next to the start is fixed by F(x)
    # only to the rounding bound of root_bounds (two correct methods differ
    # by that much)
    from root_bounds import root_bars
    bar_m, bar_p = root_bars(inst, x[ok], v[ok], tm_r[ok], tp_r[ok], T_REL)
    assert (np.abs(tp[ok] - tp_r[ok]) <= bar_p).all()
    assert (np.abs(tm[ok] - tm_r[ok]) <= bar_m).all()
    near = np.minimum(np.abs(tm_r), tp_r)
    for arr, ref in ((tp, tp_r), (tm, tm_r)):
        far = ok & (np.abs(ref) > near)
        assert (np.abs(arr - ref)[far] <= T_REL * np.abs(ref[far])).all()


def test_reflect_parity():
    for inst, batch, seed in [(I.gbase(10, 10, seed=101, scale=math.sqrt(10)), 64, 11),
                              (I.gbase(30, 41, seed=12), 50, 12), (I.arrow_ball(7), 30, 13)]:
        S = _spec()
        o, g = O.Oracle(inst), S.Spectrahedron(inst)
        rng = np.random.default_rng(seed)
        x, v = _points(o, inst, rng, batch)
        tp_r, s_r, w_r, st_r = o.reflect(x, v)
        tp, s, w, st = [_np(a) for a in g.reflect(x, v)]
        ok = st_r == O.OK
        assert np.array_equal(st[ok], st_r[ok])
        assert np.allclose(tp[ok], tp_r[ok], rtol=T_REL, atol=0)
        # normal and reflected direction: Ritz-vector accuracy
        assert np.allclose(w[ok], w_r[ok], atol=1e-7)
        assert np.allclose(s[ok], s_r[ok], atol=2e-7)


def test_reflect_full_size_sampled():
    inst = I.gbase(200, 200, seed=103)
    S = _spec()
    o, g = O.Oracle(inst), S.Spectrahedron(inst)
    rng = np.random.default_rng(14)
    x, v = _points(o, inst, rng, 6)
    tp_r, s_r, w_r, st_r = o.reflect(x, v)
    tp, s, w, st = [_np(a) for a in g.reflect(x, v)]
    assert np.allclose(tp, tp_r, rtol=T_REL, atol=0)
    assert np.allclose(w, w_r, atol=1e-7)
    assert np.allclose(s, s_r, atol=2e-7)


def test_membership_and_statuses():
    S = _spec()
    inst = I.gbase(8, 12, seed=15)
    o, g = O.Oracle(inst), S.Spectrahedron(inst)
    rng = np.random.default_rng(15)
    x = rng.standard_normal((200, 8)) * 0.6
    assert np.array_equal(_np(g.membership(x)), o.membership(x))
    # outside point: NOT_INTERIOR with NaN values, and a NaN certificate
    # beside an interior call's [t_lo, t+] (an interior call first, so that a
    # stale interval would show)
    xs = np.vstack([np.zeros((1, 8)), np.full((1, 8), 20.0)])
    g.intersect(np.zeros((2, 8)), np.ones((2, 8)))
    tm, tp, st = [_np(a) for a in g.intersect(xs, np.ones((2, 8)))]
    assert st[1] == S.NOT_INTERIOR and np.isnan(tp[1]) and np.isnan(tm[1])
    lo, hi = g.certificates(2)
    assert st[0] == S.OK and hi[0] == tp[0] and lo[0] <= tp[0]
    assert np.isnan(lo[1]) and np.isnan(hi[1])
    # a half-space is unbounded
    hs = I.polytope(np.array([[1.0, 0.0]]), np.array([1.0]))
    tm, tp, st = [_np(a) for a in S.Spectrahedron(hs).intersect(np.zeros((2, 2)), np.array([[0.0, 1.0], [1, 0]]))]
    assert st[0] == S.UNBOUNDED and tp[0] == np.inf and tm[0] == -np.inf
    assert st[1] == S.UNBOUNDED and tp[1] == pytest.approx(1.0) and tm[1] == -np.inf


def test_empty_batch_and_repeat_calls():
    S = _spec()
    inst = I.gbase(6, 9, seed=16)
    g = S.Spectrahedron(inst)
    tm, tp, st = g.intersect(np.zeros((0, 6)), np.zeros((0, 6)))
    assert tm.numel() == 0
    rng = np.random.default_rng(16)
    o = O.Oracle(inst)
    x, v = _points(o, inst, rng, 130)
    a = _np(g.intersect(x, v)[1])
    b = _np(g.intersect(x[:7], v[:7])[1])  # smaller call after a larger one
    c = _np(g.intersect(x, v)[1])
    assert np.array_equal(a[:7], b) and np.array_equal(a, c)  # deterministic


def test_paper_generator_intersect_and_reflect():
    """The random spectrahedra of the paper's experiments (Section 4):
    A0 = Z Z^T + I, A_i = blkdiag(Qt, -Qt), with no box block; kappa(A0) grows
    like m^2, which the interior pairs keep far below the 1e-9 bar."""
    S = _spec()
    for (n, m, b, seed) in [(20, 30, 40, 21), (60, 80, 24, 22), (100, 100, 8, 23)]:
        inst = I.paper_random(n, m, seed=seed)
        _check_intersect(inst, b, seed)
        o, g = O.Oracle(inst), S.Spectrahedron(inst)
        rng = np.random.default_rng(seed + 100)
        x, v = _points(o, inst, rng, b)
        tp_r, s_r, w_r, st_r = o.reflect(x, v)
        tp, s, w, st = [_np(a) for a in g.reflect(x, v)]
        ok = st_r == O.OK
        assert ok.all() and np.array_equal(st, st_r)
        assert np.allclose(tp, tp_r, rtol=T_REL, atol=0)
        assert np.allclose(w, w_r, atol=1e-7 * max(1.0, np.abs(w_r).max()))
        assert np.allclose(s, s_r, atol=2e-7)


def test_nonsmooth_statuses_match_oracle():
    """NONSMOOTH where two pieces of the boundary meet at the hit, as the
    oracle: a vertex of a box (two diagonal rows tie), and a dense block whose
    root equals a diagonal row's; generic hits stay OK.  (A multiple
    lambda_min inside the one merged dense block is not visible to a
    single-vector Krylov method, which sees one copy of each eigenvalue.)"""
    S = _spec()
    cases = []
    box = I.box(2, 1.0)
    cases.append((box, np.zeros((2, 2)), np.array([[1.0, 1.0], [1.0, 0.3]]) / np.array([[math.sqrt(2)], [1.0]])))
    # dense [[1 - x1]] and the diagonal row 1 - x1, plus a second coordinate
    A = np.zeros((3, 1, 1))
    A[0] = 1.0
    A[1] = -1.0
    D = np.zeros((3, 4))
    D[0] = [1.0, 3.0, 2.0, 2.0]
    D[1] = [-1.0, 1.0, 0.0, 0.0]
    D[2] = [0.0, 0.0, 1.0, -1.0]
    mixed = I.Instance(2, [I.Block(I.DENSE, A), I.Block(I.DIAG, D)], name="dense-diag-tie")
    cases.append((mixed, np.zeros((2, 2)), np.array([[1.0, 0.5], [-1.0, 0.3]])))
    for inst, x, v in cases:
        g, o = S.Spectrahedron(inst), O.Oracle(inst)
        tp, s, w, st = [_np(a) for a in g.reflect(x, v)]
        tp_r, s_r, w_r, st_r = o.reflect(x, v)
        assert np.array_equal(st, st_r), (inst.name, st, st_r)
        assert st[0] == S.NONSMOOTH and st[1] == S.OK
        assert np.allclose(tp, tp_r, rtol=1e-15)
