"""Pins of the FP64 CPU oracle against facts fixed outside the oracle itself:
closed forms, library routines on special cases, brute force on tiny inputs,
the paper's worked example, invariants.  CPU only."""
import json
import math
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.linalg
import scipy.stats

from oracle import oracle as O
from paper_2010_03817_amd import instances as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense_F(inst, x):
    D = inst.dense_matrix()
    return D[0] + np.tensordot(x, D[1:], axes=(0, 0))


def dense_B(inst, v):
    D = inst.dense_matrix()
    return np.tensordot(v, D[1:], axes=(0, 0))


def scipy_tpm(inst, x, v):
    """t+- from the generalized symmetric eigenproblem B y = mu F y (LAPACK)."""
    mu = scipy.linalg.eigh(dense_B(inst, v), dense_F(inst, x), eigvals_only=True)
    tp = -1.0 / mu.min() if mu.min() < 0 else np.inf
    tm = -1.0 / mu.max() if mu.max() > 0 else -np.inf
    return tm, tp


def is_pd(M):
    try:
        np.linalg.cholesky(M)
        return True
    except np.linalg.LinAlgError:
        return False


def bisect_boundary(inst, x, v, sign=1.0, iters=200):
    """Largest t with F(x + s t v) > 0 on [0, t], by halving with LAPACK Cholesky."""
    lo, hi = 0.0, 1.0
    while is_pd(dense_F(inst, x + sign * hi * v)):
        lo, hi = hi, 2 * hi
        if hi > 1e8:
            return np.inf
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        if is_pd(dense_F(inst, x + sign * mid * v)):
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


# ---------------------------------------------------------------- RNG


def _rocrand_philox(ctrs, seed):
    """Philox4x32-10 blocks from rocRAND's host-callable engine (a library
    implementation independent of the oracle)."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    src = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
#include <cstdlib>
int main(int argc, char** argv) {
  unsigned long long seed = strtoull(argv[1], 0, 10);
  for (int a = 2; a + 3 < argc; a += 4) {
    unsigned x = strtoul(argv[a],0,10), y = strtoul(argv[a+1],0,10);
    unsigned z = strtoul(argv[a+2],0,10), w = strtoul(argv[a+3],0,10);
    unsigned long long sub = (unsigned long long)z | ((unsigned long long)w << 32);
    unsigned long long off = 4ull * ((unsigned long long)x | ((unsigned long long)y << 32));
    rocrand_device::philox4x32_10_engine e(seed, sub, off);
    unsigned r0 = e(), r1 = e(), r2 = e(), r3 = e();
    printf("%u %u %u %u\n", r0, r1, r2, r3);
  }
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        cpp = os.path.join(d, "p.cpp")
        exe = os.path.join(d, "p")
        open(cpp, "w").write(src)
        subprocess.check_call([hipcc, "-O1", cpp, "-o", exe, "-w"],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        args = [exe, str(seed)] + [str(c) for ctr in ctrs for c in ctr]
        out = subprocess.check_output(args).decode().split("\n")
    return [[int(t) for t in line.split()] for line in out if line.strip()]


@pytest.mark.slow
def test_philox_matches_rocrand():
    rng = np.random.default_rng(5)
    ctrs = [[0, 0, 0, 0], [1, 0, 0, 0], [7, 3, 2, 1], [0xFFFFFFFF, 5, 9, 0x80000000]]
    # rocRAND reaches a counter through a 64-bit offset of 4 * (x + 2^32 y),
    # so keep y below 2^30 to stay inside that range
    ctrs += [[int(rng.integers(0, 2**32)), int(rng.integers(0, 2**30)), int(rng.integers(0, 2**32)),
              int(rng.integers(0, 2**32))] for _ in range(12)]
    for seed in (0, 12345, 0xDEADBEEFCAFE1234):
        ref = _rocrand_philox(ctrs, seed)
        mine = [O.philox(c, [seed & 0xFFFFFFFF, seed >> 32]) for c in ctrs]
        assert mine == ref


# ---------------------------------------------------------------- lines


def test_polytope_ratio_test():
    """A diagonal LMI is a polytope {Ax <= b}; t+ is the min positive ratio."""
    rng = np.random.default_rng(1)
    n, rows = 6, 17
    A = rng.standard_normal((rows, n))
    b = rng.uniform(0.5, 2.0, rows)
    inst = I.polytope(A, b)
    o = O.Oracle(inst)
    x = rng.standard_normal((50, n)) * 0.05
    v = rng.standard_normal((50, n))
    tm, tp, st = o.intersect(x, v)
    assert (st == O.OK).all()
    for k in range(50):
        slack = b - A @ x[k]
        rate = A @ v[k]
        ratios = slack / rate
        assert tp[k] == pytest.approx(ratios[rate > 0].min(), rel=1e-14)
        assert tm[k] == pytest.approx(ratios[rate < 0].max(), rel=1e-14)
    # reflection is the specular reflection at the facet attaining t+
    tp2, s, w, st = o.reflect(x, v)
    for k in range(50):
        j = np.argmin(np.where(A @ v[k] > 0, (b - A @ x[k]) / (A @ v[k]), np.inf))
        nrm = A[j] / np.linalg.norm(A[j])
        assert np.allclose(w[k], nrm, atol=1e-14)
        assert np.allclose(s[k], v[k] - 2 * (v[k] @ nrm) * nrm, atol=1e-13)


def test_dense_and_diag_blocks_agree():
    n = 4
    d, D = I.box(n, 1.5), I.box_as_dense(n, 1.5)
    od, oD = O.Oracle(d), O.Oracle(D)
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, (40, n))
    v = I.random_directions(rng, 40, n)
    a, b = od.reflect(x, v), oD.reflect(x, v)
    assert np.allclose(a[0], b[0], rtol=1e-12)
    assert np.allclose(a[1], b[1], atol=1e-10)
    assert np.allclose(a[2], b[2], atol=1e-10)
    assert np.allclose(od.intersect(x, v)[0], oD.intersect(x, v)[0], rtol=1e-12)


def test_ball_quadratic_roots_and_normal():
    n = 7
    o = O.Oracle(I.arrow_ball(n))
    rng = np.random.default_rng(3)
    x = rng.standard_normal((60, n))
    x *= (rng.uniform(0, 0.999, 60) / np.linalg.norm(x, axis=1))[:, None]
    v = rng.standard_normal((60, n))
    tm, tp, st = o.intersect(x, v)
    a = (v * v).sum(1)
    bq = 2 * (x * v).sum(1)
    c = (x * x).sum(1) - 1.0
    q = -0.5 * (bq + np.sign(bq) * np.sqrt(bq * bq - 4 * a * c))
    r1, r2 = q / a, c / q
    assert np.allclose(tp, np.maximum(r1, r2), rtol=1e-12)
    assert np.allclose(tm, np.minimum(r1, r2), rtol=1e-12)
    tp2, s, w, st = o.reflect(x, v)
    hit = x + tp2[:, None] * v
    assert np.allclose(w, hit / np.linalg.norm(hit, axis=1, keepdims=True), atol=1e-9)


def test_bisection_tiny_instances():
    """t+- against bisection with an independent (LAPACK) membership test."""
    insts = [I.gbase(3, m, seed=10 + m, box=False) for m in (2, 4, 5, 8)] + [I.paper_example_2d()]
    rng = np.random.default_rng(4)
    for inst in insts:
        o = O.Oracle(inst)
        for _ in range(4):
            v = I.random_directions(rng, 1, inst.n)[0]
            d = I.random_directions(rng, 1, inst.n)[0]
            x = 0.3 * d * o.intersect(np.zeros(inst.n), d)[1][0]
            if inst.name.startswith("paper"):
                x = np.array([-1.0, 1.0]) + 0.1 * rng.standard_normal(2)
            tm, tp, st = o.intersect(x, v)
            assert st[0] == O.OK
            assert tp[0] == pytest.approx(bisect_boundary(inst, x, v), rel=1e-12)
            assert -tm[0] == pytest.approx(bisect_boundary(inst, x, v, -1.0), rel=1e-12)


def test_paper_generator_structure_and_bisection():
    """The random spectrahedra of the paper's experiments (Section 4):
    A0 = Z Z^T + I is positive definite (the origin is interior), each A_i is
    blkdiag(Qt, -Qt) with Qt symmetric, so B(v) has trace zero and eigenvalues
    of both signs and every line leaves S on both sides (t+- finite).  The
    oracle's t+- agree with bisection on LAPACK membership."""
    rng = np.random.default_rng(8)
    for n, m in [(3, 4), (5, 6), (8, 10)]:
        inst = I.paper_random(n, m, seed=40 + m)
        A = inst.blocks[0].A
        h = m // 2
        assert np.linalg.eigvalsh(A[0]).min() >= 1.0 - 1e-12
        for i in range(1, n + 1):
            assert np.array_equal(A[i], A[i].T)
            assert np.array_equal(A[i][h:, h:], -A[i][:h, :h])
            assert not A[i][:h, h:].any()
        o = O.Oracle(inst)
        for _ in range(3):
            d = I.random_directions(rng, 1, n)[0]
            v = I.random_directions(rng, 1, n)[0]
            x = 0.4 * d * o.intersect(np.zeros(n), d)[1][0]
            tm, tp, st = o.intersect(x, v)
            assert st[0] == O.OK and np.isfinite(tm[0]) and np.isfinite(tp[0])
            assert tp[0] == pytest.approx(bisect_boundary(inst, x, v), rel=1e-12)
            assert -tm[0] == pytest.approx(bisect_boundary(inst, x, v, -1.0), rel=1e-12)


@pytest.mark.parametrize("m", [7, 30])
def test_generalized_eigen_special_case(m):
    inst = I.gbase(9, m, seed=m)
    o = O.Oracle(inst)
    rng = np.random.default_rng(m)
    v = I.random_directions(rng, 12, 9)
    d = I.random_directions(rng, 12, 9)
    frac = rng.uniform(0, 0.99, 12)
    x = (frac * o.intersect(np.zeros((12, 9)), d)[1])[:, None] * d
    tm, tp, st = o.intersect(x, v)
    for k in range(12):
        rtm, rtp = scipy_tpm(inst, x[k], v[k])
        assert tp[k] == pytest.approx(rtp, rel=1e-11)
        assert tm[k] == pytest.approx(rtm, rel=1e-11)


def test_paper_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "paper_example_2d.json")))
    inst = I.paper_example_2d()
    o = O.Oracle(inst)
    p0, u = np.array(g["p0"]), np.array(g["u"])
    tm, tp, st = o.intersect(p0, u)
    tp2, s, w, st2 = o.reflect(p0, u)
    # exact for the rounded matrices: LAPACK generalized eigenproblem
    rtm, rtp = scipy_tpm(inst, p0, u)
    assert tp[0] == pytest.approx(rtp, rel=1e-13) and tm[0] == pytest.approx(rtm, rel=1e-13)
    # the printed values (from unrounded matrices) lie in the envelope the
    # one-decimal rounding allows: redraw every entry within +-0.05
    rng = np.random.default_rng(0)
    D = inst.dense_matrix()
    env = []
    for _ in range(3000):
        E0 = rng.uniform(-0.05, 0.05, (6, 6))
        A0 = D[0] + np.triu(E0) + np.triu(E0, 1).T
        As = []
        for i in (1, 2):
            Eq = rng.uniform(-0.05, 0.05, (3, 3))
            Q = D[i, :3, :3] + np.triu(Eq) + np.triu(Eq, 1).T
            As.append(scipy.linalg.block_diag(Q, -Q))
        Bm = u[0] * As[0] + u[1] * As[1]
        F = A0 + p0[0] * As[0] + p0[1] * As[1]
        mu, Y = scipy.linalg.eigh(Bm, F)
        y = Y[:, 0]
        wv = np.array([y @ As[0] @ y, y @ As[1] @ y])
        wv /= np.linalg.norm(wv)
        env.append([-1 / mu[-1], -1 / mu[0], *wv, *(u - 2 * (u @ wv) * wv)])
    env = np.array(env)
    lo, hi = env.min(0), env.max(0)
    printed = [g["t_minus_printed"], g["t_plus_printed"]]
    assert lo[0] <= printed[0] <= hi[0] and lo[1] <= printed[1] <= hi[1]
    wp = np.array(g["w_printed"]) / np.linalg.norm(g["w_printed"])
    # orientation of w is arbitrary in the paper; the oracle orients it outward
    assert (lo[2] <= -wp[0] <= hi[2]) or (lo[2] <= wp[0] <= hi[2])
    up = np.array(g["u_reflected_printed"])
    assert lo[4] - 0.05 <= up[0] <= hi[4] + 0.05 and lo[5] - 0.05 <= up[1] <= hi[5] + 0.05
    # and the oracle's own values are inside it too
    assert lo[0] <= tm[0] <= hi[0] and lo[1] <= tp[0] <= hi[1]
    assert np.allclose(s[0], u - 2 * (u @ w[0]) * w[0])
    # the literal printed +Q lower blocks would give a far-off t+
    A_lit = D.copy()
    A_lit[1:, 3:, 3:] = A_lit[1:, :3, :3]
    lit = I.Instance(2, [I.Block(I.DENSE, A_lit)])
    assert O.Oracle(lit).intersect(p0, u)[1][0] > 1.0


# ---------------------------------------------------------------- invariants


def test_congruence_and_scaling_invariance():
    inst = I.gbase(6, 9, seed=21)
    o = O.Oracle(inst)
    oc = O.Oracle(I.congruent(inst, 3))
    scaled = I.Instance(inst.n, [I.Block(b.kind, 3.7 * b.A) for b in inst.blocks])
    os_ = O.Oracle(scaled)
    rng = np.random.default_rng(22)
    v = I.random_directions(rng, 20, 6)
    d = I.random_directions(rng, 20, 6)
    x = 0.5 * (o.intersect(np.zeros((20, 6)), d)[1])[:, None] * d
    a, b, c = o.reflect(x, v), oc.reflect(x, v), os_.reflect(x, v)
    for r in (b, c):
        assert np.allclose(a[0], r[0], rtol=1e-11)
        assert np.allclose(a[1], r[1], atol=1e-9)
        assert np.allclose(a[2], r[2], atol=1e-9)


def test_block_diagonal_is_min_over_blocks():
    g1, g2 = I.gbase(5, 6, seed=1, box=False), I.gbase(5, 8, seed=2, box=False)
    both = I.Instance(5, g1.blocks + g2.blocks)
    rng = np.random.default_rng(23)
    x = np.zeros((30, 5))
    v = I.random_directions(rng, 30, 5)
    r1, r2, rb = O.Oracle(g1).intersect(x, v), O.Oracle(g2).intersect(x, v), O.Oracle(both).intersect(x, v)
    assert np.array_equal(rb[1], np.minimum(r1[1], r2[1]))
    assert np.array_equal(rb[0], np.maximum(r1[0], r2[0]))


def test_reflection_identities():
    inst = I.gbase(8, 12, seed=5)
    o = O.Oracle(inst)
    rng = np.random.default_rng(24)
    v = I.random_directions(rng, 25, 8)
    x = np.zeros((25, 8))
    tp, s, w, st = o.reflect(x, v)
    assert np.allclose(np.linalg.norm(s, axis=1), 1.0, atol=1e-14)
    assert np.allclose((s * w).sum(1), -(v * w).sum(1), atol=1e-14)
    assert ((v * w).sum(1) > 0).all()  # outward orientation


def test_normal_is_gradient_of_lambda_min():
    """Hellmann-Feynman: grad of lambda_min(F(x)) at the hit point is
    (u^T A_i u), checked by central differences with LAPACK eigvalsh."""
    inst = I.gbase(5, 7, seed=8, box=False)
    o = O.Oracle(inst)
    rng = np.random.default_rng(25)
    for _ in range(5):
        v = I.random_directions(rng, 1, 5)[0]
        tp, s, w, st = o.reflect(np.zeros(5), v)
        hit = tp[0] * v
        h = 1e-6
        g = np.array([(np.linalg.eigvalsh(dense_F(inst, hit + h * e))[0]
                       - np.linalg.eigvalsh(dense_F(inst, hit - h * e))[0]) / (2 * h) for e in np.eye(5)])
        g /= np.linalg.norm(g)
        assert np.allclose(w[0], -g, atol=1e-6)  # lambda_min grows inward; w points outward


def test_log_det_gradient_jacobi_formula():
    """Appendix A: d det F / dx_k = Tr(adj(F) A_k); for the normal at a rank
    m-1 point this is a positive multiple of u^T A_k u.  Check the direction
    by differentiating det F along the boundary normal numerically."""
    inst = I.gbase(4, 5, seed=9, box=False)
    o = O.Oracle(inst)
    v = np.array([0.3, -0.5, 0.7, 0.2])
    v /= np.linalg.norm(v)
    tp, s, w, st = o.reflect(np.zeros(4), v)
    hit = tp[0] * v
    h = 1e-7
    g = np.array([(np.linalg.det(dense_F(inst, hit + h * e)) - np.linalg.det(dense_F(inst, hit - h * e))) / (2 * h)
                  for e in np.eye(4)])
    g /= np.linalg.norm(g)
    assert np.allclose(np.abs(g @ w[0]), 1.0, atol=1e-6)


def test_membership_elliptope_closed_form():
    o = O.Oracle(I.elliptope3())
    rng = np.random.default_rng(26)
    x = rng.uniform(-1, 1, (4000, 3))
    x1, x2, x3 = x.T
    det = 1 - x1**2 - x2**2 - x3**2 + 2 * x1 * x2 * x3
    inside = det > 0  # unit diagonal and |x_i| < 1: PD iff det > 0
    got = o.membership(x)
    margin = np.abs(det) > 1e-12
    assert np.array_equal(got[margin], inside[margin])
    # volume of the elliptope is pi^2/2: the hit fraction of the cube [-1,1]^3
    frac = inside.mean()
    assert abs(8 * frac - math.pi**2 / 2) < 4 * 8 * math.sqrt(frac * (1 - frac) / 4000)


def test_status_not_interior_and_unbounded():
    inst = I.gbase(4, 6, seed=3)
    o = O.Oracle(inst)
    x = np.full((1, 4), 50.0)  # outside the box block
    tm, tp, st = o.intersect(x, np.ones((1, 4)))
    assert st[0] == O.NOT_INTERIOR and np.isnan(tp[0]) and np.isnan(tm[0])
    # a half-space is unbounded along directions inside it
    hs = I.polytope(np.array([[1.0, 0.0]]), np.array([1.0]))
    oh = O.Oracle(hs)
    tm, tp, st = oh.intersect(np.zeros((1, 2)), np.array([[0.0, 1.0]]))
    assert st[0] == O.UNBOUNDED and tp[0] == np.inf and tm[0] == -np.inf
    tm, tp, st = oh.intersect(np.zeros((1, 2)), np.array([[1.0, 0.0]]))
    assert st[0] == O.UNBOUNDED and tp[0] == pytest.approx(1.0) and tm[0] == -np.inf


# ---------------------------------------------------------------- degree two


def test_curve2_degree_one_equals_line():
    inst = I.gbase(5, 8, seed=31)
    o = O.Oracle(inst)
    rng = np.random.default_rng(31)
    x = np.zeros((10, 5))
    v = I.random_directions(rng, 10, 5)
    coef = np.zeros((10, 3, 6))
    coef[:, 0, 0] = 1.0
    coef[:, 0, 1:] = x
    coef[:, 1, 1:] = v
    tm2, tp2, st2, it = o.intersect_curve2(coef)
    tm, tp, st = o.intersect(x, v)
    assert np.allclose(tp2, tp, rtol=1e-13) and np.allclose(tm2, tm, rtol=1e-13)


def test_curve2_against_grid_scan():
    """First root of det Q(t) for a degree-2 curve, by a fine scan of
    lambda_min(Q(t)) (LAPACK) and bisection, including curves that leave and
    re-enter the set."""
    rng = np.random.default_rng(32)
    for trial in range(6):
        inst = I.gbase(3, 5, seed=40 + trial, box=False)
        o = O.Oracle(inst)
        p = np.zeros(3)
        v = rng.standard_normal(3)
        a = 3.0 * rng.standard_normal(3)
        coef = np.zeros((1, 3, 4))
        coef[0, 0, 0] = 1.0
        coef[0, 1, 1:] = v
        coef[0, 2, 1:] = a
        tm, tp, st, it = o.intersect_curve2(coef)

        def lam(t):
            return np.linalg.eigvalsh(dense_F(inst, p + t * v + t * t * a))[0]

        ts = np.linspace(0, 5, 20001)
        vals = np.array([lam(t) for t in ts])
        neg = np.nonzero(vals <= 0)[0]
        if len(neg) == 0:
            assert tp[0] == np.inf or tp[0] > 5
            continue
        lo, hi = ts[neg[0] - 1], ts[neg[0]]
        for _ in range(100):
            mid = 0.5 * (lo + hi)
            if lam(mid) > 0:
                lo = mid
            else:
                hi = mid
        assert tp[0] == pytest.approx(lo, rel=1e-9)


def test_curve2_ellipse_on_ball_closed_form():
    """Exact Gaussian HMC trajectory Phi(theta) = p cos + sigma v sin on the
    unit ball; with u = tan(theta/2), coefficient rows [1,p],[0,2 sigma v],[2,-p].
    |Phi|^2 = 1 is R cos(2 theta - phi) = 1 - (|p|^2 + sigma^2 |v|^2)/2."""
    n = 6
    o = O.Oracle(I.arrow_ball(n))
    rng = np.random.default_rng(33)
    for _ in range(10):
        p = rng.standard_normal(n)
        p *= rng.uniform(0.1, 0.9) / np.linalg.norm(p)
        v = rng.standard_normal(n)
        sigma = 0.7
        coef = np.zeros((1, 3, n + 1))
        coef[0, 0, 0] = 1.0
        coef[0, 0, 1:] = p
        coef[0, 1, 1:] = 2 * sigma * v
        coef[0, 2, 0] = 1.0
        coef[0, 2, 1:] = -p
        tm, tp, st, it = o.intersect_curve2(coef, horizon=1.0)
        # closed form: |Phi|^2 = A + Bc cos 2th + Bs sin 2th
        P2, V2, PV = p @ p, sigma**2 * (v @ v), sigma * (p @ v)
        A = 0.5 * (P2 + V2)
        Bc, Bs = 0.5 * (P2 - V2), PV
        R, phi = math.hypot(Bc, Bs), math.atan2(Bs, Bc)
        if R < 1e-12 or abs((1 - A) / R) > 1:
            assert tp[0] == np.inf
            continue
        base = math.acos((1 - A) / R)
        cands = sorted(((phi + sgn * base) / 2) % math.pi for sgn in (1, -1))
        cands = [c for c in cands if c > 1e-12]
        th = cands[0]
        if th > math.pi / 2:
            assert tp[0] == np.inf
        else:
            assert tp[0] == pytest.approx(math.tan(th / 2), rel=1e-10)


# ---------------------------------------------------------------- MLP


def test_mlp_gelu_value_and_fd_gradients():
    dims = [5, 7, 6, 2]
    npar = O.mlp_nparams(dims)
    assert npar == 5 * 7 + 7 + 7 * 6 + 6 + 6 * 2 + 2
    # GELU(1) = Phi(1) = 0.8413447460685429 (standard normal table)
    P1 = np.array([1.0, 0.0, 1.0, 0.0])
    y = O.mlp_forward([1, 1, 1], P1, np.array([[1.0]]))
    assert y[0, 0] == pytest.approx(0.8413447460685429, rel=1e-15)
    rng = np.random.default_rng(41)
    P = rng.standard_normal(npar) * 0.5
    X = rng.standard_normal((9, 5))
    T = rng.standard_normal((9, 2))
    loss, G = O.mlp_loss_grad(dims, P, X, T)
    h = 1e-6
    for k in rng.choice(npar, 40, replace=False):
        e = np.zeros(npar)
        e[k] = h
        fd = (O.mlp_loss_grad(dims, P + e, X, T)[0] - O.mlp_loss_grad(dims, P - e, X, T)[0]) / (2 * h)
        assert G[k] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_adam_first_step_closed_form():
    g = np.array([0.3, -2.0, 1e-3])
    p = np.zeros(3)
    m = np.zeros(3)
    v = np.zeros(3)
    O.adam_step(p, g.copy(), m, v, 1, lr=0.01, eps=0.0)
    assert np.allclose(p, -0.01 * np.sign(g), rtol=1e-12)


# ---------------------------------------------------------------- walks


def test_hnr_uniform_on_box_marginals():
    n = 3
    o = O.Oracle(I.box(n, 1.0))
    x0 = np.zeros((64, n))
    xo, samples, stats = o.walk(O.HNR, x0, 400, seed=7, thin=20)
    pts = samples[:, 5:].reshape(-1, n)
    for i in range(n):
        assert scipy.stats.kstest((pts[:, i] + 1) / 2, "uniform").pvalue > 1e-3


def test_billiard_uniform_on_ball_moment():
    n = 5
    o = O.Oracle(I.arrow_ball(n))
    xo, samples, stats = o.walk(O.BILLIARD, np.zeros((64, n)), 300, seed=8, tau=2.0, thin=10)
    r2 = (samples[:, 3:] ** 2).sum(-1).ravel()
    se = r2.std() / math.sqrt(len(r2) / 4)  # thinned chain, conservative
    assert abs(r2.mean() - n / (n + 2)) < 4 * se
    assert stats[1] > 0 and stats[2] <= 1e-3 * stats[5]  # reflection cap rarely reached


def test_chnr_uniform_on_box():
    n = 4
    o = O.Oracle(I.box(n, 2.0))
    xo, samples, stats = o.walk(O.CHNR, np.zeros((32, n)), 800, seed=9, thin=20)
    pts = samples[:, 5:].reshape(-1, n)
    for i in range(n):
        assert scipy.stats.kstest((pts[:, i] + 2) / 4, "uniform").pvalue > 1e-3


def _trunc_gauss_r2(n, sigma):
    c = 1 / sigma**2
    return n * sigma**2 * scipy.stats.chi2.cdf(c, n + 2) / scipy.stats.chi2.cdf(c, n)


def test_gaussian_hnr_and_hmc_on_ball_moment():
    n, sigma = 4, 0.6
    o = O.Oracle(I.arrow_ball(n))
    a = 1 / (2 * sigma**2)
    want = _trunc_gauss_r2(n, sigma)
    xo, s1, _ = o.walk(O.HNR, np.zeros((64, n)), 400, seed=10, gauss_a=a, thin=10)
    xo, s2, st2 = o.walk(O.HMC, np.zeros((64, n)), 200, seed=11, gauss_a=a, tau=1.0, thin=5)
    for s in (s1, s2):
        r2 = (s[:, 4:] ** 2).sum(-1).ravel()
        se = r2.std() / math.sqrt(len(r2) / 4)
        assert abs(r2.mean() - want) < 4 * se


# ---------------------------------------------------------------- volume


@pytest.mark.slow
@pytest.mark.parametrize("which", ["ball", "box", "simplex"])
def test_volume_known_bodies(which):
    if which == "ball":
        n = 6
        inst = I.arrow_ball(n)
        truth = (n / 2) * math.log(math.pi) - math.lgamma(n / 2 + 1)
        dh = 2.0
    elif which == "box":
        n = 5
        inst = I.box(n, 1.0)
        truth = n * math.log(2.0)
        dh = 2 * math.sqrt(n)
    else:
        n = 4
        inst = I.simplex(n)
        truth = -math.lgamma(n + 1)
        dh = math.sqrt(2)
    o = O.Oracle(inst)
    a0 = 4.0 * n
    lv, lo, hi, lr = o.volume(phases=20, samples_per_phase=1600, chains=32, walk_len=3, seed=13, a0=a0,
                              a_end=1.0 / (4 * dh * dh), groups=8)
    width = hi - lo
    assert lo - 0.5 * width <= truth <= hi + 0.5 * width, (lv, lo, hi, truth)
