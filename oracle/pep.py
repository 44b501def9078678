"""First roots of det F(Phi(t)) along a polynomial curve of any degree d
(the paper's polynomial eigenvalue problem, eq. (PEP), solved by its
companion linearisation), and the plain definition by bisection on
membership.  Test infrastructure, like the rest of oracle/.

The curve is Phi(t) = sum_k t^k c_k with coefficient rows coef[k] =
(c_k0, c_k1 .. c_kn): the A0 weight and the coordinates (c_00 = 1 for the
start point, 0 for the other rows).  For every block, F(Phi(t)) is the matrix
polynomial P(t) = sum_k t^k B_k, B_k = c_k0 A0 + sum_i c_ki A_i, with
P(0) = F(p) > 0; its first positive root is where the curve leaves S.

Companion linearisation (the paper's PEP section): the roots of det P are
the eigenvalues of the pencil C0 - lambda C1 of size d m with
C0 = blkdiag(B_d, I, .., I) and C1 the block companion matrix with first
block row (B_{d-1}, .., B_0) and -I on the block subdiagonal; a singular B_d
adds infinite eigenvalues, which do not count.  The real positive ones are
candidates; the first is the smallest (among candidates a nearby complex pair
at the rounding level of a double real root is taken as real)."""
import numpy as np
import scipy.linalg


def _block_polys(inst, coef):
    """Per block: (kind, list of B_k)."""
    coef = np.asarray(coef, dtype=np.float64)
    out = []
    for b in inst.blocks:
        A = np.asarray(b.A, dtype=np.float64)
        Bs = [np.tensordot(coef[k], A, 1) for k in range(coef.shape[0])]
        out.append((b.kind, Bs))
    return out


def _companion_roots(Bs):
    """All finite eigenvalues of the companion pencil of sum_k t^k B_k."""
    d = len(Bs) - 1
    m = Bs[0].shape[0]
    if d == 1:  # B_0 x = -t B_1 x
        w = scipy.linalg.eigvals(-Bs[0], Bs[1])
        return w[np.isfinite(w)]
    C0 = np.eye(d * m)
    C0[:m, :m] = Bs[d]
    C1 = np.zeros((d * m, d * m))
    for j in range(d):
        C1[:m, j * m:(j + 1) * m] = -Bs[d - 1 - j]
    for j in range(1, d):
        C1[j * m:(j + 1) * m, (j - 1) * m:j * m] = np.eye(m)
    # C1 z = lambda C0 z  <=>  P(lambda) x = 0 with z = (lambda^{d-1} x, .., lambda x, x):
    # the first block row is lambda B_d lambda^{d-1} x = -sum_{k<d} B_k lambda^k x,
    # the others lambda (lambda^{d-1-j} x) = lambda^{d-j} x
    w = scipy.linalg.eigvals(C1, C0)
    return w[np.isfinite(w)]


def _first_positive(roots, horizon, scale):
    best = np.inf
    for r in roots:
        if abs(r.imag) <= 1e-7 * max(abs(r.real), scale) and r.real > 0 and r.real <= horizon:
            best = min(best, r.real)
    return best


def first_roots_companion(inst, coef, horizon=np.inf):
    """(t-, t+): the first roots of det F(Phi(t)) on both sides of 0, by the
    companion linearisation of every block (+-inf when none within the
    horizon)."""
    coef = np.asarray(coef, dtype=np.float64)
    d = coef.shape[0] - 1
    flip = np.array([(-1.0) ** k for k in range(d + 1)])[:, None]
    res = []
    for c in (coef, coef * flip):
        best = np.inf
        for kind, Bs in _block_polys(inst, c):
            if kind == 0:
                roots = _companion_roots(Bs)
                best = min(best, _first_positive(roots, horizon, 1e-300))
            else:
                for j in range(Bs[0].shape[0]):
                    p = [B[j] for B in Bs]  # ascending
                    while len(p) > 1 and p[-1] == 0.0:
                        p = p[:-1]
                    if len(p) == 1:
                        continue
                    roots = np.roots(p[::-1])
                    best = min(best, _first_positive(roots, horizon, 1e-300))
        res.append(best)
    return -res[1], res[0]


def _member(inst, coef, t):
    y = sum((t ** k) * np.asarray(coef[k]) for k in range(len(coef)))
    for b in inst.blocks:
        A = np.asarray(b.A, dtype=np.float64)
        F = np.tensordot(y, A, 1)
        if b.kind == 0:
            try:
                np.linalg.cholesky(F)
            except np.linalg.LinAlgError:
                return False
        elif not np.all(F > 0.0):
            return False
    return True


def first_root_bisect(inst, coef, horizon, grid=4000):
    """The plain definition: sup{t > 0 : F(Phi(s)) > 0 for all s in [0, t)},
    by the first grid point of [0, horizon] where membership fails, then
    bisection between it and the grid point before (to adjacent doubles).
    +inf when every grid point is inside.  A root pair closer than one grid
    step can be missed, so the grid is fine and the pins use it on curves
    whose roots are well separated."""
    coef = np.asarray(coef, dtype=np.float64)
    ts = np.linspace(0.0, horizon, grid + 1)
    prev = 0.0
    for t in ts[1:]:
        if not _member(inst, coef, t):
            lo, hi = prev, t
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                if mid <= lo or mid >= hi:
                    break
                if _member(inst, coef, mid):
                    lo = mid
                else:
                    hi = mid
            return hi
        prev = t
    return np.inf
