"""Rounding bound of a boundary root that is NEAR its start point (test
helper, numpy only).

A root t* of det F(x + t v) whose unit kernel vector u spans the kernel of
F(x + t* v) moves, to first order, by u^T E u / (u^T B(v) u) when F(x) is
perturbed by E: the crossing eigenvalue changes by u^T E u and its slope in t
is u^T B u (Lemma "PEP and S cap C" with the first-order eigenvalue
perturbation).  Every method computes with a perturbed F(x): the assembly
A0 + sum_i x_i A_i is a sum of n + 1 products, off by at most
gamma_{n+1} M entrywise with M = |A0| + sum_i |x_i| |A_i|, and a Cholesky
factor L of it is exact for F + dF with |dF| <= gamma_{m+1} |L| |L|^T.  Two
correct methods therefore differ in t* by at most twice
(gamma_{n+1} |M|_2 + gamma_{m+1} | |L| |L|^T |_2) / |u^T B u|.

For the FAR root this bound is at the rounding level of t* itself; for the
root next to a start on the boundary (|t*| ~ 1e-6 t+) it is what F(x) fixes
the root to, whatever the method.  A diagonal row j crossing zero: the
assembly term alone, 2 gamma_{n+1} M_j / |B_j|.
"""
import numpy as np

EPS = 2.220446049250313e-16


def _gamma(k):
    return k * EPS / (1 - k * EPS)


def near_root_bound(inst, x, v, t):
    """Absolute bound on the difference of two correct evaluations of the
    boundary root t of the line x + t v (t from either side)."""
    n = inst.n
    best = None  # (|crossing eigenvalue| relative to the block scale, bound)
    for b in inst.blocks:
        A = b.A
        Fx = A[0] + np.tensordot(x, A[1:], 1)
        Bv = np.tensordot(v, A[1:], 1)
        M = np.abs(A[0]) + np.tensordot(np.abs(x), np.abs(A[1:]), 1)
        Ft = Fx + t * Bv
        if b.kind == 0:  # dense
            w, U = np.linalg.eigh(Ft)
            k = int(np.argmin(np.abs(w)))
            u = U[:, k]
            slope = abs(u @ Bv @ u)
            L = np.linalg.cholesky(Fx)
            chol = np.linalg.norm(np.abs(L) @ np.abs(L).T, 2)
            bound = 2 * (_gamma(n + 1) * np.linalg.norm(M, 2) + _gamma(b.m + 1) * chol) / max(slope, 1e-300)
            score = abs(w[k]) / max(np.abs(w).max(), 1e-300)
        else:  # diagonal rows
            k = int(np.argmin(np.abs(Ft) / np.maximum(np.abs(Fx), 1e-300)))
            bound = 2 * _gamma(n + 1) * M[k] / max(abs(Bv[k]), 1e-300)
            score = abs(Ft[k]) / max(abs(Fx[k]), 1e-300)
        if best is None or score < best[0]:
            best = (score, bound)
    return best[1]


def root_bars(inst, x, v, tm_r, tp_r, rel=1e-9):
    """Absolute bars for (t-, t+) of each pair: rel |t| for the far root and
    rel |t| + near_root_bound for the root nearer the start."""
    bar_m = rel * np.abs(tm_r)
    bar_p = rel * np.abs(tp_r)
    for k in range(len(x)):
        if np.abs(tm_r[k]) < np.abs(tp_r[k]):
            bar_m[k] += near_root_bound(inst, x[k], v[k], tm_r[k])
        else:
            bar_p[k] += near_root_bound(inst, x[k], v[k], tp_r[k])
    return bar_m, bar_p
