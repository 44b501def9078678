"""Reference optimum of the semidefinite program min <c, x> subject to
F(x) = blkdiag_b(A_b0 + sum_i x_i A_bi) >= 0 (the paper's optimisation
section, eq. (sdp)), by a primal log-barrier path-following method.

Test infrastructure, like the rest of oracle/: only tests, the smoke check
and the benchmark's CPU baseline use it (and the script that writes the
stored optima).  It shares nothing with the device path.

The central path x(t) = argmin t <c, x> - log det F(x) is followed by damped
Newton steps (gradient t c_i - tr(F^-1 A_i), Hessian tr(F^-1 A_i F^-1 A_j);
for diagonal blocks the same with scalars); on the central path
<c, x(t)> - min <c, x> <= M / t with M the total size of the blocks (the
barrier's parameter), so t grows by 10 until M / t is below the requested
gap.  S must be bounded with x0 interior."""
import numpy as np


def _blocks(inst):
    return [(b.kind, np.asarray(b.A, dtype=np.float64)) for b in inst.blocks]


def _F(blocks, x):
    return [A[0] + np.tensordot(x, A[1:], 1) for _, A in blocks]


def _definite(blocks, Fs):
    for (kind, _), F in zip(blocks, Fs):
        if kind == 0:
            try:
                np.linalg.cholesky(F)
            except np.linalg.LinAlgError:
                return False
        elif not np.all(F > 0.0):
            return False
    return True


def _barrier(blocks, Fs):
    v = 0.0
    for (kind, _), F in zip(blocks, Fs):
        if kind == 0:
            v -= 2.0 * np.sum(np.log(np.diag(np.linalg.cholesky(F))))
        else:
            v -= np.sum(np.log(F))
    return v


def _grad_hess(blocks, Fs, n):
    g = np.zeros(n)
    H = np.zeros((n, n))
    for (kind, A), F in zip(blocks, Fs):
        Ai = A[1:]
        if kind == 0:
            # with F = L L^T and K_i = L^-1 A_i L^-T: tr(F^-1 A_i) = tr(K_i) and
            # tr(F^-1 A_i F^-1 A_j) = <K_i, K_j> (Frobenius)
            Li = np.linalg.inv(np.linalg.cholesky(F))
            K = np.matmul(np.matmul(Li, Ai), Li.T).reshape(n, -1)
            m = F.shape[0]
            g -= K[:, :: m + 1].sum(axis=1)
            H += K @ K.T
        else:
            w = 1.0 / F
            g -= Ai @ w
            H += (Ai * w**2) @ Ai.T
    return g, H


def sdp_min(inst, c, x0=None, gap=1e-10, max_newton=200):
    """(x*, <c, x*>, barrier parameter t) with <c, x*> within gap * max(1, |f*|)
    of the optimum."""
    blocks = _blocks(inst)
    n = inst.n
    c = np.asarray(c, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    if not _definite(blocks, _F(blocks, x)):
        raise ValueError("x0 is not interior")
    M = sum(A.shape[1] for _, A in blocks)
    t = 1.0
    for _ in range(60):
        for _ in range(max_newton):
            Fs = _F(blocks, x)
            gb, H = _grad_hess(blocks, Fs, n)
            g = t * c + gb
            dx = -np.linalg.solve(H, g)
            dec = -g @ dx  # squared Newton decrement
            if dec / 2.0 <= 1e-12:
                break
            f0 = t * (c @ x) + _barrier(blocks, Fs)
            a = 1.0
            while True:
                xn = x + a * dx
                Fn = _F(blocks, xn)
                if _definite(blocks, Fn) and t * (c @ xn) + _barrier(blocks, Fn) <= f0 - 0.25 * a * dec:
                    break
                a *= 0.5
                if a < 1e-20:
                    break
            x = xn
        f = c @ x
        if M / t <= gap * max(1.0, abs(f)):
            return x, f, t
        t *= 10.0
    raise RuntimeError("barrier method did not reach the requested gap")
