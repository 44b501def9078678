"""ctypes wrapper around the plain FP64 C oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by tests/, by __graft_entry__.smoke() and by
the CPU-baseline leg of bench.py.  The product path never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")

OK, EINVAL, ENOMEM, NOT_INTERIOR, UNBOUNDED, NONSMOOTH, REFLECT_CAP, NOCONV = 0, 1, 2, 4, 5, 6, 7, 9
HNR, CHNR, BILLIARD, HMC = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (reproducible FP: no fast-math, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC_PATH):
        subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared",
                               "-o", LIB_PATH, SRC_PATH, "-lm"], cwd=_HERE)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        dp, ip, i8p, i32p = (C.POINTER(C.c_double), C.POINTER(C.c_int), C.POINTER(C.c_int8),
                             C.POINTER(C.c_int32))
        vp = C.c_void_p
        L.orc_create.argtypes = [C.c_int, C.c_int, ip, ip, dp, C.POINTER(vp)]
        L.orc_destroy.argtypes = [vp]
        L.orc_philox.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
        L.orc_membership.argtypes = [vp, C.c_int, dp, i8p]
        L.orc_intersect.argtypes = [vp, C.c_int, dp, dp, dp, dp, i32p]
        L.orc_line_bisect.argtypes = [vp, C.c_int, dp, dp, dp, dp, dp, i32p]
        L.orc_reflect.argtypes = [vp, C.c_int, dp, dp, dp, dp, dp, i32p]
        L.orc_intersect_curve2.argtypes = [vp, C.c_int, dp, C.c_double, dp, dp, i32p, i32p]
        L.orc_walk.argtypes = [vp, C.c_int, C.c_int, dp, C.c_int64, C.c_uint64, C.c_double, C.c_int,
                               C.c_double, C.c_double, C.c_int, dp, dp, dp]
        L.orc_billiard_segment.argtypes = [vp, C.c_int, dp, dp, dp, C.c_double, dp, dp, dp, i32p]
        L.orc_volume_balls.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_double, C.c_int, C.c_int,
                                       C.c_uint64, C.c_double, C.c_int, dp, dp, dp, dp, ip]
        L.orc_walk_boltz.argtypes = [vp, C.c_int, C.c_int, dp, C.c_int64, C.c_int64, C.c_uint64, C.c_double,
                                     C.c_int, dp, C.c_double, C.c_double, C.c_int, dp, dp, dp]
        L.orc_sdp_anneal.argtypes = [vp, C.c_int, C.c_int, dp, dp, C.c_double, C.c_double, C.c_int, C.c_int,
                                     C.c_uint64, C.c_double, C.c_int, C.c_double, dp, dp, dp]
        L.orc_volume.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_uint64, C.c_double,
                                 C.c_double, C.c_int, dp, dp, dp, dp]
        L.orc_mlp_nparams.argtypes = [C.c_int, ip]
        L.orc_mlp_nparams.restype = C.c_int64
        L.orc_mlp_forward.argtypes = [C.c_int, ip, dp, C.c_int, dp, dp]
        L.orc_mlp_loss_grad.argtypes = [C.c_int, ip, dp, C.c_int, dp, dp, dp]
        L.orc_mlp_loss_grad.restype = C.c_double
        L.orc_adam_step.argtypes = [C.c_int64, dp, dp, dp, dp, C.c_int, C.c_double, C.c_double,
                                    C.c_double, C.c_double]
        _lib = L
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t=C.c_double):
    return a.ctypes.data_as(C.POINTER(t))


def philox(ctr, key):
    """Philox4x32-10 block for one (4-word counter, 2-word key)."""
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox(c, k, o)
    return [int(v) for v in o]


class Oracle:
    """Oracle bound to one instance (paper_2010_03817_amd.instances.Instance)."""

    def __init__(self, inst):
        self.inst = inst
        self.n = inst.n
        sizes, kinds, A = inst.flat()
        self._sizes, self._kinds, self._A = sizes, kinds, _d(A)
        h = C.c_void_p()
        rc = lib().orc_create(self.n, len(sizes), _p(sizes, C.c_int), _p(kinds, C.c_int), _p(self._A),
                              C.byref(h))
        if rc != OK:
            raise ValueError(f"orc_create failed: {rc}")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def membership(self, x):
        x = _d(x).reshape(-1, self.n)
        out = np.zeros(x.shape[0], dtype=np.int8)
        lib().orc_membership(self._h, x.shape[0], _p(x), _p(out, C.c_int8))
        return out.astype(bool)

    def intersect(self, x, v):
        x = _d(x).reshape(-1, self.n)
        v = _d(v).reshape(-1, self.n)
        B = x.shape[0]
        tm, tp = np.empty(B), np.empty(B)
        st = np.empty(B, dtype=np.int32)
        lib().orc_intersect(self._h, B, _p(x), _p(v), _p(tm), _p(tp), _p(st, C.c_int32))
        return tm, tp, st

    def line_bisect(self, x, v, guess=None):
        """(t-, t+, status) by bisection on membership (no eigen solve)."""
        x = _d(x).reshape(-1, self.n)
        v = _d(v).reshape(-1, self.n)
        B = x.shape[0]
        tm, tp = np.empty(B), np.empty(B)
        st = np.empty(B, dtype=np.int32)
        g = None if guess is None else _d(guess).reshape(B, 2)
        lib().orc_line_bisect(self._h, B, _p(x), _p(v), None if g is None else _p(g), _p(tm), _p(tp),
                              _p(st, C.c_int32))
        return tm, tp, st

    def reflect(self, x, v):
        x = _d(x).reshape(-1, self.n)
        v = _d(v).reshape(-1, self.n)
        B = x.shape[0]
        tp = np.empty(B)
        s, w = np.empty((B, self.n)), np.empty((B, self.n))
        st = np.empty(B, dtype=np.int32)
        lib().orc_reflect(self._h, B, _p(x), _p(v), _p(tp), _p(s), _p(w), _p(st, C.c_int32))
        return tp, s, w, st

    def intersect_curve2(self, coef, horizon=np.inf):
        coef = _d(coef).reshape(-1, 3, self.n + 1)
        B = coef.shape[0]
        tm, tp = np.empty(B), np.empty(B)
        st = np.empty(B, dtype=np.int32)
        it = np.empty(B, dtype=np.int32)
        lib().orc_intersect_curve2(self._h, B, _p(coef), float(horizon), _p(tm), _p(tp),
                                   _p(st, C.c_int32), _p(it, C.c_int32))
        return tm, tp, st, it

    def walk(self, kind, x0, steps, seed, tau=1.0, rho=None, gauss_a=0.0, pullback=1e-6, thin=0):
        x0 = _d(x0).reshape(-1, self.n)
        ch = x0.shape[0]
        rho = 10 * self.n if rho is None else rho
        xo = np.empty_like(x0)
        ns = steps // thin if thin > 0 else 0
        samples = np.empty((ch, max(ns, 1), self.n))
        stats = np.zeros(8)
        rc = lib().orc_walk(self._h, kind, ch, _p(x0), steps, seed, tau, rho, gauss_a, pullback, thin,
                            _p(xo), _p(samples), _p(stats))
        if rc != OK:
            raise ValueError(f"orc_walk failed: {rc}")
        return xo, samples[:, :ns], stats

    def walk_boltz(self, kind, x0, steps, seed, c, T, tau=1.0, rho=None, pullback=1e-6, thin=0, step0=0):
        """Walk on exp(-<c, x> / T) truncated to S (HNR, CHNR or HMC)."""
        x0 = _d(x0).reshape(-1, self.n)
        ch = x0.shape[0]
        rho = 10 * self.n if rho is None else rho
        c = _d(c).reshape(self.n)
        xo = np.empty_like(x0)
        ns = steps // thin if thin > 0 else 0
        samples = np.empty((ch, max(ns, 1), self.n))
        stats = np.zeros(8)
        rc = lib().orc_walk_boltz(self._h, kind, ch, _p(x0), step0, steps, seed, tau, rho, _p(c), T, pullback,
                                  thin, _p(xo), _p(samples), _p(stats))
        if rc != OK:
            raise ValueError(f"orc_walk_boltz failed: {rc}")
        return xo, samples[:, :ns], stats

    def sdp_anneal(self, kind, x0, c, T0, cool, iters, walk_len, seed, tau0, rho=None, pullback=1e-6):
        """Annealing for min <c, x> over S: (x_best, f_best, best per iteration)."""
        x0 = _d(x0).reshape(-1, self.n)
        ch = x0.shape[0]
        rho = 10 * self.n if rho is None else rho
        c = _d(c).reshape(self.n)
        xb, fb = np.empty_like(x0), np.empty(ch)
        best = np.empty((ch, max(iters, 1)))
        rc = lib().orc_sdp_anneal(self._h, kind, ch, _p(x0), _p(c), T0, cool, iters, walk_len, seed, tau0, rho,
                                  pullback, _p(xb), _p(fb), _p(best))
        if rc != OK:
            raise ValueError(f"orc_sdp_anneal failed: {rc}")
        return xb, fb, best[:, :iters]

    def volume_balls(self, chains, spc, walk_len, burn_in, q, max_phases, ball_draws, seed, tau, groups=8):
        """Ball-sequence volume: (log_vol, ci_lo, ci_hi, radii, phases, status)."""
        lv, lo, hi = C.c_double(), C.c_double(), C.c_double()
        radii = np.full(max_phases + 1, np.nan)
        ph = C.c_int()
        rc = lib().orc_volume_balls(self._h, chains, spc, walk_len, burn_in, q, max_phases, ball_draws, seed, tau,
                                    groups, C.byref(lv), C.byref(lo), C.byref(hi), _p(radii), C.byref(ph))
        if rc not in (OK, NOCONV):
            raise ValueError(f"orc_volume_balls failed: {rc}")
        return lv.value, lo.value, hi.value, radii[:ph.value + 1], ph.value, rc

    def billiard_segment(self, x, v, ell, pullback=1e-6):
        x = _d(x).reshape(-1, self.n)
        v = _d(v).reshape(-1, self.n)
        ell = _d(ell).reshape(-1)
        B = x.shape[0]
        xn, vn, el = np.empty_like(x), np.empty_like(v), np.empty(B)
        fl = np.empty((B, 2), dtype=np.int32)
        lib().orc_billiard_segment(self._h, B, _p(x), _p(v), _p(ell), pullback, _p(xn), _p(vn), _p(el),
                                   _p(fl, C.c_int32))
        return xn, vn, el, fl[:, 0].astype(bool), fl[:, 1]

    def volume(self, phases, samples_per_phase, chains, walk_len, seed, a0, a_end, groups=8):
        lv, lo, hi = C.c_double(), C.c_double(), C.c_double()
        lr = np.empty(phases + 1)
        rc = lib().orc_volume(self._h, phases, samples_per_phase, chains, walk_len, seed, a0, a_end, groups,
                              C.byref(lv), C.byref(lo), C.byref(hi), _p(lr))
        if rc != OK:
            raise ValueError(f"orc_volume failed: {rc}")
        return lv.value, lo.value, hi.value, lr


def mlp_nparams(dims):
    d = np.ascontiguousarray(dims, dtype=np.int32)
    return int(lib().orc_mlp_nparams(len(d) - 1, _p(d, C.c_int)))


def mlp_forward(dims, params, X):
    d = np.ascontiguousarray(dims, dtype=np.int32)
    X = _d(X)
    P = _d(params)
    Y = np.empty((X.shape[0], d[-1]))
    lib().orc_mlp_forward(len(d) - 1, _p(d, C.c_int), _p(P), X.shape[0], _p(X), _p(Y))
    return Y


def mlp_loss_grad(dims, params, X, T):
    d = np.ascontiguousarray(dims, dtype=np.int32)
    X, T, P = _d(X), _d(T), _d(params)
    G = np.empty_like(P)
    loss = lib().orc_mlp_loss_grad(len(d) - 1, _p(d, C.c_int), _p(P), X.shape[0], _p(X), _p(T), _p(G))
    return loss, G


def adam_step(params, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In-place Adam update of float64 arrays."""
    for a in (params, grad, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().orc_adam_step(params.size, _p(params), _p(grad), _p(m), _p(v), step, lr, b1, b2, eps)
