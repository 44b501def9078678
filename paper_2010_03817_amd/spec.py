"""Python binding of the C ABI in include/spec.h (argument marshalling only).

Every step of the oracle runs in the HIP kernels of libspec.so.  Tensors are
torch float64 CUDA (ROCm) tensors; calls are enqueued on torch's current
stream.  There is no CPU fallback: if libspec.so is missing or no device is
usable the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspec.so")
HEADERS = [os.path.join(os.path.dirname(_HERE), "include", h) for h in ("spec.h", "spec_diag.h")]

OK, EINVAL, ENOMEM, EDEVICE, NOT_INTERIOR, UNBOUNDED, NONSMOOTH, REFLECT_CAP, CERT_FALLBACK, NOCONV, ENOTSUP = range(11)
DENSE, DIAG = 0, 1
HNR, CHNR, BILLIARD, HMC = 0, 1, 2, 3
PREC_FP64, PREC_FP32_ASM, PREC_BF16X2_ASM = 0, 1, 2
PHASE_SLOTS = 24  # SPEC_DIAG_PHASE_SLOTS


class SpecError(RuntimeError):
    pass


class WalkParams(C.Structure):
    _fields_ = [("tau", C.c_double), ("rho", C.c_int), ("gauss_a", C.c_double), ("pullback", C.c_double),
                ("thin", C.c_int), ("max_rounds", C.c_longlong), ("resume", C.c_int), ("log_chains", C.c_int),
                ("log_cap", C.c_int),
                ("log_buf", C.c_void_p), ("log_count", C.c_void_p), ("boltz_c", C.c_void_p),
                ("boltz_T", C.c_double), ("ball_radius", C.c_double)]


class VolumeBallsParams(C.Structure):
    _fields_ = [("chains", C.c_int), ("groups", C.c_int), ("samples_per_chain", C.c_int), ("walk_len", C.c_int),
                ("burn_in", C.c_int), ("q", C.c_double), ("max_phases", C.c_int), ("ball_draws", C.c_int),
                ("tau", C.c_double)]


class VolumeBallsStats(C.Structure):
    _fields_ = [("phases", C.c_int), ("radii", C.c_double * 257), ("log_ratios", C.c_double * 257),
                ("points", C.c_double), ("oracle_calls", C.c_double), ("tau", C.c_double)]


class AnnealParams(C.Structure):
    _fields_ = [("kind", C.c_int), ("iterations", C.c_int), ("walk_len", C.c_int), ("T0", C.c_double),
                ("cool", C.c_double), ("tau0", C.c_double), ("rho", C.c_int), ("pullback", C.c_double),
                ("f_star", C.c_double), ("eps", C.c_double), ("stop_when_reached", C.c_int)]


class WalkStats(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("calls", "reflections", "cap_hits", "not_interior", "nonsmooth", "steps",
                                          "noconv", "rounds", "cert_fallback", "refined", "refine_failed",
                                          "uncertified", "chol_cert_failed", "escalated")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Options(C.Structure):
    _fields_ = [("precision", C.c_int), ("kmax", C.c_int), ("tol", C.c_double), ("refine_ratio", C.c_double),
                ("tol_loose", C.c_double), ("certify", C.c_int), ("escalate_ratio", C.c_double),
                ("refresh_period", C.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class VolumeParams(C.Structure):
    _fields_ = [("phases", C.c_int), ("samples_per_phase", C.c_int), ("chains", C.c_int), ("walk_len", C.c_int),
                ("groups", C.c_int), ("a0", C.c_double), ("a_end", C.c_double), ("burn_in", C.c_int)]


class VolumeStats(C.Structure):
    _fields_ = [("a0", C.c_double), ("a_end", C.c_double), ("p_inside", C.c_double), ("oracle_calls", C.c_double),
                ("phases", C.c_int), ("log_terms", C.c_double * 257)]


class MlpTrainParams(C.Structure):
    _fields_ = [("epochs", C.c_int), ("batch", C.c_int), ("lr", C.c_double), ("lr_final", C.c_double),
                ("val_frac", C.c_double), ("quantile", C.c_double), ("seed", C.c_uint64), ("keep_best", C.c_int)]


class MlpTrainStats(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("train_loss", "val_loss", "delta", "err_median", "err_p99", "err_max",
                                          "steps", "val_rows")] + [("err_q", C.c_double * 8),
                                                                   ("val_loss_const", C.c_double),
                                                                   ("best_epoch", C.c_double)]
    QUANTILE_LEVELS = (0.5, 0.7, 0.8, 0.9, 0.95, 0.99, 0.995, 0.999)

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "err_q"}
        d["err_q"] = dict(zip(self.QUANTILE_LEVELS, list(self.err_q)))
        return d


_lib = None


def declared_symbols():
    """Function names declared in include/spec*.h."""
    names = []
    for h in HEADERS:
        txt = open(h).read()
        names += re.findall(r"^\s*(?:spec_status|const char\*)\s+(spec_\w+)\s*\(", txt, re.M)
    return names


def lib():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise SpecError(f"{LIB_PATH} is not built; run `python -m paper_2010_03817_amd.build`")
    # torch ships its own HIP runtime with the same soname as the system one;
    # initialise torch first so that libspec.so binds to the runtime torch uses.
    import torch
    torch.cuda.is_available()
    L = C.CDLL(LIB_PATH)
    vp, ip, dp = C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_double)
    L.spec_create.argtypes = [C.c_int, C.c_int, ip, ip, dp, C.POINTER(vp)]
    L.spec_destroy.argtypes = [vp]
    L.spec_dims.argtypes = [vp, ip, ip, ip]
    L.spec_status_str.argtypes = [C.c_int]
    L.spec_status_str.restype = C.c_char_p
    L.spec_set_lanczos.argtypes = [vp, C.c_int, C.c_double]
    L.spec_walk_state.argtypes = [vp, C.c_int]
    L.spec_certificates.argtypes = [vp, C.c_int, vp, vp]
    L.spec_options_default.argtypes = [C.POINTER(Options)]
    L.spec_create_ex.argtypes = [C.c_int, C.c_int, ip, ip, dp, C.POINTER(Options), C.POINTER(vp)]
    L.spec_set_options.argtypes = [vp, C.POINTER(Options)]
    L.spec_get_options.argtypes = [vp, C.POINTER(Options)]
    L.spec_set_precision.argtypes = [vp, C.c_int]
    L.spec_membership_dev.argtypes = [vp, C.c_int, vp, vp, vp]
    L.spec_intersect_dev.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp, vp]
    L.spec_intersect_noalloc_dev.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp, vp]
    L.spec_reflect_dev.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp, vp, vp]
    L.spec_membership.argtypes = [vp, C.c_int, vp, vp]
    L.spec_intersect.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp]
    L.spec_intersect_curve.argtypes = [vp, C.c_int, C.c_int, vp, C.c_double, vp, vp, vp]
    L.spec_intersect_curve_dev.argtypes = [vp, C.c_int, C.c_int, vp, C.c_double, vp, vp, vp, vp]
    L.spec_reflect.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp, vp]
    L.spec_walk_run_dev.argtypes = [vp, C.c_int, C.c_int, vp, C.c_longlong, C.c_uint64, C.POINTER(WalkParams), vp,
                                    vp, C.POINTER(WalkStats), vp]
    L.spec_walk_run.argtypes = [vp, C.c_int, C.c_int, vp, C.c_longlong, C.c_uint64, C.POINTER(WalkParams), vp,
                                vp, C.POINTER(WalkStats)]
    L.spec_diag_timing.argtypes = [vp, C.c_int]
    L.spec_diag_phase_profile.argtypes = [vp, C.c_int]
    L.spec_diag_phase_stamps.argtypes = [vp, C.c_int, vp]
    L.spec_diag_stage_times.argtypes = [vp, vp, vp]
    L.spec_diag_assembly_rows.argtypes = [vp, vp]
    L.spec_diag_mfma_layout.argtypes = [vp]
    L.spec_diag_gemm_f64.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, vp, vp, vp]
    L.spec_diag_lanczos_info.argtypes = [vp, C.c_int, vp]
    L.spec_diag_call_flags.argtypes = [vp, C.c_int, vp]
    L.spec_diag_mfma_raw.argtypes = [C.c_int, C.c_int, vp, vp, vp]
    L.spec_diag_gemm_f32.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, vp, C.c_int, vp,
                                     C.c_int, vp, C.c_int, vp, C.c_int]
    L.spec_mlp_create.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_uint64, C.POINTER(vp)]
    L.spec_mlp_create_ex.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, C.c_uint64, C.c_int, C.POINTER(vp)]
    L.spec_mlp_standardization.argtypes = [vp, vp, vp, vp]
    L.spec_mlp_destroy.argtypes = [vp]
    L.spec_mlp_nparams.argtypes = [vp, C.POINTER(C.c_longlong)]
    L.spec_mlp_get_params.argtypes = [vp, vp]
    L.spec_mlp_set_params.argtypes = [vp, vp]
    L.spec_mlp_forward_dev.argtypes = [vp, C.c_int, vp, vp, vp]
    L.spec_mlp_loss_grad_dev.argtypes = [vp, C.c_int, vp, vp, vp, C.POINTER(C.c_double), vp]
    L.spec_mlp_adam_dev.argtypes = [vp, vp, C.c_double, vp]
    L.spec_mlp_train_dev.argtypes = [vp, C.c_int, vp, vp, vp, vp, C.POINTER(MlpTrainParams),
                                     C.POINTER(MlpTrainStats), vp]
    L.spec_mlp_train.argtypes = [vp, C.c_int, vp, vp, vp, vp, C.POINTER(MlpTrainParams), C.POINTER(MlpTrainStats)]
    L.spec_mlp_predict_dev.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp]
    L.spec_set_mlp.argtypes = [vp, vp, C.c_double, C.c_int]
    L.spec_batch_create.argtypes = [C.c_int, C.POINTER(vp), C.POINTER(vp)]
    L.spec_batch_destroy.argtypes = [vp]
    L.spec_batch_set_strategy.argtypes = [vp, C.c_int, C.c_int]
    L.spec_batch_tune.argtypes = [vp, C.c_int, C.c_int, vp, C.POINTER(C.c_int)]
    L.spec_batch_volume.argtypes = [vp, C.POINTER(VolumeParams), C.c_uint64, vp, vp, vp, C.POINTER(C.c_double)]
    L.spec_batch_intersect.argtypes = [vp, C.c_int, vp, vp, vp, vp, vp]
    L.spec_volume_balls.argtypes = [vp, C.POINTER(VolumeBallsParams), C.c_uint64, C.POINTER(C.c_double),
                                    C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(VolumeBallsStats)]
    L.spec_sdp_anneal.argtypes = [vp, C.POINTER(AnnealParams), C.c_int, vp, vp, C.c_uint64, vp, vp, vp, vp,
                                  C.POINTER(WalkStats)]
    L.spec_volume_estimate.argtypes = [vp, C.POINTER(VolumeParams), C.c_uint64, C.POINTER(C.c_double),
                                       C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(VolumeStats), vp]
    L.spec_tune_mlp_delta_dev.argtypes = [vp, vp, C.c_int, vp, vp, C.c_int, vp, C.c_int, vp, C.POINTER(C.c_double),
                                          vp]
    for name in declared_symbols():
        if name != "spec_status_str":
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(rc):
    if rc != OK:
        msg = lib().spec_status_str(rc).decode()
        raise SpecError(f"spec call failed: {msg} ({rc})")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise SpecError("no GPU device available to torch")
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _f64(t, shape=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t, dtype=np.float64))
    t = t.to(device="cuda", dtype=torch.float64).contiguous()
    if shape is not None:
        t = t.reshape(shape)
    return t


class Spectrahedron:
    """Device handle of an LMI (instances.Instance)."""

    def __init__(self, inst, kmax: int | None = None, tol: float | None = None, **options):
        """options: fields of spec_options (precision, kmax, tol, refine_ratio,
        tol_loose, certify, escalate_ratio, refresh_period) over
        spec_options_default."""
        _torch()
        self.inst = inst
        self.n = inst.n
        sizes, kinds, A = inst.flat()
        self._keep = (sizes, kinds, np.ascontiguousarray(A, dtype=np.float64))
        h = C.c_void_p()
        opt = None
        if options:
            opt = Options()
            check(lib().spec_options_default(C.byref(opt)))
            for k, val in options.items():
                if k not in opt.as_dict():
                    raise TypeError(f"unknown option {k}")
                setattr(opt, k, val)
        check(lib().spec_create_ex(self.n, len(sizes), sizes.ctypes.data_as(C.POINTER(C.c_int)),
                                   kinds.ctypes.data_as(C.POINTER(C.c_int)),
                                   self._keep[2].ctypes.data_as(C.POINTER(C.c_double)),
                                   C.byref(opt) if opt is not None else None, C.byref(h)))
        self._h = h
        n, m, md = C.c_int(), C.c_int(), C.c_int()
        check(lib().spec_dims(h, C.byref(n), C.byref(m), C.byref(md)))
        self.m, self.md = m.value, md.value
        if kmax is not None or tol is not None:
            self.set_lanczos(kmax or 80, tol or 1e-8)

    def set_lanczos(self, kmax: int, tol: float):
        check(lib().spec_set_lanczos(self._h, int(kmax), float(tol)))

    def options(self):
        o = Options()
        check(lib().spec_get_options(self._h, C.byref(o)))
        return o.as_dict()

    def set_options(self, **changes):
        o = Options()
        check(lib().spec_get_options(self._h, C.byref(o)))
        for k, val in changes.items():
            if k not in o.as_dict():
                raise TypeError(f"unknown option {k}")
            setattr(o, k, val)
        check(lib().spec_set_options(self._h, C.byref(o)))

    def set_precision(self, mode: int):
        """Pencil assembly precision: PREC_FP64, PREC_FP32_ASM, PREC_BF16X2_ASM."""
        check(lib().spec_set_precision(self._h, int(mode)))

    def close(self):
        if getattr(self, "_h", None):
            lib().spec_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ oracle calls

    def membership(self, x):
        torch = _torch()
        x = _f64(x)
        x = x.reshape(-1, self.n)
        out = torch.empty(x.shape[0], dtype=torch.int8, device="cuda")
        check(lib().spec_membership_dev(self._h, x.shape[0], _ptr(x), _ptr(out), _stream()))
        return out.bool()

    def intersect(self, x, v):
        torch = _torch()
        x, v = _f64(x).reshape(-1, self.n), _f64(v).reshape(-1, self.n)
        B = x.shape[0]
        tm = torch.empty(B, dtype=torch.float64, device="cuda")
        tp = torch.empty_like(tm)
        st = torch.empty(B, dtype=torch.int32, device="cuda")
        check(lib().spec_intersect_dev(self._h, B, _ptr(x), _ptr(v), _ptr(tm), _ptr(tp), _ptr(st), _stream()))
        return tm, tp, st

    def intersect_noalloc(self, x, v, tm, tp, st):
        """spec_intersect_noalloc_dev into caller-provided device tensors
        (float64 t-, t+ and int32 status of the batch size)."""
        x, v = _f64(x).reshape(-1, self.n), _f64(v).reshape(-1, self.n)
        B = x.shape[0]
        assert tm.numel() >= B and tp.numel() >= B and st.numel() >= B
        check(lib().spec_intersect_noalloc_dev(self._h, B, _ptr(x), _ptr(v), _ptr(tm), _ptr(tp), _ptr(st),
                                               _stream()))
        return tm[:B], tp[:B], st[:B]

    def intersect_curve(self, coef, horizon=float("inf"), degree=2):
        """First positive / negative roots of det(sum_k t^k Q_k) within the
        horizon; coef: batch x (degree+1) x (n+1), degree 1 .. 6."""
        torch = _torch()
        coef = _f64(coef).reshape(-1, degree + 1, self.n + 1)
        B = coef.shape[0]
        tm = torch.empty(B, dtype=torch.float64, device="cuda")
        tp = torch.empty_like(tm)
        st = torch.empty(B, dtype=torch.int32, device="cuda")
        check(lib().spec_intersect_curve_dev(self._h, B, degree, _ptr(coef), float(horizon), _ptr(tm), _ptr(tp),
                                             _ptr(st), _stream()))
        return tm, tp, st

    def reflect(self, x, v):
        torch = _torch()
        x, v = _f64(x).reshape(-1, self.n), _f64(v).reshape(-1, self.n)
        B = x.shape[0]
        tp = torch.empty(B, dtype=torch.float64, device="cuda")
        s = torch.empty_like(x)
        w = torch.empty_like(x)
        st = torch.empty(B, dtype=torch.int32, device="cuda")
        check(lib().spec_reflect_dev(self._h, B, _ptr(x), _ptr(v), _ptr(tp), _ptr(s), _ptr(w), _ptr(st),
                                     _stream()))
        return tp, s, w, st

    def walk(self, kind, x0, steps, seed, tau=1.0, rho=0, gauss_a=0.0, pullback=1e-6, thin=0, max_rounds=0,
             log_chains=0, log_cap=0, resume=False, boltz_c=None, boltz_T=0.0, ball_radius=0.0):
        """Run chains of a walk (HNR, CHNR, BILLIARD) from x0; returns
        (x_out, samples or None, stats dict, log or None).  The log holds rows
        (x, v, t-, t+, chain, status) of segments of the first log_chains chains."""
        torch = _torch()
        x0 = _f64(x0).reshape(-1, self.n)
        ch = x0.shape[0]
        x_out = torch.empty_like(x0)
        ns = steps // thin if thin > 0 else 0
        samples = torch.empty((ch, ns, self.n), dtype=torch.float64, device="cuda") if ns > 0 else None
        log = cnt = None
        if log_cap > 0:
            log = torch.empty((log_cap, 2 * self.n + 4), dtype=torch.float64, device="cuda")
            cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
        bc = None if boltz_c is None else _f64(boltz_c).reshape(self.n)
        p = WalkParams(tau=tau, rho=rho, gauss_a=gauss_a, pullback=pullback, thin=thin, max_rounds=max_rounds,
                       resume=int(resume), log_chains=log_chains, log_cap=log_cap, log_buf=_ptr(log),
                       log_count=_ptr(cnt), boltz_c=_ptr(bc), boltz_T=boltz_T, ball_radius=ball_radius)
        st = WalkStats()
        check(lib().spec_walk_run_dev(self._h, kind, ch, _ptr(x0), steps, seed, C.byref(p), _ptr(x_out),
                                      _ptr(samples), C.byref(st), _stream()))
        if log is not None:
            k = min(int(cnt.item()), log_cap)
            log = log[:k]
        return x_out, samples, st.as_dict(), log

    def walk_host(self, kind, x0, steps, seed, tau=1.0, rho=0, gauss_a=0.0, pullback=1e-6, thin=0,
                  max_rounds=0):
        """spec_walk_run on host arrays: (x_out, samples or None, stats)."""
        x0 = np.ascontiguousarray(x0, dtype=np.float64).reshape(-1, self.n)
        ch = x0.shape[0]
        x_out = np.empty_like(x0)
        ns = steps // thin if thin > 0 else 0
        samples = np.empty((ch, ns, self.n)) if ns > 0 else None
        p = WalkParams(tau=tau, rho=rho, gauss_a=gauss_a, pullback=pullback, thin=thin, max_rounds=max_rounds)
        st = WalkStats()
        check(lib().spec_walk_run(self._h, kind, ch, x0.ctypes.data, steps, seed, C.byref(p), x_out.ctypes.data,
                                  samples.ctypes.data if samples is not None else None, C.byref(st)))
        return x_out, samples, st.as_dict()

    def volume_balls(self, chains=1024, groups=8, samples_per_chain=16, walk_len=1, burn_in=-1, q=0.2,
                     max_phases=256, ball_draws=4096, tau=0.0, seed=1):
        """spec_volume_balls: (log_vol, ci_lo, ci_hi, stats dict with radii and
        log_ratios trimmed to the phases run)."""
        p = VolumeBallsParams(chains=chains, groups=groups, samples_per_chain=samples_per_chain, walk_len=walk_len,
                              burn_in=burn_in, q=q, max_phases=max_phases, ball_draws=ball_draws, tau=tau)
        lv, lo, hi = C.c_double(), C.c_double(), C.c_double()
        st = VolumeBallsStats()
        check(lib().spec_volume_balls(self._h, C.byref(p), int(seed), C.byref(lv), C.byref(lo), C.byref(hi),
                                      C.byref(st)))
        k = st.phases
        return lv.value, lo.value, hi.value, {"phases": k, "radii": list(st.radii[:k]),
                                              "log_ratios": list(st.log_ratios[:k + 1]), "points": st.points,
                                              "oracle_calls": st.oracle_calls, "tau": st.tau}

    def sdp_anneal(self, x0, c, T0, tau0, iterations=70, walk_len=1, kind=None, cool=0.0, seed=1, rho=0,
                   pullback=1e-6, f_star=float("nan"), eps=0.05, stop_when_reached=False):
        """spec_sdp_anneal on host arrays: (x_best, f_best, best history
        (chains x iterations), hit_iter, stats)."""
        kind = HMC if kind is None else kind
        x0 = np.ascontiguousarray(x0, dtype=np.float64).reshape(-1, self.n)
        c = np.ascontiguousarray(c, dtype=np.float64).reshape(self.n)
        ch = x0.shape[0]
        p = AnnealParams(kind=kind, iterations=iterations, walk_len=walk_len, T0=T0, cool=cool, tau0=tau0, rho=rho,
                         pullback=pullback, f_star=f_star, eps=eps, stop_when_reached=int(bool(stop_when_reached)))
        xb, fb = np.empty_like(x0), np.empty(ch)
        best = np.empty((ch, max(iterations, 1)))
        hit = np.empty(ch, np.int32)
        st = WalkStats()
        check(lib().spec_sdp_anneal(self._h, C.byref(p), ch, x0.ctypes.data_as(C.c_void_p),
                                    c.ctypes.data_as(C.c_void_p), int(seed), xb.ctypes.data_as(C.c_void_p),
                                    fb.ctypes.data_as(C.c_void_p), best.ctypes.data_as(C.c_void_p),
                                    hit.ctypes.data_as(C.c_void_p), C.byref(st)))
        return xb, fb, best[:, :iterations], hit, st.as_dict()

    def save_walk_state(self):
        check(lib().spec_walk_state(self._h, 0))

    def restore_walk_state(self):
        check(lib().spec_walk_state(self._h, 1))

    def timing(self, on: bool):
        check(lib().spec_diag_timing(self._h, int(on)))

    def stage_times(self):
        """{stage: (ms total, launches)} and the summed Lanczos steps."""
        out = np.zeros(10)
        ls = C.c_double()
        check(lib().spec_diag_stage_times(self._h, out.ctypes.data_as(C.c_void_p), C.byref(ls)))
        names = ["assemble", "predict", "fused", "normal", "update"]
        return {k: (out[i], out[5 + i]) for i, k in enumerate(names)}, ls.value

    def assembly_rows(self):
        """Pencil rows assembled by line-oracle rounds while timing was on."""
        r = C.c_double()
        check(lib().spec_diag_assembly_rows(self._h, C.byref(r)))
        return r.value

    def phase_profile(self, max_chains: int):
        check(lib().spec_diag_phase_profile(self._h, int(max_chains)))

    def phase_stamps(self, batch):
        out = np.zeros((batch, PHASE_SLOTS), dtype=np.int64)
        check(lib().spec_diag_phase_stamps(self._h, batch, out.ctypes.data_as(C.c_void_p)))
        return out

    def volume(self, phases=20, samples_per_phase=2000, chains=64, walk_len=10, groups=8, a0=0.0, a_end=0.0,
               seed=1, burn_in=-1):
        """Gaussian-cooling volume estimate: (log vol, ci_lo, ci_hi, stats)."""
        p = VolumeParams(phases=phases, samples_per_phase=samples_per_phase, chains=chains, walk_len=walk_len,
                         groups=groups, a0=a0, a_end=a_end, burn_in=burn_in)
        lv, lo, hi = C.c_double(), C.c_double(), C.c_double()
        st = VolumeStats()
        check(lib().spec_volume_estimate(self._h, C.byref(p), int(seed), C.byref(lv), C.byref(lo), C.byref(hi),
                                         C.byref(st), _stream()))
        d = {"a0": st.a0, "a_end": st.a_end, "p_inside": st.p_inside, "oracle_calls": st.oracle_calls,
             "log_terms": list(st.log_terms[:st.phases + 1])}
        return lv.value, lo.value, hi.value, d

    def set_mlp(self, net, delta=0.0, mode=1):
        """Attach a trained Mlp (learned bracket for reflect and billiard walks);
        net None or mode 0 detaches."""
        check(lib().spec_set_mlp(self._h, net._h if net is not None else None, float(delta),
                                 int(mode) if net is not None else 0))
        self._net = net

    def tune_mlp_delta(self, net, x, v, deltas, reps=2):
        """Time the learned reflection of (x, v) for each candidate half-width;
        attaches the fastest.  Returns (best delta, list of ms)."""
        x, v = _f64(x).reshape(-1, self.n), _f64(v).reshape(-1, self.n)
        d = np.ascontiguousarray(deltas, dtype=np.float64)
        ms = np.empty(d.size)
        best = C.c_double()
        check(lib().spec_tune_mlp_delta_dev(self._h, net._h, x.shape[0], _ptr(x), _ptr(v), d.size,
                                            d.ctypes.data_as(C.c_void_p), int(reps), ms.ctypes.data_as(C.c_void_p),
                                            C.byref(best), _stream()))
        self._net = net
        return best.value, list(ms)

    def certificates(self, batch):
        """(t_lo, t_hi) certified interval of t+ of each element of the last call."""
        lo, hi = np.empty(batch), np.empty(batch)
        check(lib().spec_certificates(self._h, batch, lo.ctypes.data, hi.ctypes.data))
        return lo, hi

    def call_flags(self, batch):
        """Per-element bits of the last call: 1 bracket not certified, 4 far root
        refined, 8 refining factor failed."""
        torch = _torch()
        torch.cuda.synchronize()
        out = np.empty(batch, dtype=np.int32)
        check(lib().spec_diag_call_flags(self._h, batch, out.ctypes.data_as(C.c_void_p)))
        return out

    def lanczos_info(self, batch):
        """(lambda_min, lambda_max, learned-bracket code, steps) of the last call."""
        torch = _torch()
        torch.cuda.synchronize()
        out = np.empty((batch, 4))
        check(lib().spec_diag_lanczos_info(self._h, batch, out.ctypes.data_as(C.c_void_p)))
        return out


class Batch:
    """Uneven batch of spectrahedra (include/spec.h, spec_batch_*)."""

    def __init__(self, specs):
        _torch()
        self.specs = list(specs)
        arr = (C.c_void_p * len(self.specs))(*[g._h.value for g in self.specs])
        h = C.c_void_p()
        check(lib().spec_batch_create(len(self.specs), arr, C.byref(h)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().spec_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_strategy(self, strategy, use_graph=True):
        check(lib().spec_batch_set_strategy(self._h, int(strategy), int(bool(use_graph))))

    def tune(self, chains=64, rounds=4):
        ms = np.empty(3)
        k = C.c_int()
        check(lib().spec_batch_tune(self._h, int(chains), int(rounds), ms.ctypes.data_as(C.c_void_p), C.byref(k)))
        return k.value, list(ms)

    def intersect(self, xs, vs):
        """One batched oracle round on host pairs: xs[i], vs[i] of shape
        (chains, n_i) for instance i; returns (t_minus, t_plus, status), each of
        shape (count, chains)."""
        K = len(self.specs)
        chains = int(np.shape(xs[0])[0])
        for i, g in enumerate(self.specs):
            if np.shape(xs[i]) != (chains, g.n) or np.shape(vs[i]) != (chains, g.n):
                raise ValueError(f"instance {i}: pairs must have shape ({chains}, {g.n})")
        x = np.ascontiguousarray(np.concatenate([np.asarray(a, np.float64).ravel() for a in xs]))
        v = np.ascontiguousarray(np.concatenate([np.asarray(a, np.float64).ravel() for a in vs]))
        tm, tp = np.empty((K, chains)), np.empty((K, chains))
        st = np.empty((K, chains), np.int32)
        check(lib().spec_batch_intersect(self._h, chains, x.ctypes.data_as(C.c_void_p), v.ctypes.data_as(C.c_void_p),
                                         tm.ctypes.data_as(C.c_void_p), tp.ctypes.data_as(C.c_void_p),
                                         st.ctypes.data_as(C.c_void_p)))
        return tm, tp, st

    def volume(self, phases=20, samples_per_phase=2000, chains=64, walk_len=10, groups=8, a0=0.0, a_end=0.0,
               seed=1, burn_in=-1):
        K = len(self.specs)
        p = VolumeParams(phases=phases, samples_per_phase=samples_per_phase, chains=chains, walk_len=walk_len,
                         groups=groups, a0=a0, a_end=a_end, burn_in=burn_in)
        lv, lo, hi = np.empty(K), np.empty(K), np.empty(K)
        calls = C.c_double()
        check(lib().spec_batch_volume(self._h, C.byref(p), int(seed), lv.ctypes.data_as(C.c_void_p),
                                      lo.ctypes.data_as(C.c_void_p), hi.ctypes.data_as(C.c_void_p), C.byref(calls)))
        return lv, lo, hi, calls.value


class Mlp:
    """Learned-bracket network (include/spec.h, spec_mlp_*)."""

    def __init__(self, n, width=256, hidden=3, bf16=True, seed=1, products=False):
        _torch()
        h = C.c_void_p()
        check(lib().spec_mlp_create_ex(int(n), int(width), int(hidden), int(bool(bf16)), int(seed),
                                       int(bool(products)), C.byref(h)))
        self._h = h
        self.n = n
        self.nin = 2 * n + (2 if products else 0)
        k = C.c_longlong()
        check(lib().spec_mlp_nparams(h, C.byref(k)))
        self.nparams = k.value
        self.train_stats = None

    def close(self):
        if getattr(self, "_h", None):
            lib().spec_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def standardization(self):
        """(mu, isd, target (mean, sd of log t+, of log(-t-))) of the features."""
        mu, isd, tg = np.empty(self.nin, np.float32), np.empty(self.nin, np.float32), np.empty(4, np.float32)
        check(lib().spec_mlp_standardization(self._h, mu.ctypes.data_as(C.c_void_p), isd.ctypes.data_as(C.c_void_p),
                                             tg.ctypes.data_as(C.c_void_p)))
        return mu, isd, tg

    def get_params(self):
        out = np.empty(self.nparams, dtype=np.float32)
        check(lib().spec_mlp_get_params(self._h, out.ctypes.data_as(C.c_void_p)))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.nparams
        check(lib().spec_mlp_set_params(self._h, p.ctypes.data_as(C.c_void_p)))

    def _f32(self, a, cols):
        torch = _torch()
        if not isinstance(a, torch.Tensor):
            a = torch.as_tensor(np.asarray(a, dtype=np.float32))
        return a.to(device="cuda", dtype=torch.float32).contiguous().reshape(-1, cols)

    def forward(self, X):
        """Raw network outputs (rows x 2) for raw features X (rows x inputs)."""
        torch = _torch()
        X = self._f32(X, self.nin)
        Y = torch.empty((X.shape[0], 2), dtype=torch.float32, device="cuda")
        check(lib().spec_mlp_forward_dev(self._h, X.shape[0], _ptr(X), _ptr(Y), _stream()))
        return Y

    def loss_grad(self, X, T):
        torch = _torch()
        X = self._f32(X, self.nin)
        T = self._f32(T, 2)
        G = torch.empty(self.nparams, dtype=torch.float32, device="cuda")
        loss = C.c_double()
        check(lib().spec_mlp_loss_grad_dev(self._h, X.shape[0], _ptr(X), _ptr(T), _ptr(G), C.byref(loss), _stream()))
        return loss.value, G

    def adam(self, grad, lr):
        check(lib().spec_mlp_adam_dev(self._h, _ptr(grad), float(lr), _stream()))

    def train(self, x, v, t_minus, t_plus, epochs=20, batch=4096, lr=1e-3, lr_final=1e-5, val_frac=0.1,
              quantile=0.999, seed=7, keep_best=False):
        x, v = _f64(x).reshape(-1, self.n), _f64(v).reshape(-1, self.n)
        tm, tp = _f64(t_minus).reshape(-1), _f64(t_plus).reshape(-1)
        p = MlpTrainParams(epochs=epochs, batch=batch, lr=lr, lr_final=lr_final, val_frac=val_frac,
                           quantile=quantile, seed=seed, keep_best=int(bool(keep_best)))
        st = MlpTrainStats()
        check(lib().spec_mlp_train_dev(self._h, x.shape[0], _ptr(x), _ptr(v), _ptr(tm), _ptr(tp), C.byref(p),
                                       C.byref(st), _stream()))
        self.train_stats = st.as_dict()
        return self.train_stats

    def train_host(self, x, v, t_minus, t_plus, epochs=20, batch=4096, lr=1e-3, lr_final=1e-5, val_frac=0.1,
                   quantile=0.999, seed=7):
        """spec_mlp_train on host (numpy) triples."""
        a = [np.ascontiguousarray(t, dtype=np.float64) for t in (x, v, t_minus, t_plus)]
        p = MlpTrainParams(epochs=epochs, batch=batch, lr=lr, lr_final=lr_final, val_frac=val_frac,
                           quantile=quantile, seed=seed)
        st = MlpTrainStats()
        check(lib().spec_mlp_train(self._h, a[2].shape[0], a[0].ctypes.data, a[1].ctypes.data, a[2].ctypes.data,
                                   a[3].ctypes.data, C.byref(p), C.byref(st)))
        self.train_stats = st.as_dict()
        return self.train_stats

    def predict(self, x, v):
        """(log t+_hat, log(-t-_hat)) of the trained network."""
        torch = _torch()
        x, v = _f64(x).reshape(-1, self.n), _f64(v).reshape(-1, self.n)
        a = torch.empty(x.shape[0], dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        check(lib().spec_mlp_predict_dev(self._h, x.shape[0], _ptr(x), _ptr(v), _ptr(a), _ptr(b), _stream()))
        return a, b


def mfma_raw(kind, a, b):
    """One MFMA per trial with per-lane operands (see spec_diag_mfma_raw)."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    b = np.ascontiguousarray(b, dtype=np.float32)
    per = 64 if kind == 0 else 512
    trials = a.size // per
    d = np.empty((trials, 64, 4), dtype=np.float32)
    check(lib().spec_diag_mfma_raw(kind, trials, a.ctypes.data_as(C.c_void_p), b.ctypes.data_as(C.c_void_p),
                                   d.ctypes.data_as(C.c_void_p)))
    return d


def gemm_f32(A, B, ta=False, tb=False, bf16=False, mode=0, aux=None, C0=None):
    """The MLP GEMM on host arrays: returns (C, aux)."""
    A = np.ascontiguousarray(A, dtype=np.float32)
    B = np.ascontiguousarray(B, dtype=np.float32)
    M = A.shape[1] if ta else A.shape[0]
    K = A.shape[0] if ta else A.shape[1]
    N = B.shape[0] if tb else B.shape[1]
    Cm = np.zeros((M, N), dtype=np.float32) if C0 is None else np.ascontiguousarray(C0, dtype=np.float32).copy()
    X = None
    if mode:
        X = np.ascontiguousarray(aux, dtype=np.float32).copy()
    check(lib().spec_diag_gemm_f32(int(ta), int(tb), int(bf16), int(mode), M, N, K, A.ctypes.data_as(C.c_void_p),
                                   A.shape[1], B.ctypes.data_as(C.c_void_p), B.shape[1],
                                   Cm.ctypes.data_as(C.c_void_p), N,
                                   X.ctypes.data_as(C.c_void_p) if X is not None else None,
                                   X.shape[1] if X is not None else 0))
    return Cm, X


def mfma_layout():
    out = np.empty(256)
    check(lib().spec_diag_mfma_layout(out.ctypes.data_as(C.c_void_p)))
    return out.reshape(64, 4)


def gemm_f64(A, B, transB=False):
    A = np.ascontiguousarray(A, dtype=np.float64)
    B = np.ascontiguousarray(B, dtype=np.float64)
    M, K = A.shape
    N = B.shape[0] if transB else B.shape[1]
    Cm = np.empty((M, N))
    check(lib().spec_diag_gemm_f64(int(transB), M, N, K, A.ctypes.data_as(C.c_void_p),
                                   B.ctypes.data_as(C.c_void_p), Cm.ctypes.data_as(C.c_void_p)))
    return Cm
