"""Benchmark of the boundary-oracle hot path on one MI355X.

Workload: billiard walk (Alg. Billiard) on the n = m = 200 spectrahedron
(dense block A0 = I, A_i = (G_i + G_i^T)/(2 sqrt(m)), plus the |x_i| <= 10
box as 400 diagonal rows), 16384 chains, step length ell = -tau ln(eta) with
tau = 2 x (diameter estimate), FP64.  One bench "step" is one round of the
walk: every chain runs one segment through the whole oracle (assembly GEMM of
F(x) and B(v), Cholesky + inverse, Lanczos extreme eigenvalue, normal GEMM,
reflection / step logic).  Metric: oracle calls per second (one call per chain
per round) with billiard steps per second beside it, for the plain path and
for the learned-bracket path (network trained on the walk's own segment
starts, half-width autotuned, every t+ certified by an FP64 Cholesky factor);
`value` is the learned path's rate, the plain path's is under "plain".

Prints ONE JSON line.  --gpus N with N > 1 exits: the benchmark runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_DIM, M_DIM, SEED_INST, CHAINS = 200, 200, 103, 16384
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
FUSED_STAGE = "k_line_fused+k_line_refine<false>"


def _fused_traffic(chains, leg):
    """HBM bytes per launch of the fused kernel over the timed rounds of one
    leg ("plain" or "learned"), from the committed counter summary, while the
    kernel sources are those that were profiled."""
    import hashlib
    import re
    src = os.path.join(ROOT, "paper_2010_03817_amd", "csrc")
    hs = "".join(hashlib.sha256(open(os.path.join(src, f), "rb").read()).hexdigest() + "\n"
                 for f in ("line_fused.hip", "line_fused.h", "common.h"))
    digest = hashlib.sha256(hs.encode()).hexdigest()[:16]
    try:
        txt = open(os.path.join(ROOT, "profiles", "k_line_fused_billiard_n200_m200.md")).read()
    except OSError:
        return None
    for m in re.finditer(r"^traffic: (\d+) bytes/launch at (\d+) chains, leg (\w+), sources ([0-9a-f]+)",
                         txt, re.M):
        if m.group(3) == leg and m.group(4) == digest and int(m.group(2)) == chains:
            return float(m.group(1))
    return None


def _cpu_worker(args):
    """Oracle billiard steps for one chain (CPU baseline)."""
    from oracle import oracle as O
    from paper_2010_03817_amd import instances as I
    chain, steps, tau, seed, x0 = args
    o = O.Oracle(I.gbase(N_DIM, M_DIM, seed=SEED_INST))
    t0 = time.time()
    _, _, st = o.walk(O.BILLIARD, x0[None, :], steps, seed=seed + chain, tau=tau)
    return time.time() - t0, st[0], st[5]


def _cpu_reflect_worker(args):
    """Oracle reflections of a chunk of logged pairs (CPU baseline)."""
    from oracle import oracle as O
    from paper_2010_03817_amd import instances as I
    x, v = args
    o = O.Oracle(I.gbase(N_DIM, M_DIM, seed=SEED_INST))
    t0 = time.time()
    o.reflect(x, v)
    return time.time() - t0, len(x)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(tau, x0s, px, pv, workers=16):
    """The FP64 CPU oracle on the host of the GPU: single-thread latency of
    oracle reflect / intersect calls on logged walk pairs of the n = m = 200
    workload, throughput of reflect calls over `workers` processes (one
    process per core of the machine's CPU share), and billiard steps of whole
    oracle walks, one chain per process."""
    from oracle import oracle as O
    from paper_2010_03817_amd import instances as I
    o = O.Oracle(I.gbase(N_DIM, M_DIM, seed=SEED_INST))
    ns = 48
    t0 = time.time()
    o.reflect(px[:ns], pv[:ns])
    lat_reflect = (time.time() - t0) / ns
    t0 = time.time()
    o.intersect(px[ns:2 * ns], pv[ns:2 * ns])
    lat_intersect = (time.time() - t0) / ns
    per = 12
    jobs = [(px[k * per:(k + 1) * per], pv[k * per:(k + 1) * per]) for k in range(workers)]
    t0 = time.time()
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_cpu_reflect_worker, jobs)
    wall = time.time() - t0
    calls = sum(r[1] for r in res)
    busy = max(r[0] for r in res)
    steps = 2
    wjobs = [(c, steps, tau, 9000, x0s[c % len(x0s)]) for c in range(workers)]
    with mp.get_context("spawn").Pool(workers) as pool:
        wres = pool.map(_cpu_worker, wjobs)
    wcalls = sum(r[1] for r in wres)
    wsteps = sum(r[2] for r in wres)
    wbusy = max(r[0] for r in wres)
    try:
        affinity = len(os.sched_getaffinity(0))
    except AttributeError:
        affinity = None
    return {
        "value": calls / busy,
        "unit": "oracle calls/s",
        "cores": workers,
        "kind": "oracle",
        "sample": f"{calls} oracle reflect calls on logged billiard-walk pairs of the n=m=200 workload, "
                  f"{per} per process over {workers} processes (wall {wall:.1f} s); single-thread latency on "
                  f"{ns} pairs each; {workers} chains x {steps} billiard steps of the oracle walk",
        "cpu_model": _cpu_model(),
        "nproc": os.cpu_count(),
        "affinity_cpus": affinity,
        "single_thread_s_per_call": {"reflect": lat_reflect, "intersect": lat_intersect},
        "walk_oracle_calls_per_s": wcalls / wbusy,
        "billiard_steps_per_s": wsteps / wbusy,
    }


def progress(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed_rounds(g, S, x0, tau, rounds, chains):
    """`rounds` oracle rounds of the resumed billiard chains, timed with the
    device synchronised on both sides; stage timers on the launch stream."""
    import torch
    big = 1 << 40
    torch.cuda.synchronize()
    g.timing(True)
    t0 = time.perf_counter()
    _, _, st, _ = g.walk(S.BILLIARD, x0, big, seed=2024, tau=tau, max_rounds=rounds, resume=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    g.timing(False)
    stages, lz_steps = g.stage_times()
    return {"wall": wall, "stats": st, "stages": stages, "lz_steps": lz_steps, "asm_rows": g.assembly_rows()}


def roofline(run, chains, extra_chol=0.0):
    """FP64 roofline of the dominant kernel of a timed run."""
    stages, lz_steps, calls = run["stages"], run["lz_steps"], run["stats"]["calls"]
    dom = max(stages, key=lambda k: stages[k][0])
    launches = max(stages[dom][1], 1)
    ms_dom = stages[dom][0] / launches
    P = M_DIM * (M_DIM + 1) // 2
    if dom == "fused":
        # fused per-chain kernel (Cholesky, inverse, Lanczos, Ritz vector): FP64
        # arithmetic on MFMA and the vector ALUs, both at the FP64 peak.  Counted
        # work is the method's own: Cholesky m^3/3 (and the second one of each
        # learned-bracket fallback), 4 m^2 per Lanczos step, Ritz vector and
        # u = L^-T z, the packed u u^T for the normal GEMM, and the ratio test of
        # the diagonal block, and F(x) = F(x_prev) + s B(v_prev) in the rounds
        # that carry F over; the triangular inverse (m^3/3) is a design choice
        # and is not counted.
        md = 2 * N_DIM
        per_call = M_DIM**3 / 3.0 + 2.0 * M_DIM**2 + P + 3.0 * md
        carried = max(calls - (run["asm_rows"] - calls), 0.0)  # F rows not assembled
        per_call += 2.0 * (P + md) * carried / max(calls, 1.0)
        flops = (calls * per_call + extra_chol * M_DIM**3 / 3.0
                 + lz_steps * (4.0 * M_DIM**2 + 2.0 * M_DIM)) / launches
        roof = {"bound": "alu", "achieved": flops / (ms_dom * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s"}
    else:
        rows = run["asm_rows"] / launches if dom == "assemble" else calls / launches
        K = N_DIM + 1 if dom == "assemble" else P
        Nc = P + 2 * N_DIM if dom == "assemble" else N_DIM
        flops = 2.0 * rows * K * Nc
        roof = {"bound": "mfma", "achieved": flops / (ms_dom * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    roof["traffic_unit"] = "bytes per launch"
    roof["kernel"] = {"fused": FUSED_STAGE, "assemble": "k_gemm_f64_128<false>", "normal": "k_gemm_f64_128<true>",
                      "predict": "k_gemm_f32", "update": "k_walk_update"}[dom]
    if dom == "fused":
        roof["launches"] = "per round: k_line_fused over every chain, then k_line_refine<false> over the queued ones"
    roof["ms_per_launch"] = ms_dom
    return roof


def summary(run, chains, calls_per_step=None):
    """Rates of a timed run.  Billiard steps per second are the steps the
    chains completed inside the timed rounds per second (the chains are
    state_rounds rounds old, several steps each, so step ends are no longer
    in phase); calls per completed step of the same window beside them."""
    st, wall = run["stats"], run["wall"]
    calls = st["calls"]
    return {
        "oracle_calls_per_s": calls / wall,
        "billiard_steps_per_s": st["steps"] / wall,
        "calls_per_step": calls / max(st["steps"], 1),
        "ms_per_round": 1e3 * wall / max(st["rounds"], 1),
        "reflections_per_step": st["reflections"] / max(st["steps"], 1),
        "lanczos_steps_per_call": run["lz_steps"] / max(calls, 1),
        "noconv": st["noconv"],
        "not_interior": st["not_interior"],
        "cert_fallback_rate": st["cert_fallback"] / max(calls, 1),
        # calls whose t+ carries a certified interval of width <= 2e-9 t+
        "certified_rate": 1.0 - st["uncertified"] / max(calls, 1),
        "refined_rate": st["refined"] / max(calls, 1),
        "refine_failed": st["refine_failed"],
        "stage_ms_per_round": {k: v[0] / max(v[1], 1) for k, v in run["stages"].items()},
    }


def train_learned(g, S, tau, chains, rows_target, epochs, data_chains, burn_rounds, seed=77):
    """Walk-generated (x, v, t-, t+) triples -> trained network, and the
    constant-prediction control (the same network with zero weights predicts
    the training mean of log t+ for every pair).  The triples are the segment
    starts of data_chains billiard chains (their own seed) after burn_rounds
    rounds from the centre, the same age as the timed chains: many chains over
    few rounds, since the network generalises to unseen chains far better
    than from fewer, longer chains.  Rows of one chain in ten are held out
    whole: half of them tune each bracket half-width through the real learned
    kernel, the other half measure errors and Lanczos steps.  Returns the
    network with its half-width, the control with its half-width, and a
    report."""
    import torch
    n = N_DIM
    t0 = time.perf_counter()
    rounds = max(1, -(-rows_target // data_chains))
    xd = torch.zeros((data_chains, n), dtype=torch.float64, device="cuda")
    g.walk(S.BILLIARD, xd, 1 << 40, seed=seed, tau=tau, max_rounds=max(burn_rounds, 1))
    _, _, wst, log = g.walk(S.BILLIARD, xd, 1 << 40, seed=seed, tau=tau, max_rounds=rounds, resume=True,
                            log_chains=data_chains, log_cap=rounds * data_chains)
    del xd
    calls_per_step = wst["calls"] / max(wst["steps"], 1)
    # whole chains held out: chain % 10 == 8 is the trainer's validation set
    # (early stopping), chain % 10 == 9 the half-width tuning and evaluation
    # rows, which training never sees
    cid = log[:, 2 * n + 2].to(torch.int64) % 10
    val8, held = cid == 8, cid == 9
    train = ~(val8 | held)
    order = torch.cat([torch.nonzero(train).flatten(), torch.nonzero(val8).flatten(), torch.nonzero(held).flatten()])
    x = log[order, :n].contiguous()
    v = log[order, n:2 * n].contiguous()
    nheld = int(held.sum())
    nval8 = int(val8.sum())
    del log
    tm = torch.empty(x.shape[0], dtype=torch.float64, device="cuda")
    tp = torch.empty_like(tm)
    ok = torch.empty(x.shape[0], dtype=torch.bool, device="cuda")
    for r0 in range(0, x.shape[0], chains):
        a, b, st = g.intersect(x[r0:r0 + chains], v[r0:r0 + chains])
        tm[r0:r0 + chains], tp[r0:r0 + chains] = a, b
        ok[r0:r0 + chains] = (st == S.OK) & torch.isfinite(a) & torch.isfinite(b) & (a < 0) & (b > 0)
    nval = int(ok[x.shape[0] - nheld:].sum())
    nv8 = int(ok[x.shape[0] - nheld - nval8:x.shape[0] - nheld].sum())
    x, v, tm, tp = x[ok], v[ok], tm[ok], tp[ok]
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    rows = x.shape[0]
    ntv = rows - nval  # training and validation rows (the trainer holds out the last nv8 of them)
    vf = (nv8 + 0.25) / ntv
    xv, vv, tpv = x[rows - nval:], v[rows - nval:], tp[rows - nval:]
    half = min(nval // 2, chains)
    xa, va = xv[:half], vv[:half]                      # half-width tuning
    xb, vb, tpb = xv[half:half + chains], vv[half:half + chains], tpv[half:half + chains]  # evaluation
    ltpa = torch.log(tpv[:half]).cpu().numpy()
    ltpb = torch.log(tpb).cpu().numpy()
    levels = (0.5, 0.7, 0.8, 0.9, 0.95, 0.99)

    def reflect_eval(model, delta):
        g.set_mlp(model, delta, 1) if model is not None else g.set_mlp(None)
        tpx = g.reflect(xb, vb)[0]
        info = g.lanczos_info(xb.shape[0])
        return tpx, float(info[:, 3].mean()), float(np.mean(info[:, 2] == 1))

    def tune(model):
        """Half-width candidates from the model's errors on the tuning rows,
        chosen by timing the real learned kernel."""
        lpa = model.predict(xa, va)[0].cpu().numpy()
        cands = [float(np.quantile(np.abs(lpa - ltpa), q)) for q in levels]
        best, ms = g.tune_mlp_delta(model, xa, va, cands, reps=2)
        return best, ms, cands

    def fit(products):
        """Train a network (early stopping on the index % 10 == 8 chains), tune
        its half-width and evaluate it on the unseen chains."""
        net = S.Mlp(n, width=256, hidden=3, bf16=True, seed=seed, products=products)
        t1 = time.perf_counter()
        tr = net.train(x[:ntv], v[:ntv], tm[:ntv], tp[:ntv], epochs=epochs, batch=4096, lr=1e-3,
                       lr_final=1e-5, val_frac=vf, seed=seed, keep_best=True)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t1
        best, ms, cands = tune(net)
        tpl, steps, fb = reflect_eval(net, best)
        err = np.abs(net.predict(xb, vb)[0].cpu().numpy() - ltpb)
        rep = {"inputs": net.nin, "train_seconds": t_train, "best_epoch": tr.get("best_epoch"),
               "adam_steps": tr["steps"], "train_loss": tr["train_loss"], "val_loss": tr["val_loss"],
               "val_loss_constant_predictor": tr.get("val_loss_const"),
               "val_logtp_err": {str(k): val for k, val in tr["err_q"].items()},
               "delta_candidates": dict(zip([str(q) for q in levels], cands)), "tune_ms": ms, "delta": best,
               "eval_logtp_err_median": float(np.median(err)), "eval_logtp_err_rms": float(np.sqrt(np.mean(err**2))),
               "eval_lanczos_steps_per_call": steps, "eval_fallback_rate": fb}
        return net, best, tpl, rep

    progress(f"training on {ntv - nv8} triples, {nv8} for early stopping, {nval} held out "
             f"({t_data:.1f} s to generate)")
    net, best, tpl, rep = fit(True)
    net400, best400, _, rep400 = fit(False)
    # the control: constant log t+ prediction (training mean), tuned the same way
    ctl = S.Mlp(n, width=256, hidden=3, bf16=True, seed=seed + 1)
    ctl.train(x[:ntv], v[:ntv], tm[:ntv], tp[:ntv], epochs=1, batch=4096, lr=1e-3, lr_final=1e-5, val_frac=vf,
              seed=seed)
    ctl.set_params(np.zeros(ctl.nparams, dtype=np.float32))
    cbest, cms, ccands = tune(ctl)
    tpc, steps_c, fb_c = reflect_eval(ctl, cbest)
    tpp, steps_p, _ = reflect_eval(None, 0.0)
    err_ctl = np.abs(ctl.predict(xb, vb)[0].cpu().numpy() - ltpb)

    def relstats(a, b):
        r = (torch.abs(a - b) / b).cpu().numpy()
        return {"median": float(np.median(r)), "p99": float(np.quantile(r, 0.99)), "max": float(r.max())}

    report = {
        "calls_per_step": calls_per_step, "walk_calls": wst["calls"], "walk_steps": wst["steps"],
        "rows": rows, "held_out_rows": nval, "early_stopping_rows": nv8,
        "holdout": "whole chains: index % 10 == 8 early stopping (the trainer's validation rows), "
                   "index % 10 == 9 half-width tuning and evaluation (never seen by training)",
        "data_chains": data_chains, "data_rounds": rounds, "data_burn_in_rounds": burn_rounds,
        "data_seconds": t_data, "epochs": epochs,
        "network": dict(rep, inputs_are="[x, v, <x, v>, |x|^2] (the two products computed from x and v)"),
        "network_400_inputs": dict(rep400, inputs_are="[x, v]"),
        "control": {"kind": "constant log t+ (training mean), zero-weight network",
                    "delta_candidates": dict(zip([str(q) for q in levels], ccands)), "tune_ms": cms,
                    "delta": cbest, "eval_logtp_err_median": float(np.median(err_ctl)),
                    "eval_logtp_err_rms": float(np.sqrt(np.mean(err_ctl**2))),
                    "eval_lanczos_steps_per_call": steps_c, "eval_fallback_rate": fb_c},
        "eval_rows": int(xb.shape[0]),
        "eval_lanczos_steps_per_call_plain": steps_p,
        "learned_vs_plain_tp_rel": relstats(tpl, tpp),
        "control_vs_plain_tp_rel": relstats(tpc, tpp),
    }
    g.set_mlp(None)
    return net, best, ctl, cbest, report, net400, best400


def uneven_volume_all(S, I, samples_per_phase, chunk=32):
    """The batched Gaussian-cooling volume of all 256 spectrahedra of the
    uneven workload (the 16 balls of known volume among them), in batches of
    `chunk` instances that advance together (the cooling rule's phase count is
    the largest of a batch), `samples_per_phase` samples per phase."""
    insts, balls = _uneven_family(I)
    res, t0 = [], time.perf_counter()
    calls = 0.0
    for c0 in range(0, len(insts), chunk):
        specs = [S.Spectrahedron(i) for i in insts[c0:c0 + chunk]]
        b = S.Batch(specs)
        lv, lo, hi, cl = b.volume(phases=0, samples_per_phase=samples_per_phase, chains=64, walk_len=4, groups=8,
                                  seed=404 + c0, burn_in=200)
        calls += cl
        for j in range(len(specs)):
            res.append((float(lv[j]), float(lo[j]), float(hi[j])))
        b.close()
        del specs
        progress(f"uneven volume: {min(c0 + chunk, len(insts))}/{len(insts)} instances, "
                 f"{time.perf_counter() - t0:.0f} s")
    wall = time.perf_counter() - t0
    inside = inside2 = 0
    per_ball = []
    for k in balls:
        nb = insts[k].n
        truth = 0.5 * nb * math.log(math.pi) - math.lgamma(0.5 * nb + 1)
        lv, lo, hi = res[k]
        w = hi - lo
        inside += int(lo <= truth <= hi)
        inside2 += int(lo - 0.5 * w <= truth <= hi + 0.5 * w)
        per_ball.append({"n": nb, "err": lv - truth, "ci_half": 0.5 * w})
    widths = np.array([r[2] - r[1] for r in res])
    return {"instances": len(insts), "samples_per_phase": samples_per_phase, "chains_per_instance": 64,
            "batch": chunk, "seconds": wall, "oracle_calls": calls, "oracle_calls_per_s": calls / wall,
            "balls_within_ci": f"{inside}/{len(balls)}", "balls_within_doubled_ci": f"{inside2}/{len(balls)}",
            "balls": per_ball, "ci_width_median": float(np.median(widths)), "ci_width_max": float(widths.max()),
            "finite": int(np.isfinite([r[0] for r in res]).sum())}


def _uneven_family(I):
    rng = np.random.default_rng(104)
    insts, balls = [], []
    for k in range(256):
        n = int(round(math.exp(rng.uniform(math.log(20), math.log(200)))))
        m = int(round(math.exp(rng.uniform(math.log(20), math.log(200)))))
        if k % 16 == 0:
            m = min(n, 199) + 1
            insts.append(I.arrow_ball(m - 1))
            balls.append(k)
        else:
            insts.append(I.gbase(n, m, seed=1000 + k))
    return insts, balls


def uneven_leg(S, I, samples_per_phase):
    """256 spectrahedra, n and m log-uniform in [20, 200] (every 16th an arrow
    ball of known volume), 64 chains each: launch strategy autotuned, oracle
    round rate of the whole mixed batch, and a batched Gaussian-cooling
    volume of the 16 balls (phase count from the cooling rule: a fixed 20
    phases leaves the ratio estimators' variance exponential in n / 20 at
    n ~ 200) with their errors against pi^(n/2) / Gamma(n/2 + 1)."""
    insts, balls = _uneven_family(I)
    specs = [S.Spectrahedron(i) for i in insts]
    b = S.Batch(specs)
    chains = 64
    chosen, ms = b.tune(chains=chains, rounds=10)
    out = {"instances": len(insts), "chains_per_instance": chains,
           "sum_m3": float(sum(g.m ** 3 for g in specs)),
           "strategy_ms_per_round": {"persistent": ms[0], "size_classes": ms[1], "per_instance": ms[2]},
           "chosen": ["persistent", "size_classes", "per_instance"][chosen - 1],
           "oracle_calls_per_s": len(insts) * chains / (min(ms) * 1e-3)}
    b.close()
    # volume of the 16 balls as one batch (known volumes): phase count from the
    # cooling rule, 200 burn-in steps per phase and samples every 4th step.
    # Shorter walks leave the phases' samples short of mixing in the largest
    # balls and bias the log-volume low (1 step and 50 burn-in: -0.36 to -0.56
    # at n = 138-184, outside the interval)
    progress("uneven batch: batched volume of the 16 balls")
    bb = S.Batch([specs[k] for k in balls])
    t0 = time.perf_counter()
    lv, lo, hi, calls = bb.volume(phases=0, samples_per_phase=samples_per_phase, chains=chains, walk_len=4,
                                  groups=8, seed=404, burn_in=200)
    wall = time.perf_counter() - t0
    progress(f"uneven batch: volume done in {wall:.1f} s")
    # "within": the closed form inside the estimator's own interval; "within_doubled":
    # inside that interval widened to twice its half-width about its centre
    per_ball, inside, inside2 = [], 0, 0
    for j, k in enumerate(balls):
        nb = insts[k].n
        truth = 0.5 * nb * math.log(math.pi) - math.lgamma(0.5 * nb + 1)
        w = hi[j] - lo[j]
        ok = bool(lo[j] <= truth <= hi[j])
        ok2 = bool(lo[j] - 0.5 * w <= truth <= hi[j] + 0.5 * w)
        inside += int(ok)
        inside2 += int(ok2)
        per_ball.append({"n": nb, "log_vol": float(lv[j]), "truth": truth, "err": float(lv[j] - truth),
                         "ci_half": float(0.5 * w), "within": ok, "within_doubled": ok2})
    out["volume_balls"] = {"instances": len(balls), "phases": "cooling rule a_(i+1) = a_i (1 - 1/sqrt(n))",
                           "samples_per_phase": samples_per_phase, "walk_len": 4, "burn_in": 200,
                           "seconds": wall, "oracle_calls": calls, "oracle_calls_per_s": calls / wall,
                           "within_ci": f"{inside}/{len(balls)}",
                           "within_doubled_ci": f"{inside2}/{len(balls)}", "balls": per_ball}
    bb.close()
    return out


def hmc_precision_leg(g, S, tau, chains, rounds):
    """HMC with reflections for the Gaussian exp(-|x|^2 / 2) (sigma = 1) on the
    n = m = 200 instance, travel time tau eta with tau = the diameter
    estimate, in each precision of the pencil assembly (FP64; FP32 and BF16
    hi+lo with escalation to FP64 pencils when the reduced-precision F(p) has
    min pivot / max pivot < 1e-3): segment (curve-oracle call) and step rates
    of the same chain state, escalation rates, and on logged segments of the
    FP64 walk the first-root error of each mode against FP64, bucketed by
    kappa(F(p)) (numpy eigenvalues on a sample), with hit / no-hit
    disagreements inside and outside the escalated segments."""
    import torch
    n = N_DIM
    sigma, a = 1.0, 0.5
    x0 = torch.zeros((chains, n), dtype=torch.float64, device="cuda")
    g.walk(S.HMC, x0, 1 << 40, seed=77, gauss_a=a, tau=tau, max_rounds=8)
    g.save_walk_state()
    out = {"chains": chains, "sigma": sigma, "tau": tau, "rounds": rounds, "escalate_ratio": 1e-3}
    log = None
    modes = (("fp64", S.PREC_FP64), ("fp32", S.PREC_FP32_ASM), ("bf16x2", S.PREC_BF16X2_ASM))
    for name, mode in modes:
        g.restore_walk_state()
        g.set_precision(mode)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kw = dict(log_chains=chains, log_cap=chains * rounds) if mode == S.PREC_FP64 else {}
        _, _, st, lg = g.walk(S.HMC, x0, 1 << 40, seed=77, gauss_a=a, tau=tau, max_rounds=rounds, resume=True,
                              **kw)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if lg is not None:
            log = lg
        out[name] = {"seconds": wall, "curve_calls_per_s": st["calls"] / wall, "steps_per_s": st["steps"] / wall,
                     "reflections_per_call": st["reflections"] / max(st["calls"], 1),
                     "escalated_rate": st["escalated"] / max(st["calls"], 1),
                     "not_interior": st["not_interior"], "noconv": st["noconv"]}
    g.set_precision(S.PREC_FP64)
    # first roots of logged segments' pencils in each mode
    L = log[: min(log.shape[0], 4096)]
    p, v = L[:, :n], L[:, n:2 * n]
    coef = torch.zeros((L.shape[0], 3, n + 1), dtype=torch.float64, device="cuda")
    coef[:, 0, 0], coef[:, 0, 1:] = 1.0, p
    coef[:, 1, 1:] = 2 * sigma * v
    coef[:, 2, 0], coef[:, 2, 1:] = 1.0, -p
    roots = {}
    for name, mode in modes:
        g.set_precision(mode)
        _, tp, stc = g.intersect_curve(coef, 1.0)
        roots[name] = (tp.cpu().numpy(), stc.cpu().numpy(), (g.call_flags(coef.shape[0]) & 128) > 0)
    g.set_precision(S.PREC_FP64)
    # kappa(F(p)) on a sample of the segments (dense block and box rows)
    pn = p.cpu().numpy()
    A = g.inst.blocks[0].A
    D = g.inst.blocks[1].A if len(g.inst.blocks) > 1 else None
    samp = np.linspace(0, len(pn) - 1, min(384, len(pn))).astype(int)
    kap = np.empty(len(samp))
    for j, k in enumerate(samp):
        ev = np.linalg.eigvalsh(A[0] + np.tensordot(pn[k], A[1:], 1))
        lo, hi = ev.min(), ev.max()
        if D is not None:
            dv = D[0] + pn[k] @ D[1:]
            lo, hi = min(lo, dv.min()), max(hi, dv.max())
        kap[j] = hi / lo
    edges = [1.0, 1e2, 1e4, 1e6, np.inf]
    ref, rst, _ = roots["fp64"]
    for name in ("fp32", "bf16x2"):
        tp, stc, esc = roots[name]
        ok = (rst == 0) & (stc == 0)
        both = ok & np.isfinite(ref) & np.isfinite(tp)
        rel = np.where(both, np.abs(tp - ref) / np.where(both, ref, 1.0), np.nan)
        dis = ok & (np.isfinite(ref) != np.isfinite(tp))
        buckets = []
        for lo, hi in zip(edges[:-1], edges[1:]):
            sel = samp[(kap >= lo) & (kap < hi)]
            r = rel[sel]
            r = r[np.isfinite(r)]
            buckets.append({"kappa": [lo, hi], "segments": int(len(sel)), "escalated": int(esc[sel].sum()),
                            "median": float(np.median(r)) if len(r) else None,
                            "max": float(r.max()) if len(r) else None,
                            "hit_disagreements": int(dis[sel].sum())})
        r_all = rel[np.isfinite(rel)]
        out[f"{name}_vs_fp64_root_rel"] = {
            "segments": int(ok.sum()), "escalated": int(esc.sum()),
            "median": float(np.median(r_all)), "p99": float(np.quantile(r_all, 0.99)), "max": float(r_all.max()),
            "max_not_escalated": float(np.nanmax(np.where(esc, np.nan, rel))) if np.any(both & ~esc) else None,
            "hit_disagreements": int(dis.sum()),
            "hit_disagreements_not_escalated": int((dis & ~esc).sum()),
            "by_kappa_sample": buckets}
    return out


def paper_workload_leg(S, I, chains, rounds, warmup):
    """Billiard walk on the paper's own random spectrahedra (Section 4: A0 =
    Z Z^T + I, A_i = blkdiag(Qt, -Qt), no box block) at n = m = 100 and 200, the
    sizes of its walk-length table.  Calls per completed step come from a
    two-step walk of every chain; the rate from timed rounds as on the main
    leg.  The paper's own average time per point (one sequential CPU walk) is
    quoted beside it as context."""
    import torch
    out = {}
    paper_ms = {100: 0.3, 200: 7.2}
    for n in (100, 200):
        inst = I.paper_random(n, n, seed=1000 + n)
        g = S.Spectrahedron(inst)
        pre = 64
        _, _, _, log = g.walk(S.HNR, np.zeros((pre, n)), 20, seed=11, log_chains=pre, log_cap=pre * 20)
        lg = log.cpu().numpy()
        tau = 2.0 * float(np.max(lg[:, 2 * n + 1] - lg[:, 2 * n]))
        x0 = torch.zeros((chains, n), dtype=torch.float64, device="cuda")
        _, _, st2, _ = g.walk(S.BILLIARD, x0, 2, seed=77, tau=tau)
        cps = st2["calls"] / max(st2["steps"], 1)
        g.walk(S.BILLIARD, x0, 1 << 40, seed=2024, tau=tau, max_rounds=max(warmup, 1))
        run = timed_rounds(g, S, x0, tau, rounds, chains)
        calls_s = run["stats"]["calls"] / run["wall"]
        out[f"S-{n}-{n}"] = {
            "chains": chains, "tau": tau, "instance_seed": 1000 + n,
            "oracle_calls_per_s": calls_s, "calls_per_step": cps,
            "billiard_steps_per_s": calls_s / cps,
            "lanczos_steps_per_call": run["lz_steps"] / max(run["stats"]["calls"], 1),
            "paper_ms_per_point": paper_ms[n],
            "paper_hardware": "Intel Core i7-6700 @3.4 GHz, one sequential walk (context, not the target)",
        }
        del g, x0
    return out


def _tau_of(g, S, n):
    """2 x the longest chord of a 64-chain, 20-step Hit-and-Run pre-run."""
    _, _, _, log = g.walk(S.HNR, np.zeros((64, n)), 20, seed=11, log_chains=64, log_cap=64 * 20)
    lg = log.cpu().numpy()
    return 2.0 * float(np.max(lg[:, 2 * n + 1] - lg[:, 2 * n]))


TABLE3_W = (1, 5, 10, 20, 30, 40, 50)
TABLE3_PAPER_S = {100: (1.4, 3.2, 7.7, 9.5, 16.1, 21.4, 28.2), 200: (16.2, 75.7, 148.0, 303.0, 443.0, 584.0, 722.0)}


def walk_length_leg(S, I, instances, points, sizes=(100, 200)):
    """The walk-length table of the paper's expectation experiments (Section 4,
    sampling for expectations): seconds to draw `points` points with the
    billiard walk at walk lengths 1..50 on S-n-n spectrahedra of the paper's
    generator, averaged over `instances` seeds.  One point per chain: `points`
    chains walk W steps from the centre, all in one batch (the paper's run is
    one sequential chain that keeps every W-th point).  Wall time of each walk
    call, device synchronised on both sides; the paper's seconds (one CPU core)
    beside them as context."""
    import torch
    out = {}
    for n in sizes:
        secs = {W: [] for W in TABLE3_W}
        calls = {W: [] for W in TABLE3_W}
        rounds = {W: [] for W in TABLE3_W}
        for k in range(instances):
            seed = 10000 + 100 * n + k
            g = S.Spectrahedron(I.paper_random(n, n, seed=seed))
            tau = _tau_of(g, S, n)
            x0 = torch.zeros((points, n), dtype=torch.float64, device="cuda")
            g.walk(S.BILLIARD, x0, 1, seed=1, tau=tau)  # workspaces
            for W in TABLE3_W:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, _, st, _ = g.walk(S.BILLIARD, x0, W, seed=5000 + 7 * k + W, tau=tau)
                torch.cuda.synchronize()
                secs[W].append(time.perf_counter() - t0)
                calls[W].append(st["calls"])
                rounds[W].append(st["rounds"])
                assert st["steps"] == points * W and st["not_interior"] == 0
            del g, x0
            progress(f"walk-length table: S-{n}-{n} instance {k + 1}/{instances}")
        out[f"S-{n}-{n}"] = {
            "instances": instances, "points": points, "walk_lengths": list(TABLE3_W),
            "seconds_mean": [float(np.mean(secs[W])) for W in TABLE3_W],
            "seconds_sd": [float(np.std(secs[W])) for W in TABLE3_W],
            "oracle_calls_mean": [float(np.mean(calls[W])) for W in TABLE3_W],
            "rounds_mean": [float(np.mean(rounds[W])) for W in TABLE3_W],
            "oracle_calls_per_s": [float(np.sum(calls[W]) / np.sum(secs[W])) for W in TABLE3_W],
            "paper_seconds": list(TABLE3_PAPER_S[n]),
            "paper_hardware": "Intel Core i7-6700 @3.4 GHz, one sequential walk, average of 10 instances "
                              "(context, not the target)",
        }
    return out


def estimator_leg(S, I, n, trials, points, lengths=TABLE3_W):
    """Expectation estimators of the paper's uniform-sampling experiment
    (Section 4, eq. estimator_error): I = E_pi[f] for f = 1(S cap H), H = {c x <=
    b1 or c x >= b2}, estimated by the mean of f over N = `points` points, M =
    `trials` times, for Hit-and-Run, coordinate Hit-and-Run and the billiard
    walk at each walk length W.  Each trial is one chain from the centre that
    keeps every W-th point (the paper's form); all trials of a walk run as one
    batch.  S is S-n-n of the paper's generator (seed 20050), c a seeded unit
    vector; b1 < b2 are chosen on a long reference run so that the two
    functions have means near the paper's 0.0993 and 0.588, and a second,
    independent reference run gives the values reported as the truth."""
    import torch
    g = S.Spectrahedron(I.paper_random(n, n, seed=20050))
    tau = _tau_of(g, S, n)
    c = np.random.default_rng(20051).standard_normal(n)
    c /= np.linalg.norm(c)

    def proj(samples):
        return samples.cpu().numpy() @ c

    ref_chains = 8192
    x0 = torch.zeros((ref_chains, n), dtype=torch.float64, device="cuda")
    xa, _, _, _ = g.walk(S.BILLIARD, x0, 100, seed=31, tau=tau)
    xb, _, _, _ = g.walk(S.BILLIARD, x0, 100, seed=32, tau=tau)
    ya, yb = proj(xa), proj(xb)
    funcs = {}
    for name, tail in (("f1", 0.0993), ("f2", 0.588)):
        b1, b2 = np.quantile(ya, [tail / 2, 1 - tail / 2])
        fb = ((yb <= b1) | (yb >= b2)).astype(float)
        funcs[name] = {"b1": float(b1), "b2": float(b2), "truth": float(fb.mean()),
                       "truth_se": float(fb.std() / np.sqrt(len(fb)))}
    out = {"n": n, "m": n, "instance_seed": 20050, "trials": trials, "points": points, "walk_lengths": list(lengths),
           "functions": funcs, "reference": f"{ref_chains} billiard chains x 100 steps from the centre, twice"}
    xs = torch.zeros((trials, n), dtype=torch.float64, device="cuda")
    for kind, name in ((S.HNR, "hit_and_run"), (S.CHNR, "coordinate_hit_and_run"), (S.BILLIARD, "billiard")):
        res = {f: {"mean": [], "sd": []} for f in funcs}
        secs = []
        for W in lengths:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, smp, st, _ = g.walk(kind, xs, points * W, seed=900 + W, tau=tau, thin=W)
            torch.cuda.synchronize()
            secs.append(time.perf_counter() - t0)
            y = proj(smp)  # trials x points
            for f, d in funcs.items():
                est = ((y <= d["b1"]) | (y >= d["b2"])).mean(axis=1)
                res[f]["mean"].append(float(est.mean()))
                res[f]["sd"].append(float(est.std(ddof=1)))
        res["seconds"] = secs
        out[name] = res
        progress(f"estimators: {name} done")
    return out


def config2_leg(S, I, chains=4096, steps=10000, chunk=500, log_per_chunk=128, start=None, save=None, seed=2020):
    """Plain batched billiard at the paper's scale: G-BASE n = m = 100 (plus
    the 200-row box block), FP64, `chains` chains of `steps` steps each with
    tau = 2 x the diameter estimate, walked in chunks of `chunk` steps (the
    chains resume where they stopped).  In every chunk the first segments of
    64 chains are logged; afterwards the oracle recomputes >= 1000 of the
    logged (x, v) by bisection on membership in parallel host threads, and
    every far root must agree to 1e-9 (the near root of a start next to the
    boundary to 1e-9 plus the rounding bound of its assembly and factor)."""
    import torch
    n = 100
    inst = I.gbase(n, n, seed=102)
    g = S.Spectrahedron(inst)
    _, _, _, log = g.walk(S.HNR, np.zeros((64, n)), 20, seed=11, log_chains=64, log_cap=64 * 20)
    lg = log.cpu().numpy()
    tau = 2.0 * float(np.max(lg[:, 2 * n + 1] - lg[:, 2 * n]))
    # start: chain positions saved by an earlier run (a step boundary, where the
    # walk is Markov: the continuation draws new directions and lengths)
    x0 = torch.zeros((chains, n), dtype=torch.float64, device="cuda")
    if start:
        x0 = torch.from_numpy(np.load(start)).to(device="cuda", dtype=torch.float64)
        assert tuple(x0.shape) == (chains, n)
    logs, tot = [], {"calls": 0.0, "steps": 0.0, "reflections": 0.0, "not_interior": 0.0, "noconv": 0.0}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        done = min(steps, done + chunk)
        xo, _, st, lgc = g.walk(S.BILLIARD, x0, done, seed=seed, tau=tau, resume=done > chunk,
                                log_chains=64, log_cap=log_per_chunk)
        logs.append(lgc.cpu().numpy())
        for k in tot:
            tot[k] += st[k]
        wall = time.perf_counter() - t0
        progress(f"config 2: {done}/{steps} steps per chain, {tot['steps'] / wall:.0f} billiard steps/s")
    wall = time.perf_counter() - t0
    if save:
        np.save(save, xo.cpu().numpy())
    pairs = np.concatenate(logs)
    x, v, tpw = pairs[:, :n], pairs[:, n:2 * n], pairs[:, 2 * n + 1]
    out = {"n": n, "m": n, "box_rows": 2 * n, "chains": chains, "steps_per_chain": steps, "tau": tau,
           "instance_seed": 102, "seconds": wall, "billiard_steps_per_s": tot["steps"] / wall,
           "oracle_calls_per_s": tot["calls"] / wall, "calls_per_step": tot["calls"] / max(tot["steps"], 1),
           "not_interior": tot["not_interior"], "noconv": tot["noconv"], "logged_pairs": len(pairs)}
    return out, (x, v, tpw)


def cpu_baseline_config2(x, v, tpw, workers=16):
    """The CPU oracle on the logged pairs of the paper-scale walk: its
    bisection on membership over `workers` host threads (oracle calls/s on
    the host cores), and the walk's own t+ against it (every far root to
    1e-9)."""
    import concurrent.futures as cf
    from oracle import oracle as O
    from paper_2010_03817_amd import instances as I
    o = O.Oracle(I.gbase(100, 100, seed=102))
    workers = min(workers, os.cpu_count() or 1)
    tm_r, tp_r = np.empty(len(x)), np.empty(len(x))
    parts = [q for q in np.array_split(np.arange(len(x)), workers) if len(q)]

    def job(ix):
        a, b, _ = o.line_bisect(x[ix], v[ix])
        tm_r[ix], tp_r[ix] = a, b

    t1 = time.perf_counter()
    with cf.ThreadPoolExecutor(len(parts)) as ex:
        list(ex.map(job, parts))
    wall = time.perf_counter() - t1
    rel = np.abs(tpw - tp_r) / tp_r
    return {"kind": "oracle", "pairs": len(x), "threads": len(parts), "seconds": wall,
            "oracle_calls_per_s": len(x) / wall, "method": "bisection on Cholesky membership",
            "tplus_rel_max": float(rel.max()), "tplus_rel_median": float(np.median(rel)),
            "within_1e-9": int((rel <= 1e-9).sum())}


TABLE2_PAPER = {  # volume (mean +- t s / sqrt(10)), points, seconds; one CPU core (context, not the target)
    40: ("(1.34 +- 0.12)e-06", 9975.2, 6.7), 60: ("(1.23 +- 0.11)e-20", 20370.9, 28.5),
    80: ("(4.24 +- 0.26)e-33", 31539.1, 124.4), 100: ("(1.21 +- 0.10)e-51", 52962.7, 362.3),
}


def volume_balls_leg(S, I, sizes=(40, 60, 80, 100), chains=2048, samples_per_chain=20):
    """The volume table of the paper (ball sequence, eq. (mmc_vol)): log10 of
    vol(S-n-n) of its generator (one seeded instance per size; the paper's
    instances are not published, so the volumes differ), the 95 % interval
    over 8 groups of chains, the balls, billiard points and wall time."""
    import torch
    out = {}
    for n in sizes:
        g = S.Spectrahedron(I.paper_random(n, n, seed=40000 + n))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        lv, lo, hi, st = g.volume_balls(chains=chains, samples_per_chain=samples_per_chain, seed=41000 + n)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ln10 = math.log(10.0)
        out[f"S-{n}-{n}"] = {
            "instance_seed": 40000 + n, "log10_volume": lv / ln10, "log10_ci": [lo / ln10, hi / ln10],
            "relative_half_width": math.expm1(0.5 * (hi - lo)), "balls": st["phases"], "points": st["points"],
            "oracle_calls": st["oracle_calls"], "seconds": dt,
            "paper": {"volume": TABLE2_PAPER[n][0], "points": TABLE2_PAPER[n][1], "seconds": TABLE2_PAPER[n][2],
                      "note": "its own random instances, one CPU core (context, not the target)"},
        }
        progress(f"ball-sequence volume: S-{n}-{n} done")
        del g
    return out


TABLE4_PAPER = {  # iterations / seconds / failures out of 10, one CPU core (context, not the target)
    30: {"hmc_r": (20.1, 2.9, 0), "hnr_w1": (184.3, 3.4, 1), "hnr_w2": (52.1, 5.2, 0)},
    40: {"hmc_r": (24.6, 7.9, 0), "hnr_w1": (223.3, 9.9, 2), "hnr_w2": (61.9, 17.1, 0)},
    50: {"hmc_r": (29.2, 12.7, 0), "hnr_w1": (251.2, 22.3, 3), "hnr_w2": (72.3, 44.6, 0)},
    60: {"hmc_r": (32.8, 24.32, 0), "hnr_w1": (272.7, 41.1, 3), "hnr_w2": (81.5, 98.9, 0)},
}


def anneal_leg(S, I, per_size, chains, max_iters):
    """The annealing table of the paper's optimisation section: iterations
    (temperatures) until the best <c, x> is within 5 % of the optimum, run
    time and failures, for HMC with reflections (walk length one) and
    Hit-and-Run with walk lengths 4 sqrt(n) and 4 n, on S-n-n of the paper's
    generator (n = 30 .. 60) with seeded unit objectives.  The optima are the
    stored ones of the oracle's barrier method (tests/golden/sdp_optima.json).
    Every chain is one run of the method: T0 = d |c| and tau0 = d with d the
    longest chord of a Hit-and-Run pre-run, cooling 1 - 1/sqrt(n), starts drawn
    by 20 billiard steps from the centre; a chain that is not within 5 % after
    `max_iters` temperatures is a failure.  Wall time of each call (all chains
    of one instance together) with the device synchronised."""
    import torch
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "tests", "golden", "sdp_optima.json")) as fh:
        optima = json.load(fh)["optima"]
    methods = (("hmc_r", S.HMC, lambda n: 1), ("hnr_w1", S.HNR, lambda n: int(round(4 * math.sqrt(n)))),
               ("hnr_w2", S.HNR, lambda n: 4 * n))
    out = {"chains_per_instance": chains, "max_iterations": max_iters, "eps": 0.05}
    for n in sorted({e["n"] for e in optima}):
        rows = [e for e in optima if e["n"] == n][:per_size]
        res = {k: {"iters": [], "seconds": [], "failures": 0, "runs": 0, "calls": 0.0} for k, _, _ in methods}
        for e in rows:
            g = S.Spectrahedron(I.paper_random(n, n, seed=e["instance_seed"]))
            c = I.objective(n, e["objective_seed"])
            _, _, _, log = g.walk(S.HNR, np.zeros((64, n)), 20, seed=11, log_chains=64, log_cap=64 * 20)
            lg = log.cpu().numpy()
            d = float(np.max(lg[:, 2 * n + 1] - lg[:, 2 * n]))
            x0, _, _, _ = g.walk(S.BILLIARD, torch.zeros((chains, n), dtype=torch.float64, device="cuda"), 20,
                                 seed=12, tau=2.0 * d)
            x0 = x0.cpu().numpy()
            for name, kind, wl in methods:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, fb, _, hit, st = g.sdp_anneal(x0, c, d * np.linalg.norm(c), d, iterations=max_iters,
                                                 walk_len=wl(n), kind=kind, seed=13, f_star=e["f_star"],
                                                 stop_when_reached=True)
                torch.cuda.synchronize()
                r = res[name]
                r["seconds"].append(time.perf_counter() - t0)
                ok = hit >= 0
                r["iters"].extend((hit[ok] + 1).tolist())
                r["failures"] += int((~ok).sum())
                r["runs"] += len(hit)
                r["calls"] += st["calls"]
                assert np.all(fb >= e["f_star"] - 1e-9 * abs(e["f_star"]))
            del g
        progress(f"annealing table: S-{n}-{n} done")
        out[f"S-{n}-{n}"] = {
            name: {"walk_len": wl(n), "mean_iterations": float(np.mean(r["iters"])) if r["iters"] else None,
                   "seconds_per_instance": float(np.mean(r["seconds"])),
                   "failure_rate": r["failures"] / max(r["runs"], 1), "instances": len(rows),
                   "oracle_calls_per_s": r["calls"] / max(sum(r["seconds"]), 1e-9),
                   "paper": {"iterations": TABLE4_PAPER[n][name][0], "seconds": TABLE4_PAPER[n][name][1],
                             "failures_of_10": TABLE4_PAPER[n][name][2]} if n in TABLE4_PAPER else None}
            for (name, _, wl), r in ((m, res[m[0]]) for m in methods)}
    return out


def anneal_trace_leg(S, I, chains=16, iterations=70):
    """The objective trace of the paper's annealing figure: on S-50-50 (the
    first instance of the annealing workload) the best <c, x> after each of 70
    temperatures, HMC with reflections at walk length one against Hit-and-Run
    at walk length 500 + 4 n^2 = 10500, as the relative error to the stored
    optimum (median and range over the chains), with wall times."""
    import torch
    here = os.path.dirname(os.path.abspath(__file__))
    with open(os.path.join(here, "tests", "golden", "sdp_optima.json")) as fh:
        e = [r for r in json.load(fh)["optima"] if r["n"] == 50][0]
    n = 50
    g = S.Spectrahedron(I.paper_random(n, n, seed=e["instance_seed"]))
    c = I.objective(n, e["objective_seed"])
    _, _, _, log = g.walk(S.HNR, np.zeros((64, n)), 20, seed=11, log_chains=64, log_cap=64 * 20)
    lg = log.cpu().numpy()
    d = float(np.max(lg[:, 2 * n + 1] - lg[:, 2 * n]))
    x0, _, _, _ = g.walk(S.BILLIARD, torch.zeros((chains, n), dtype=torch.float64, device="cuda"), 20, seed=12,
                         tau=2.0 * d)
    x0 = x0.cpu().numpy()
    out = {"instance_seed": e["instance_seed"], "f_star": e["f_star"], "chains": chains, "iterations": iterations}
    for name, kind, wl in (("hmc_r", S.HMC, 1), ("hit_and_run", S.HNR, 500 + 4 * n * n)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, _, best, hit, st = g.sdp_anneal(x0, c, d * np.linalg.norm(c), d, iterations=iterations, walk_len=wl,
                                           kind=kind, seed=14, f_star=e["f_star"])
        torch.cuda.synchronize()
        rel = (best - e["f_star"]) / abs(e["f_star"])
        out[name] = {"walk_len": wl, "seconds": time.perf_counter() - t0, "oracle_calls": st["calls"],
                     "rel_err_median": [float(v) for v in np.median(rel, 0)],
                     "rel_err_min": [float(v) for v in rel.min(0)], "rel_err_max": [float(v) for v in rel.max(0)],
                     "first_within_5pc": [int(h) + 1 if h >= 0 else None for h in hit]}
        progress(f"annealing trace: {name} done")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--state-rounds", type=int, default=150,
                    help="rounds walked from the centre before the chain state shared by the legs is saved")
    ap.add_argument("--chains", type=int, default=CHAINS)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--train-rows", type=int, default=2_000_000)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--data-chains", type=int, default=65536,
                    help="billiard chains whose segment starts make the training triples")
    ap.add_argument("--no-uneven", action="store_true")
    ap.add_argument("--no-hmc", action="store_true")
    ap.add_argument("--no-paper", action="store_true")
    ap.add_argument("--hmc-chains", type=int, default=8192)
    ap.add_argument("--hmc-rounds", type=int, default=20,
                    help="timed rounds of the HMC leg per precision mode (2000 for the full walk length)")
    ap.add_argument("--uneven-samples", type=int, default=256,
                    help="samples per cooling phase of the 256-spectrahedra volume (2000 for the full run)")
    ap.add_argument("--walk-lengths", action="store_true",
                    help="also run the walk-length table (S-100-100, S-200-200) and the estimator study")
    ap.add_argument("--walk-length-instances", type=int, default=10)
    ap.add_argument("--anneal", action="store_true",
                    help="also run the annealing table (min <c, x> on S-30-30 .. S-60-60)")
    ap.add_argument("--anneal-instances", type=int, default=10)
    ap.add_argument("--anneal-trace", action="store_true",
                    help="also trace the best objective over 70 temperatures on S-50-50 (HMC-r, Hit-and-Run)")
    ap.add_argument("--config2", action="store_true",
                    help="also run the paper-scale plain walk (n = m = 100, 4096 chains x 1e4 billiard steps) and "
                         "check logged pairs with the oracle")
    ap.add_argument("--config2-steps", type=int, default=10000)
    ap.add_argument("--config2-start", default=None, help="continue from chain positions saved by --config2-save")
    ap.add_argument("--config2-save", default=None, help="save the final chain positions (.npy)")
    ap.add_argument("--config2-seed", type=int, default=2020)
    ap.add_argument("--uneven-volume-all", action="store_true",
                    help="also estimate the volume of all 256 uneven spectrahedra (--uneven-samples per phase)")
    ap.add_argument("--volume-balls", action="store_true",
                    help="also run the ball-sequence volume table (S-40-40 .. S-100-100)")
    ap.add_argument("--anneal-chains", type=int, default=64)
    ap.add_argument("--anneal-max-iters", type=int, default=400)
    ap.add_argument("--lanczos-tol", type=float, default=1e-8,
                    help="relative residual at which the Lanczos runs of the oracle stop")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this size first (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: the benchmark runs on one GPU only (asked for {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2010_03817_amd import instances as I
    from paper_2010_03817_amd import spec as S

    inst = I.gbase(N_DIM, M_DIM, seed=SEED_INST)
    g = S.Spectrahedron(inst)
    g.set_lanczos(80, args.lanczos_tol)
    # diameter estimate: longest chord seen by a short Hit-and-Run pre-run
    pre = 64
    _, _, _, log = g.walk(S.HNR, np.zeros((pre, N_DIM)), 20, seed=11, log_chains=pre, log_cap=pre * 20)
    lg = log.cpu().numpy()
    dhat = float(np.max(lg[:, 2 * N_DIM + 1] - lg[:, 2 * N_DIM]))
    tau = 2.0 * dhat

    if args.calib_copy_mib > 0:
        nb = args.calib_copy_mib << 20
        src = torch.ones(nb // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    chains = args.chains
    x0 = torch.zeros((chains, N_DIM), dtype=torch.float64, device="cuda")
    net = ctl = report = None
    if not args.no_learned:
        progress("learned path: training data, training, half-width tuning")
        net, delta, ctl, cdelta, report, net400, delta400 = train_learned(g, S, tau, chains, args.train_rows,
                                                                          args.epochs, args.data_chains,
                                                                          args.state_rounds)
    # one chain state for every leg: fresh chains walked state_rounds rounds and
    # saved; each leg restores it, runs the warm-up rounds and then the timed
    # rounds with the same seed, so the legs see the same walk states
    g.walk(S.BILLIARD, x0, 1 << 40, seed=2024, tau=tau, max_rounds=max(args.state_rounds, 1))
    g.save_walk_state()
    # logged segment starts of 64 chains for the CPU oracle's sample
    _, _, _, clog = g.walk(S.BILLIARD, np.zeros((64, N_DIM)), 1 << 30, seed=31, tau=tau, max_rounds=8,
                           log_chains=64, log_cap=512)
    clog = clog.cpu().numpy()[-256:]
    cpu_px, cpu_pv = clog[:, :N_DIM].copy(), clog[:, N_DIM:2 * N_DIM].copy()

    def leg(name, model, d):
        g.restore_walk_state()
        g.set_mlp(model, d, 1) if model is not None else g.set_mlp(None)
        g.walk(S.BILLIARD, x0, 1 << 40, seed=2024, tau=tau, max_rounds=max(args.warmup, 1), resume=True)
        progress(f"{name}: timed rounds")
        run = timed_rounds(g, S, x0, tau, args.steps, chains)
        g.set_mlp(None)
        return run

    cps = report["calls_per_step"] if report else None
    plain = leg("plain path", None, 0.0)
    roof = roofline(plain, chains, extra_chol=plain["stats"]["refined"])
    if roof["kernel"] == FUSED_STAGE:
        roof["traffic"] = _fused_traffic(chains, "plain")
    # assembly GEMM (F(x) and B(v) rows of every chain): FP64 MFMA utilisation
    P = M_DIM * (M_DIM + 1) // 2
    asm_launches = max(plain["stages"]["assemble"][1], 1)
    asm_ms = plain["stages"]["assemble"][0] / asm_launches
    asm_rows = plain["asm_rows"] / asm_launches
    asm_flops = 2.0 * asm_rows * (N_DIM + 1) * (P + 2 * N_DIM)
    assembly = {"kernel": "k_gemm_f64_128<false>", "achieved": asm_flops / (asm_ms * 1e-3) / 1e12,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "ms_per_launch": asm_ms,
                "rows_per_launch": asm_rows,
                "rows_are": "F(x) and B(v) rows in a full assembly round, B(v) rows alone in a round that "
                            "carries F(x) over (every round but one in 16)"}
    assembly["frac"] = assembly["achieved"] / assembly["peak"]
    plain_sum = summary(plain, chains, cps)
    plain_sum["roofline"] = roof

    learned_sum = control_sum = None
    if net is not None:
        learned = leg(f"learned path (delta {delta:.3f})", net, delta)
        learned_sum = summary(learned, chains, cps)
        learned_sum["roofline"] = roofline(learned, chains,
                                           extra_chol=learned["stats"]["cert_fallback"] + learned["stats"]["refined"])
        if learned_sum["roofline"]["kernel"] == FUSED_STAGE:
            learned_sum["roofline"]["traffic"] = _fused_traffic(chains, "learned")
        learned_sum["training"] = report
        control = leg(f"constant-shift control (delta {cdelta:.3f})", ctl, cdelta)
        control_sum = summary(control, chains, cps)
        learned400 = leg(f"learned path, network on [x, v] only (delta {delta400:.3f})", net400, delta400)
        learned400_sum = summary(learned400, chains, cps)

    head = learned_sum if learned_sum is not None else plain_sum
    out = {
        "metric": "oracle calls/s + billiard steps/s at n=m=200, learned vs plain @1e-9 rel",
        "value": head["oracle_calls_per_s"],
        "unit": "oracle calls/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_round"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "billiard walk, n=m=200 G-BASE spectrahedron (+400 box rows), FP64 oracle",
                   "chains": chains, "n": N_DIM, "m": M_DIM, "tau": tau, "instance_seed": SEED_INST,
                   "lanczos_tol": args.lanczos_tol,
                   "path": "learned" if learned_sum is not None else "plain"},
        "billiard_steps_per_s": head["billiard_steps_per_s"],
        "roofline": head["roofline"],
        "assembly_gemm": assembly,
        "plain": plain_sum,
    }
    if learned_sum is not None:
        out["learned"] = learned_sum
        out["control"] = control_sum
        out["learned_over_plain"] = learned_sum["oracle_calls_per_s"] / plain_sum["oracle_calls_per_s"]
        out["learned_over_control"] = learned_sum["oracle_calls_per_s"] / control_sum["oracle_calls_per_s"]
        out["learned_400_inputs"] = learned400_sum
        out["learned_over_learned_400_inputs"] = (learned_sum["oracle_calls_per_s"]
                                                  / learned400_sum["oracle_calls_per_s"])
        out["comparison"] = ("plain, learned and control legs continue the same saved chain state with the same "
                             "seed (warm-up rounds, then the timed rounds)")
    if not args.no_hmc:
        progress("HMC with reflections, precision split")
        out["hmc_precision"] = hmc_precision_leg(g, S, dhat, args.hmc_chains, args.hmc_rounds)
    if not args.no_uneven:
        progress("uneven batch: 256 spectrahedra, autotune, batched volume")
        out["uneven_batch"] = uneven_leg(S, I, args.uneven_samples)
    if not args.no_paper:
        progress("paper workload: billiard on S-100-100 and S-200-200")
        out["paper_workload"] = paper_workload_leg(S, I, chains, args.steps, args.warmup)
    if args.walk_lengths:
        progress("walk-length table and expectation estimators")
        out["walk_length_table"] = walk_length_leg(S, I, args.walk_length_instances, 200)
        out["expectation_estimators"] = estimator_leg(S, I, 50, 20, 200)
    if args.config2:
        progress("config 2: paper-scale billiard walk")
        out["config2"], c2pairs = config2_leg(S, I, steps=args.config2_steps, start=args.config2_start,
                                              save=args.config2_save, seed=args.config2_seed)
        if not args.no_cpu:
            progress("config 2: CPU oracle on the logged pairs")
            out["config2"]["cpu_baseline"] = cpu_baseline_config2(*c2pairs)
    if args.uneven_volume_all:
        progress("uneven volume of all 256 instances")
        out["uneven_volume_all"] = uneven_volume_all(S, I, args.uneven_samples)
    if args.volume_balls:
        progress("ball-sequence volume table")
        out["volume_balls_table"] = volume_balls_leg(S, I)
    if args.anneal:
        progress("annealing table")
        out["anneal_table"] = anneal_leg(S, I, args.anneal_instances, args.anneal_chains, args.anneal_max_iters)
    if args.anneal_trace:
        progress("annealing trace (HMC-r against Hit-and-Run of walk length 500 + 4 n^2)")
        out["anneal_trace"] = anneal_trace_leg(S, I)
    if not args.no_cpu:
        progress("CPU oracle baseline")
        xs = np.zeros((4, N_DIM))
        out["cpu_baseline"] = cpu_baseline(tau, xs, cpu_px, cpu_pv)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
