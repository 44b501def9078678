"""Benchmark of the boundary-oracle hot path on one MI355X.

Workload: billiard walk (Alg. Billiard) on the n = m = 200 spectrahedron
(dense block A0 = I, A_i = (G_i + G_i^T)/(2 sqrt(m)), plus the |x_i| <= 10
box as 400 diagonal rows), 16384 chains, step length ell = -tau ln(eta) with
tau = 2 x (diameter estimate), FP64.  One bench "step" is one round of the
walk: every chain runs one segment through the whole oracle (assembly GEMM of
F(x) and B(v), Cholesky + inverse, Lanczos extreme eigenvalues, normal GEMM,
reflection / step logic).  Metric: oracle calls per second (one call per chain
per round) with billiard steps per second beside it.

Prints ONE JSON line.  --gpus N with N > 1 exits: this build runs on one GPU.
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


def _fused_traffic(chains):
    """HBM bytes per launch of the fused kernel, from the committed counter
    summary, while the kernel sources are those that were profiled."""
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
    m = re.search(r"^traffic: (\d+) bytes/launch at (\d+) chains, sources ([0-9a-f]+)", txt, re.M)
    if not m or m.group(3) != digest or int(m.group(2)) != chains:
        return None
    return float(m.group(1))


def _cpu_worker(args):
    """Oracle billiard steps for one chain (CPU baseline)."""
    from oracle import oracle as O
    from paper_2010_03817_amd import instances as I
    chain, steps, tau, seed, x0 = args
    o = O.Oracle(I.gbase(N_DIM, M_DIM, seed=SEED_INST))
    t0 = time.time()
    _, _, st = o.walk(O.BILLIARD, x0[None, :], steps, seed=seed + chain, tau=tau)
    return time.time() - t0, st[0], st[5]


def cpu_baseline(tau, x0s, budget_s=15.0):
    cores = min(16, os.cpu_count() or 1)
    # one oracle call at n = m = 200 takes ~0.1-0.3 s: size the sample to the budget
    steps = 2
    jobs = [(c, steps, tau, 9000, x0s[c % len(x0s)]) for c in range(cores)]
    t0 = time.time()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_cpu_worker, jobs)
    wall = time.time() - t0
    calls = sum(r[1] for r in res)
    steps_done = sum(r[2] for r in res)
    busy = max(r[0] for r in res)
    return {
        "value": calls / busy,
        "unit": "oracle calls/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{cores} chains x {steps} billiard steps of the FP64 CPU oracle (cyclic Jacobi), "
                  f"one chain per process; {int(calls)} oracle calls, wall {wall:.1f} s",
        "billiard_steps_per_s": steps_done / busy,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--chains", type=int, default=CHAINS)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device copy of this size first (reference kernel for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2010_03817_amd import instances as I
    from paper_2010_03817_amd import spec as S

    inst = I.gbase(N_DIM, M_DIM, seed=SEED_INST)
    g = S.Spectrahedron(inst)
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
    big = 1 << 40
    # warm-up rounds (also initialises the chains)
    g.walk(S.BILLIARD, x0, big, seed=2024, tau=tau, max_rounds=max(args.warmup, 1))
    torch.cuda.synchronize()
    g.timing(True)
    t0 = time.perf_counter()
    _, _, st, _ = g.walk(S.BILLIARD, x0, big, seed=2024, tau=tau, max_rounds=args.steps, resume=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    g.timing(False)
    stages, lz_steps = g.stage_times()
    calls = st["calls"]
    steps_done = st["steps"]
    value = calls / wall

    # roofline of the dominant kernel
    dom = max(stages, key=lambda k: stages[k][0])
    launches = max(stages[dom][1], 1)
    ms_dom = stages[dom][0] / launches
    P = M_DIM * (M_DIM + 1) // 2
    if dom == "fused":
        # fused per-chain kernel (Cholesky, inverse, Lanczos, Ritz vector): FP64
        # arithmetic on MFMA and the vector ALUs, both at the FP64 peak.  Counted
        # work is the method's own: Cholesky m^3/3, 4 m^2 per Lanczos step,
        # Ritz vector and u = L^-T z, the packed u u^T for the normal GEMM, and
        # the ratio test of the diagonal block; the triangular inverse (m^3/3)
        # is a design choice and is not counted.
        md = 2 * N_DIM
        per_call = M_DIM**3 / 3.0 + 2.0 * M_DIM**2 + P + 3.0 * md
        flops = (calls * per_call + lz_steps * (4.0 * M_DIM**2 + 2.0 * M_DIM)) / launches
        roof = {"bound": "alu", "achieved": flops / (ms_dom * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s"}
    else:
        rows = 2 * calls / launches if dom == "assemble" else calls / launches
        K = N_DIM + 1 if dom == "assemble" else P
        Nc = P + 2 * N_DIM if dom == "assemble" else N_DIM
        flops = 2.0 * rows * K * Nc
        roof = {"bound": "mfma", "achieved": flops / (ms_dom * 1e-3) / 1e12, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = _fused_traffic(chains) if dom == "fused" else None
    roof["traffic_unit"] = "bytes per launch"
    roof["kernel"] = {"fused": "k_line_fused", "assemble": "k_gemm_f64<false>", "normal": "k_gemm_f64<true>",
                      "predict": "k_gemm_f32", "update": "k_walk_update"}[dom]
    roof["ms_per_launch"] = ms_dom
    # assembly GEMM (F(x) and B(v) rows of every chain): FP64 MFMA utilisation
    asm_launches = max(stages["assemble"][1], 1)
    asm_ms = stages["assemble"][0] / asm_launches
    asm_flops = 2.0 * (2 * calls / asm_launches) * (N_DIM + 1) * (P + 2 * N_DIM)
    assembly = {"kernel": "k_gemm_f64<false>", "achieved": asm_flops / (asm_ms * 1e-3) / 1e12,
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "ms_per_launch": asm_ms}
    assembly["frac"] = assembly["achieved"] / assembly["peak"]

    out = {
        "metric": "oracle calls/s + billiard steps/s at n=m=200, learned vs plain @1e-9 rel",
        "value": value,
        "unit": "oracle calls/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "billiard walk, n=m=200 G-BASE spectrahedron (+400 box rows), plain FP64 oracle",
                   "chains": chains, "n": N_DIM, "m": M_DIM, "tau": tau, "instance_seed": SEED_INST,
                   "path": "plain"},
        "billiard_steps_per_s": steps_done / wall,
        "reflections_per_step": st["reflections"] / max(steps_done, 1),
        "lanczos_steps_per_call": lz_steps / max(calls, 1),
        "stage_ms_per_round": {k: v[0] / max(v[1], 1) for k, v in stages.items()},
        "roofline": roof,
        "assembly_gemm": assembly,
    }
    if not args.no_cpu:
        xs = np.zeros((4, N_DIM))
        out["cpu_baseline"] = cpu_baseline(tau, xs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
