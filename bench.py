#!/usr/bin/env python3
"""Throughput of the LAPS hot path on one MI355X.

One benchmark step is one full LAPS run (Algorithm "LAPS Pseudocode") on the
Bayesian logistic-regression workload with synthetic data (X 5000 x 100 N(0,1)
rounded to bf16, weights N(0, 1/d), Bernoulli labels, N(0, I) prior), 4096
chains cold-started from the prior: initialisation, 1000 unadjusted steps
(leapfrog, 1 gradient each), the switch, and 67 MAMS transitions (15 MN2 steps,
2 gradients each).  Every phase runs in the library's HIP kernels; the
positions live in HBM before the timed region starts.

value = chain-gradient evaluations per second over the timed runs.
roofline: the gradient kernel (two fused contractions on bf16 matrix cores)
timed with HIP events on the library stream; algorithmic work 4 n d flops per
chain-gradient.  cpu_baseline: the FP64 CPU oracle on a bounded sample of the
same workload (its first 256 chains, 10 unadjusted steps and one transition).
f64_gpu: the same run with the plain FP64 gradient path.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "chain-grad evals/s & time to bias b²<0.01, mixed/batched vs plain FP64 GPU"
PEAK_BF16_TFLOPS = 2500.0
PEAK_HBM_GBS = 8000.0
# HBM bytes per launch of k_lr_grad_bf16<4> on the logistic-regression workload, from FETCH_SIZE and
# WRITE_SIZE counters scaled by what they read for a plain copy of known size (x2.0 and x1.0); kept
# with the counter summary under profiles/ and reset to None whenever the kernel changes.
LR_GRAD_TRAFFIC_BYTES = 29.32e6


def _run_once(s, x0, n_unadj, n_adj):
    s.reinit(x0)
    s.step_unadjusted(n_unadj)
    s.step_adjusted(n_adj)


WORKLOADS = {
    # name: (generator, default precision, gradient evaluations per step of the dominant kernel)
    "logreg": ("logreg", "bf16"),
    "gauss": ("gaussian", "f64"),
    "stochvol": ("stochvol", "f32"),
    "phi4": ("phi4", "f32"),
}


def gpu_throughput(w, prec, steps, warmup, n_unadj=1000, n_adj=67):
    import torch
    from paper_2601_16696_amd import laps
    cfg = dict(switch_policy=1, max_steps_unadj=n_unadj, max_steps_total=n_unadj + 15 * n_adj)
    s = laps.Sampler(w, prec, **cfg)
    x0 = torch.as_tensor(w["x0"], device="cuda:0").to(s.x.dtype)
    for _ in range(warmup):
        _run_once(s, x0, n_unadj, n_adj)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _run_once(s, x0, n_unadj, n_adj)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st = s.stats()
    grad_ms = s.time_gradient(50)
    ms = (t1 - t0) / steps * 1e3
    grads = st["grads_per_chain"] * w["n_chains"]
    return dict(ms=ms, value=grads / (ms * 1e-3), stats=st, grad_ms=grad_ms, sampler=s)


CPU_SAMPLE = {  # about 10 s of single-threaded oracle work on the same workload
    "logreg": dict(n_chains=256, n_unadj=10, n_adj=1),
    "gauss": dict(n_chains=1024, n_unadj=600, n_adj=4),
    "stochvol": dict(n_chains=512, n_unadj=20, n_adj=1),
    "phi4": dict(n_chains=512, n_unadj=20, n_adj=1),
}


def cpu_baseline(w, n_chains=256, n_unadj=10, n_adj=1):
    from oracle import oracle as orc
    n_chains = min(n_chains, w["n_chains"])
    sub = dict(w)
    sub["x0"] = w["x0"][:n_chains]
    sub["n_chains"] = n_chains
    t0 = time.perf_counter()
    e = orc.Ensemble(orc.Target.from_workload(sub), n_chains, w["seed"], switch_policy=1, max_steps_unadj=n_unadj,
                     max_steps_total=n_unadj + 15 * n_adj)
    e.init(sub["x0"])
    e.step_unadjusted(n_unadj)
    e.step_adjusted(n_adj)
    dt = time.perf_counter() - t0
    grads = e.stats()["grads_per_chain"] * n_chains
    return dict(value=grads / dt, unit="chain-grad evals/s", cores=1, kind="oracle",
                sample=f"first {n_chains} chains, init + {n_unadj} unadjusted steps + {n_adj} MAMS transition "
                       f"({grads} chain-gradients in {dt:.1f} s, single-threaded FP64)")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="logreg", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default=None, choices=["bf16", "f32", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-f64", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2601_16696_amd import laps, workloads
    laps.lib()
    gen, default_prec = WORKLOADS[args.workload]
    prec = args.prec or default_prec
    w = getattr(workloads, gen)()
    N, d = w["n_chains"], w["d"]

    r = gpu_throughput(w, prec, args.steps, args.warmup)
    if args.workload == "logreg":
        n = w["X"].shape[0]
        work = 4.0 * n * d * N  # flops of X theta and X^T r per ensemble gradient
        peak = PEAK_BF16_TFLOPS if prec == "bf16" else 78.6
        achieved = work / (r["grad_ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma" if prec == "bf16" else "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                "frac": achieved / peak, "traffic": LR_GRAD_TRAFFIC_BYTES if prec == "bf16" else None,
                "traffic_unit": "bytes per launch",
                "kernel": "k_lr_grad_bf16<4>" if prec == "bf16" else "k_lr_grad_f64", "kernel_ms": r["grad_ms"],
                "algorithmic_flops_per_launch": work}
        precision = ("bf16 matrix-core gradient, fp32 state, fp64 energy error and reductions"
                     if prec == "bf16" else "fp64 throughout")
        extra = {"n": n}
    else:
        rs = 8 if prec == "f64" else 4
        work = 2.0 * rs * d * N  # the gradient kernel reads x and writes the gradient once per chain
        achieved = work / (r["grad_ms"] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                "frac": achieved / PEAK_HBM_GBS, "traffic": None, "kernel": "k_eval (target gradient)",
                "kernel_ms": r["grad_ms"], "algorithmic_bytes_per_launch": work}
        precision = "fp64 throughout" if prec == "f64" else "fp32 state, fp64 energy error and reductions"
        extra = {}
    line = {
        "metric": METRIC,
        "value": r["value"],
        "unit": "chain-grad evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": prec,
        "data": "synthetic",
        "config": dict({
            "workload": f"{w['name']}: full LAPS run, 1000 unadjusted steps + 67 MAMS transitions",
            "chains": N, "d": d, "precision": precision,
            "grads_per_chain": r["stats"]["grads_per_chain"], "parallelism": "single GPU"}, **extra),
        "roofline": roof,
        "final_state": {"acc_mean": r["stats"]["acc_mean"], "eps": r["stats"]["eps"], "t": r["stats"]["t"],
                        "n_nonfinite": r["stats"]["n_nonfinite"]},
    }
    del r["sampler"]
    torch.cuda.empty_cache()
    if not args.no_f64 and prec != "f64":
        r64 = gpu_throughput(w, "f64", 1, 0)
        line["f64_gpu"] = {"value": r64["value"], "ms_per_step": r64["ms"], "gradient_ms": r64["grad_ms"],
                           "speedup_of_mixed": line["value"] / r64["value"]}
        del r64["sampler"]
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, **CPU_SAMPLE[args.workload])
    print(json.dumps(line))


if __name__ == "__main__":
    main()
